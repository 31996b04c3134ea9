"""Pins of the oracle's error norms (Sec. 6.1.2, eq. error, and the relative
max-norm every parity test uses) on arrays whose norms are known by hand.

The norms gate almost every parity assertion, so a mistake in them (a wrong
sign, a dropped element, a NaN that compares false) would hide mistakes
everywhere else.  Each case below is computed by hand in the comments.
"""
import math

import numpy as np
import pytest

import oracle


def test_norms_hand_computed():
    a = np.array([1.0, -2.0, 3.5, 0.0])
    b = np.array([0.5, 1.0, 4.0, -3.0])
    # a - b = (0.5, -3, -0.5, 3): max |a-b| = 3 (reached by a negative and a
    # positive difference), max |b| = 4, sum (a-b)^2 = 0.25 + 9 + 0.25 + 9,
    # sum b^2 = 0.25 + 1 + 16 + 9.
    out = oracle.norms(a, b)
    assert out.tolist() == [3.0, 4.0, 18.5, 26.25]
    assert oracle.rel_max_err(a, b) == 3.0 / 4.0


def test_norms_negative_difference_is_the_maximum():
    # Only a negative difference is large: max |a - b| = 7, not 0.1.
    a = np.array([0.1, -7.0, 0.0])
    b = np.zeros(3)
    out = oracle.norms(a, b)
    assert out[0] == 7.0
    assert out[1] == 0.0
    # All-zero reference: the relative error falls back to the absolute one.
    assert oracle.rel_max_err(a, b) == 7.0


def test_norms_order_independent_maximum():
    rng = np.random.default_rng(7)
    a = rng.standard_normal(1001)
    b = rng.standard_normal(1001)
    out = oracle.norms(a, b)
    assert out[0] == np.max(np.abs(a - b))
    assert out[1] == np.max(np.abs(b))
    # The sums agree with an exactly rounded sum to a few ulps.
    assert math.isclose(out[2], math.fsum((a - b) ** 2), rel_tol=1e-13)
    assert math.isclose(out[3], math.fsum(b ** 2), rel_tol=1e-13)


@pytest.mark.parametrize("pos", [0, 3, 4])
def test_norms_propagate_nan(pos):
    # A NaN anywhere (first, middle, last element) makes max|a-b| and the sum
    # NaN, however large the finite differences after it are.
    a = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    b = np.array([0.0, 0.0, 100.0, 0.0, 0.0])
    a[pos] = np.nan
    out = oracle.norms(a, b)
    assert math.isnan(out[0]) and math.isnan(out[2])
    assert out[1] == 100.0 and out[3] == 10000.0
    with pytest.raises(ValueError):
        oracle.rel_max_err(a, b)


def test_norms_nan_in_reference():
    a = np.zeros(4)
    b = np.array([1.0, np.nan, 2.0, 3.0])
    out = oracle.norms(a, b)
    assert all(math.isnan(v) for v in out)
    with pytest.raises(ValueError):
        oracle.rel_max_err(a, b)


def test_norms_infinities():
    a = np.array([np.inf, 0.0, 1.0])
    b = np.array([0.0, 0.0, 1.0])
    out = oracle.norms(a, b)
    assert out[0] == np.inf and out[2] == np.inf and out[1] == 1.0
    # inf - inf is NaN: the maximum becomes NaN and stays NaN.
    a2 = np.array([np.inf, 5.0])
    b2 = np.array([np.inf, 0.0])
    out2 = oracle.norms(a2, b2)
    assert math.isnan(out2[0]) and out2[1] == np.inf
    with pytest.raises(ValueError):
        oracle.rel_max_err(a, b)
    with pytest.raises(ValueError):
        oracle.rel_max_err(-a, b)


def test_mostly_nan_result_fails_parity():
    # A 5 x 5 result that is 24/25 NaN (one node written, matching) must not
    # pass a parity check.
    ref = np.arange(25, dtype=np.float64).reshape(5, 5)
    got = np.full((5, 5), np.nan)
    got[2, 2] = ref[2, 2]
    assert math.isnan(oracle.norms(got, ref)[0])
    with pytest.raises(ValueError):
        oracle.rel_max_err(got, ref)

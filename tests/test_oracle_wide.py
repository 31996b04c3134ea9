"""Pins of the oracle for schemes whose stencil reaches three lines out.

The scheme is the general construction of Sec. 4-5 applied to the complete
monomial set of degree 6 (the first 28 monomials in the order of eq. g):
its 28-node stencil gives weight to the centre and to the classes (1,0),
(1,1), (2,0), (2,1) (eight nodes) and (3,0), 25 nodes in all.  The oracle
runs it from node weights computed in exact arithmetic by ``oracle.derive``.

What pins it, none of it re-typing the oracle's class sums:
  * impulse responses node by node against the derivation (every node of
    every class, so a missing mirror image or a wrong offset shows);
  * exactness for polynomial solutions of the wave equation of degree <= 6
    (the interpolation is exact on span M_28 and the operators of Sec. 5 are
    exact on polynomials), which a wrong weight or sign breaks;
  * the symmetries of the square, energy conservation, time reversibility;
  * the odd-reflection rule up to three lines out against a periodic grid of
    twice the size holding the odd extension of the data;
  * periodic wrap-around on a grid of seven nodes per side against the same
    data tiled three times.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import derive

WIDE = 1003  # custom scheme slot used by these tests


@pytest.fixture(scope="module")
def wide(orc):
    w = derive.node_weights(28)
    orc.register_scheme(WIDE, w)
    return w


def _key(q):
    return tuple(sorted((abs(q[0]), abs(q[1])), reverse=True))


def test_degree6_set_has_the_expected_classes(wide):
    """The 28-node stencil of the degree-6 set: weight on the centre and on
    the classes (1,0), (1,1), (2,0), (2,1), (3,0) with all of their nodes;
    the partial classes (2,2) and (3,1) carry none; every node of a class
    has the same weights; A and B reproduce constants."""
    carried = {}
    for q, (A, B) in wide.items():
        has = any(A.values()) or any(B.values())
        carried.setdefault(_key(q), []).append((q, has, A, B))
    got = sorted(k for k, v in carried.items() if any(x[1] for x in v))
    assert got == [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (3, 0)]
    for k in ((1, 0), (1, 1), (2, 0), (2, 1), (3, 0)):
        nodes = carried[k]
        assert sorted(x[0] for x in nodes) == oracle.class_nodes(*k)
        assert all(x[2] == nodes[0][2] and x[3] == nodes[0][3] for x in nodes)
    assert sum(1 for v in carried.values() for x in v if x[1]) == 25
    for part in (0, 1):
        tot = {}
        for q, AB in wide.items():
            for p, c in AB[part].items():
                tot[p] = tot.get(p, Fraction(0)) + c
        assert {p: c for p, c in tot.items() if c} == {0: Fraction(1)}


def _impulse(n):
    e = np.zeros((n, n))
    e[n // 2, n // 2] = 1.0
    return e


@pytest.mark.parametrize("lam", [0.2, 0.45, 0.6])
def test_wide_impulse_responses_equal_derivation(orc, wide, lam):
    """First step of a node impulse, node by node: A phi_q and B phi_q / tau
    of the exact construction, and nothing outside the stencil."""
    n = 13
    h = 0.1
    tau = lam * h
    e = _impulse(n)
    zero = np.zeros_like(e)
    rA = orc.first_step(e, zero, h, tau, 1.0, WIDE)
    rB = orc.first_step(zero, e, h, tau, 1.0, WIDE)
    c = n // 2
    mask = np.zeros_like(e, dtype=bool)
    for (q1, q2), (A, B) in wide.items():
        assert abs(rA[c - q2, c - q1] - derive.evaluate(A, lam)) < 1e-14, ("A", q1, q2)
        assert abs(rB[c - q2, c - q1] / tau - derive.evaluate(B, lam)) < 1e-13, ("B", q1, q2)
        mask[c - q2, c - q1] = True
    assert np.all(rA[~mask] == 0) and np.all(rB[~mask] == 0)
    # The two-step update of an impulse is 2 A e - e_prev.
    up = orc.step(zero, e, h, tau, 1.0, WIDE)
    assert np.max(np.abs(up - 2.0 * rA)) < 1e-14


# Polynomials as {(a1, a2): coefficient} of x^a1 y^a2.
def _lap(P):
    out = {}
    for (a, b), v in P.items():
        if a >= 2:
            out[(a - 2, b)] = out.get((a - 2, b), 0.0) + v * a * (a - 1)
        if b >= 2:
            out[(a, b - 2)] = out.get((a, b - 2), 0.0) + v * b * (b - 1)
    return {k: v for k, v in out.items() if v}


def _eval(P, X, Y):
    return sum(v * X ** a * Y ** b for (a, b), v in P.items())


def _wave_poly(f, g, c, t, X, Y):
    """Exact solution of u_tt = c^2 Lap u with u(0) = f, u_t(0) = g for
    polynomial f, g: sum_k (ct)^2k/(2k)! Lap^k f + t (ct)^2k/(2k+1)! Lap^k g
    (the series ends after degree/2 terms)."""
    u = np.zeros_like(X)
    F, G, k = dict(f), dict(g), 0
    while F or G:
        u = u + (c * t) ** (2 * k) / math.factorial(2 * k) * _eval(F, X, Y) \
              + t * (c * t) ** (2 * k) / math.factorial(2 * k + 1) * _eval(G, X, Y)
        F, G, k = _lap(F), _lap(G), k + 1
    return u


def _rand_poly(rng, deg):
    return {(a, d - a): rng.standard_normal() for d in range(deg + 1) for a in range(d + 1)}


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("lam", [0.3, 0.55])
def test_wide_exact_for_degree6_wave_polynomials(orc, wide, seed, lam):
    """u0, v0 random polynomials of degree 6: every level equals the exact
    solution at t = k tau to rounding, away from the zeroed boundary (three
    lines per level)."""
    rng = np.random.default_rng(seed)
    f, g = _rand_poly(rng, 6), _rand_poly(rng, 6)
    n = 41
    h = 0.05
    tau = lam * h
    x = (np.arange(n) - n // 2) * h
    X, Y = np.meshgrid(x, x)
    u0, v0 = _eval(f, X, Y), _eval(g, X, Y)
    um1, u = u0.copy(), orc.first_step(u0, v0, h, tau, 1.0, WIDE)
    for k in range(1, 6):
        if k > 1:
            um1, u = u, orc.step(um1, u, h, tau, 1.0, WIDE)
        m = 3 * k + 1
        ex = _wave_poly(f, g, 1.0, k * tau, X, Y)
        err = np.max(np.abs(u[m:-m, m:-m] - ex[m:-m, m:-m]))
        assert err <= 1e-12 * max(1.0, np.max(np.abs(ex[m:-m, m:-m]))), (k, err)


def test_wide_not_exact_for_degree8(orc, wide):
    """The same check fails for x^8 (outside span M_28): the exactness above
    is a property of the set, not of the test."""
    n = 41
    h = 0.05
    tau = 0.5 * h
    x = (np.arange(n) - n // 2) * h
    X, Y = np.meshgrid(x, x)
    f = {(8, 0): 1.0}
    u1 = orc.first_step(_eval(f, X, Y), np.zeros((n, n)), h, tau, 1.0, WIDE)
    ex = _wave_poly(f, {}, 1.0, tau, X, Y)
    assert np.max(np.abs(u1[4:-4, 4:-4] - ex[4:-4, 4:-4])) > 1e-12


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n))
    a[0, :] = a[-1, :] = 0
    a[:, 0] = a[:, -1] = 0
    return a


def test_wide_d4_symmetry(orc, wide):
    n = 23
    h = 1.0 / 22
    tau = 0.5 * h
    u0, v0 = _rand(n, 1), _rand(n, 2)
    _, ref = orc.run(u0, v0, h, tau, 1.0, WIDE, 10)
    for f in (lambda a: a.T, lambda a: a[::-1, :], lambda a: a[:, ::-1], lambda a: a[::-1, ::-1].T):
        _, got = orc.run(f(u0), f(v0), h, tau, 1.0, WIDE, 10)
        assert np.max(np.abs(got - f(ref))) < 1e-13 * np.max(np.abs(ref))


def test_wide_energy_conserved_and_reversible(orc, wide):
    """The spatial operator is symmetric under the odd-reflection rule, so
    E = |u^{k+1} - u^k|^2 - <u^{k+1}, L u^k> is conserved; the update run
    backwards returns to the first two levels."""
    n = 25
    h = 1.0 / 24
    tau = 0.5 * h
    zero = np.zeros((n, n))

    def L(u):
        return orc.step(zero, u, h, tau, 1.0, WIDE) - 2 * u

    a, b = _rand(n, 5), _rand(n, 6)
    assert abs(np.sum(a * L(b)) - np.sum(L(a) * b)) < 1e-12 * np.sum(np.abs(a * L(b)))
    u0, v0 = _rand(n, 3), _rand(n, 4)
    um1, u = u0.copy(), orc.first_step(u0, v0, h, tau, 1.0, WIDE)
    E0 = None
    for _ in range(300):
        up1 = orc.step(um1, u, h, tau, 1.0, WIDE)
        E = np.sum((up1 - u) ** 2) - np.sum(up1 * L(u))
        E0 = E if E0 is None else E0
        assert abs(E - E0) < 1e-12 * abs(E0)
        um1, u = u, up1
    u1 = orc.first_step(u0, v0, h, tau, 1.0, WIDE)
    pm, pc = orc.steps(u0, u1, h, tau, 1.0, WIDE, 199)
    bm, bc = orc.steps(pc, pm, h, tau, 1.0, WIDE, 199)
    assert np.max(np.abs(bc - u0)) < 1e-11 * np.max(np.abs(u1))
    assert np.max(np.abs(bm - u1)) < 1e-11 * np.max(np.abs(u1))


@pytest.mark.parametrize("n", [8, 11])
def test_wide_odd_reflection_equals_odd_periodic_extension(orc, wide, n):
    """Dirichlet grid of n + 1 nodes per side against a periodic grid of 2n
    holding the odd extension of the same data: equal on the first grid, so
    every ghost node up to three lines out is the negated mirror node."""
    rng = np.random.default_rng(n)

    def odd_ext(a):  # a: (n+1) x (n+1) with zero boundary -> 2n x 2n periodic
        e = np.zeros((2 * n, 2 * n))
        e[: n + 1, : n + 1] = a
        e[:, n + 1:] = -e[:, n - 1:0:-1]
        e[n + 1:, :] = -e[n - 1:0:-1, :]
        return e

    u0, v0 = _rand(n + 1, int(rng.integers(100))), _rand(n + 1, int(rng.integers(100)))
    h = 1.0 / n
    tau = 0.5 * h
    _, ud = orc.run(u0, v0, h, tau, 1.0, WIDE, 9)
    _, up = orc.run(odd_ext(u0), odd_ext(v0), h, tau, 1.0, WIDE, 9, oracle.PERIODIC)
    assert np.max(np.abs(ud - up[: n + 1, : n + 1])) < 1e-13 * np.max(np.abs(ud))


def test_wide_periodic_wrap_on_seven_nodes(orc, wide):
    """A 7 x 7 periodic grid (the smallest one a radius-3 stencil allows)
    against the same data tiled 3 x 3 on a 21 x 21 periodic grid."""
    rng = np.random.default_rng(7)
    u0, v0 = rng.standard_normal((7, 7)), rng.standard_normal((7, 7))
    h = 1.0 / 7
    tau = 0.4 * h
    _, a = orc.run(u0, v0, h, tau, 1.0, WIDE, 8, oracle.PERIODIC)
    _, b = orc.run(np.tile(u0, (3, 3)), np.tile(v0, (3, 3)), h, tau, 1.0, WIDE, 8, oracle.PERIODIC)
    assert np.max(np.abs(np.tile(a, (3, 3)) - b)) < 1e-13 * np.max(np.abs(a))
    with pytest.raises(ValueError):
        orc.run(u0[:6, :6], v0[:6, :6], h, tau, 1.0, WIDE, 2, oracle.PERIODIC)


def test_register_rejects_asymmetric_and_far_weights(orc):
    w = derive.node_weights(28)
    bad = dict(w)
    A, B = bad[(3, 0)]
    bad[(3, 0)] = ({p: 2 * c for p, c in A.items()}, B)
    with pytest.raises(ValueError):
        orc.register_scheme(WIDE + 1, bad)
    far = {(0, 0): ({0: Fraction(1)}, {0: Fraction(1)}), (4, 0): ({2: Fraction(1)}, {})}
    with pytest.raises(ValueError):
        orc.register_scheme(WIDE + 1, far)

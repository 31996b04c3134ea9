"""Pins of the exact-rational Sec. 4-5 construction (oracle/derive.py) to what
the paper prints, and of the closed-form monomial integrals (eq. exact2) to
the operator definitions eq. Op1 / Op2 by numerical quadrature."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import derive

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "printed_basis.json")))


def _key(q):
    return f"{q[0]},{q[1]}"


def _poly_x(d):
    return {tuple(int(v) for v in k.split(",")): Fraction(c) for k, c in d.items()}


def _poly_l(d):
    return {int(k): Fraction(c) for k, c in d.items()}


def test_mckinney_map_is_a_bijection():
    # eq. alpha / eq. invMcKinney: offsets ... -2,-1,0,1,2 ... <-> exponents 3,1,0,2,4
    assert [derive.alpha(q) for q in (-2, -1, 0, 1, 2, 3)] == [3, 1, 0, 2, 4, 6]
    for q in range(-20, 21):
        assert derive.q_of(derive.alpha(q)) == q
    for a in range(40):
        assert derive.alpha(derive.q_of(a)) == a


def test_g_order_is_onto_and_graded():
    # eq. g: one-to-one onto 1, 2, 3, ... and total degree first.
    seen = {}
    for d in range(12):
        for a1 in range(d + 1):
            seen[derive.g(a1, d - a1)] = (a1, d - a1)
    assert sorted(seen)[:78] == list(range(1, 79))
    degs = [sum(seen[s]) for s in range(1, 79)]
    assert degs == sorted(degs)


@pytest.mark.parametrize("m", [6, 11, 15])
def test_monomial_sets_as_printed(m):
    assert [list(e) for e in derive.monomials(m)] == GOLD["monomials"][str(m)]


@pytest.mark.parametrize("m", [6, 11, 15])
def test_stencil_nodes_and_vanishing_nodes(m):
    st = GOLD["stencils"][str(m)]
    nodes = sorted(tuple(q) for q in st["nodes"])
    assert sorted(derive.stencil(m)) == nodes
    w = derive.node_weights(m)
    vanish = sorted(q for q, (A, B) in w.items() if not A and not B)
    assert vanish == sorted(tuple(q) for q in st["vanish"])


def test_det_D_five_point():
    _, det = derive.lagrange_basis(6)
    assert det == Fraction(GOLD["det_D_6"]["value"])
    # With spacing h every monomial of degree d scales by h^d: det -> det * h^(sum of degrees).
    assert sum(sum(e) for e in derive.monomials(6)) == GOLD["det_D_6"]["h_power"]


@pytest.mark.parametrize("m", [11, 15])
def test_larger_stencils_unisolvent(m):
    _, det = derive.lagrange_basis(m)
    assert det != 0


@pytest.mark.parametrize("m", [6, 11, 15])
def test_lagrange_property(m):
    basis, _ = derive.lagrange_basis(m)
    for q, poly in basis.items():
        for x in derive.stencil(m):
            v = sum(c * Fraction(x[0]) ** e[0] * Fraction(x[1]) ** e[1] for e, c in poly.items())
            assert v == (1 if x == q else 0)


def test_LB6_as_printed():
    basis, _ = derive.lagrange_basis(6)
    for k, d in GOLD["LB6"].items():
        if k.startswith("_"):
            continue
        q = tuple(int(v) for v in k.split(","))
        assert basis[q] == _poly_x(d), k


def test_LB11_even_parts_as_printed():
    basis, _ = derive.lagrange_basis(11)
    for k, d in GOLD["LB11_even"].items():
        if k.startswith("_"):
            continue
        q = tuple(int(v) for v in k.split(","))
        even = {e: c for e, c in basis[q].items() if e[0] % 2 == 0 and e[1] % 2 == 0}
        assert even == _poly_x(d), k


@pytest.mark.parametrize("m,akey,bkey", [(6, "A6", "B6"), (11, "A11", "B11")])
def test_operator_values_as_printed(m, akey, bkey):
    w = derive.node_weights(m)
    for key, gold in ((akey, GOLD[akey]), (bkey, GOLD[bkey])):
        for k, d in gold.items():
            if k.startswith("_"):
                continue
            q = tuple(int(v) for v in k.split(","))
            got = w[q][0] if key == akey else w[q][1]
            assert got == _poly_l(d), (key, k)


def _gauss_disk(func, n=40):
    """Integral over the unit disk of func(z1, z2) / sqrt(1 - |z|^2).

    Polar coordinates with rho = sin(psi) remove the edge singularity:
    d(z) / sqrt(1-rho^2) = rho d(rho) d(theta) / cos(psi) = sin(psi) d(psi) d(theta)."""
    xg, wg = np.polynomial.legendre.leggauss(n)
    psi = (xg + 1) * (math.pi / 4)
    wpsi = wg * (math.pi / 4)
    th = (xg + 1) * math.pi
    wth = wg * math.pi
    total = 0.0
    for p, wp in zip(psi, wpsi):
        rho = math.sin(p)
        z1 = rho * np.cos(th)
        z2 = rho * np.sin(th)
        total += wp * math.sin(p) * np.sum(wth * func(z1, z2))
    return total


@pytest.mark.parametrize("a1,a2", [(0, 0), (1, 0), (2, 0), (1, 1), (2, 2), (4, 0), (3, 1), (0, 6), (4, 2)])
@pytest.mark.parametrize("lam", [0.3, 0.7071])
def test_exact_integrals_against_operator_definition(a1, a2, lam):
    """eq. exact1/exact2 vs eq. Op1/Op2 at x = 0, h = 1, c*tau = lambda."""
    ct = lam

    def f(y1, y2):
        return y1 ** a1 * y2 ** a2

    def grad(y1, y2):
        g1 = a1 * y1 ** (a1 - 1) * y2 ** a2 if a1 else 0.0 * y1
        g2 = a2 * y1 ** a1 * y2 ** (a2 - 1) if a2 else 0.0 * y2
        return g1, g2

    def integrand_A(z1, z2):
        g1, g2 = grad(ct * z1, ct * z2)
        return f(ct * z1, ct * z2) + ct * (g1 * z1 + g2 * z2)

    A_num = _gauss_disk(integrand_A) / (2 * math.pi)
    B_num = _gauss_disk(lambda z1, z2: f(ct * z1, ct * z2)) / (2 * math.pi)  # divided by tau
    A_cf = derive.evaluate(derive.A_monomial(a1, a2), lam)
    B_cf = derive.evaluate(derive.B_monomial(a1, a2), lam)
    assert abs(A_num - A_cf) < 1e-12
    assert abs(B_num - B_cf) < 1e-12


def test_B_over_A_ratio_is_degree_dependent():
    # B mu / A mu = tau / (a1 + a2 + 1): 1/3 at degree 2 and 1/5 at degree 4,
    # so the first-step v-bracket is the u-bracket with lambda^2 -> 3 lambda^2 / 5.
    for (a1, a2) in [(2, 0), (0, 2), (4, 0), (2, 2)]:
        A = derive.A_monomial(a1, a2)
        B = derive.B_monomial(a1, a2)
        d = a1 + a2
        assert B[d] / A[d] == Fraction(1, d + 1)

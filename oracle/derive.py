"""Stencil construction of Sec. 4-5 in exact rational arithmetic.

TEST INFRASTRUCTURE (part of the oracle; see ``oracle/__init__.py``).

This follows the paper's construction in its own order and notation:

  1. McKinney's correspondence between a stencil offset q and a monomial
     exponent alpha (Sec. 4, eq. alpha) and its inverse (eq. invMcKinney).
  2. The ordering g(alpha1, alpha2) of all monomials (Sec. 4, eq. g); the set
     M*_{<=m} is the first m monomials in that order, and the stencil Q_m is
     the image of M*_{<=m} under the inverse map.
  3. The matrix D = [mu_s(x_(r))] (eq. matrix1), its inverse C (eq. matrix2)
     and the Lagrange basis L_s = sum_r c_sr mu_r (eq. Lagrange), relabelled
     phi_{q1,q2} = L_{gamma(q1,q2)} (eq. Lagrange3, Lagrange4).
  4. The exact values of the operators A and B on a scaled monomial
     (Sec. 5, eq. exact1, exact2), which make A phi_q and B phi_q polynomials
     in the Courant number lambda.

Everything runs in scaled coordinates x/h (h = 1), so stencil nodes sit at
integer offsets; a monomial of total degree d then carries h^d, which is how
det D = 4 h^8 of Sec. 6.1 arises.

Polynomials in lambda are dicts {power: Fraction}.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Dict, List, Tuple

Poly = Dict[int, Fraction]


# -- Sec. 4 ------------------------------------------------------------------

def alpha(q: int) -> int:
    """Exponent assigned to offset q (eq. alpha)."""
    return 2 * abs(q) - 1 if q < 0 else 2 * q


def q_of(a: int) -> int:
    """Inverse of ``alpha`` (eq. invMcKinney): (-1)^a * floor((a+1)/2)."""
    return (-1) ** a * ((a + 1) // 2)


def g(a1: int, a2: int) -> int:
    """Ordinal number of x1^a1 x2^a2 (eq. g)."""
    d = a1 + a2
    base = d * (d + 1) // 2
    return base + (a1 - a2 if a2 < a1 else a2 - a1 + 1)


def monomials(m: int) -> List[Tuple[int, int]]:
    """M*_{<=m}: the first m exponent pairs in the order induced by g."""
    out = {}
    d = 0
    while len(out) < m or min(out) != 1:
        for a1 in range(d + 1):
            a2 = d - a1
            s = g(a1, a2)
            if s <= m:
                out[s] = (a1, a2)
        d += 1
        if d > 2 * m + 2:
            break
    if sorted(out) != list(range(1, m + 1)):
        raise AssertionError("g is not onto 1..m")
    return [out[s] for s in range(1, m + 1)]


def stencil(m: int) -> List[Tuple[int, int]]:
    """Q_m in the order of M*_{<=m}: node (q(alpha1), q(alpha2)) per monomial."""
    return [(q_of(a1), q_of(a2)) for (a1, a2) in monomials(m)]


def _mono(e: Tuple[int, int], x: Tuple[int, int]) -> Fraction:
    return Fraction(x[0]) ** e[0] * Fraction(x[1]) ** e[1]


def _inverse(M: List[List[Fraction]]) -> Tuple[List[List[Fraction]], Fraction]:
    """Gauss-Jordan inverse and determinant over the rationals."""
    n = len(M)
    A = [row[:] + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(M)]
    det = Fraction(1)
    for col in range(n):
        piv = next((r for r in range(col, n) if A[r][col] != 0), None)
        if piv is None:
            return None, Fraction(0)
        if piv != col:
            A[col], A[piv] = A[piv], A[col]
            det = -det
        p = A[col][col]
        det *= p
        A[col] = [v / p for v in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [vr - f * vc for vr, vc in zip(A[r], A[col])]
    return [row[n:] for row in A], det


def vandermonde(m: int) -> List[List[Fraction]]:
    """D[s][r] = mu_s(x_(r)) for the monomials and nodes of M*_{<=m} (h = 1)."""
    E = monomials(m)
    X = stencil(m)
    return [[_mono(E[s], X[r]) for r in range(m)] for s in range(m)]


def lagrange_basis(m: int):
    """phi_{q} as {exponent: coefficient} for each node q of Q_m, and det D.

    L_s = sum_r C[s][r] mu_r with C = D^{-1}; then L_s(x_(t)) = (C D)[s][t],
    the Kronecker delta, so L_s is the basis function of node x_(s), and
    phi_{q1,q2} = L_{gamma(q1,q2)} with gamma(q) = g(alpha(q1), alpha(q2))."""
    E = monomials(m)
    X = stencil(m)
    C, det = _inverse(vandermonde(m))
    if C is None:
        raise ValueError(f"Q_{m} is not unisolvent")
    basis = {}
    for q in X:
        s = g(alpha(q[0]), alpha(q[1])) - 1
        assert X[s] == q
        basis[q] = {E[r]: C[s][r] for r in range(m) if C[s][r] != 0}
    return basis, det


# -- Sec. 5 ------------------------------------------------------------------

def _dfact(n: int) -> int:
    """Double factorial with (-1)!! = 0!! = 1."""
    out = 1
    while n > 1:
        out *= n
        n -= 2
    return out


def A_monomial(a1: int, a2: int) -> Poly:
    """A(x_ij, tau) applied to (y1/h)^a1 (y2/h)^a2 (eq. exact1, exact2)."""
    if a1 % 2 or a2 % 2:
        return {}
    return {a1 + a2: Fraction(_dfact(a1 - 1) * _dfact(a2 - 1), _dfact(a1 + a2 - 1))}


def B_monomial(a1: int, a2: int) -> Poly:
    """B(x_ij, tau) on the same monomial, divided by tau (eq. exact2)."""
    A = A_monomial(a1, a2)
    return {p: c / (a1 + a2 + 1) for p, c in A.items()}


def _add(P: Poly, Qp: Poly, f: Fraction) -> None:
    for p, c in Qp.items():
        P[p] = P.get(p, Fraction(0)) + f * c
        if P[p] == 0:
            del P[p]


def node_weights(m: int):
    """For each node q of Q_m: (A phi_q, B phi_q / tau) as polynomials in lambda."""
    basis, _ = lagrange_basis(m)
    out = {}
    for q, poly in basis.items():
        Aw: Poly = {}
        Bw: Poly = {}
        for e, coef in poly.items():
            _add(Aw, A_monomial(*e), coef)
            _add(Bw, B_monomial(*e), coef)
        out[q] = (Aw, Bw)
    return out


def node_weights_for(nodes: List[Tuple[int, int]], exps: List[Tuple[int, int]]):
    """Node weights for an explicit stencil and monomial set (the general
    form of Sec. 4: any unisolvent pair; Sec. 5 for the operators).

    D[s][r] = mu_s(x_r) (eq. matrix1), C = D^{-1} (eq. matrix2), the basis
    function of node r is sum_s C[r][s] mu_s (eq. Lagrange), and its weights
    are (A phi_r, B phi_r / tau) as polynomials in lambda.  Returns
    {node: (A, B)}; raises ValueError when D is singular."""
    m = len(nodes)
    if len(exps) != m:
        raise ValueError("need as many monomials as nodes")
    D = [[_mono(exps[s], nodes[r]) for r in range(m)] for s in range(m)]
    C, det = _inverse(D)
    if C is None:
        raise ValueError("the stencil is not unisolvent for these monomials")
    out = {}
    for r, q in enumerate(nodes):
        Aw: Poly = {}
        Bw: Poly = {}
        for s in range(m):
            if C[r][s] != 0:
                _add(Aw, A_monomial(*exps[s]), C[r][s])
                _add(Bw, B_monomial(*exps[s]), C[r][s])
        out[tuple(q)] = (Aw, Bw)
    return out


def evaluate(P: Poly, lam) -> float:
    return sum(float(c) * lam ** p for p, c in P.items())


def evaluate_exact(P: Poly, lam: Fraction) -> Fraction:
    return sum((c * lam ** p for p, c in P.items()), Fraction(0))


SCHEME_M = {5: 6, 9: 11, 13: 15}

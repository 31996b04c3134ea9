"""FP64 CPU oracle for the Poisson-formula wave schemes (arXiv:1904.04048).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  It shares no code with the GPU library and never
imports it.

Contents
  * ``wave2d_oracle.c`` (built into ``liboracle.so`` with gcc, -O2
    -ffp-contract=off): the schemes as printed -- first step eq. A1 through
    comp5.1 / comp9.1 / comp13.1, two-step eq. A2 through comp5.2 / comp9.2 /
    comp13.2, the conventional comparison variants, the grid boundary rule of
    Sec. 6.1.2 and the norms.
  * ``derive``: the stencil construction of Sec. 4-5 in exact rational
    arithmetic (pins the printed weights).
  * ``modes``: the discrete solution for sine-series data in closed form
    (pins the full-grid runs and checks runs too large to repeat here).

This module wraps the C library with numpy.  Arrays are float64, shape
(ny, nx), C-contiguous: ``u[j, i]`` is the node (i*h, j*h).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wave2d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

P5, P9, P13, C9 = 5, 9, 13, 109
SCHEMES = (P5, P9, P13)
FIRST_CONVENTIONAL = 1
PERIODIC = 4

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, FP contraction off, OpenMP rows)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        D, I, U, Lg = ctypes.c_double, ctypes.c_int, ctypes.c_uint, ctypes.c_long
        P = ctypes.c_void_p
        L.orc_brackets.argtypes = [I, D, P, P, P]
        L.orc_brackets.restype = I
        L.orc_lambda_max.argtypes = [I]
        L.orc_lambda_max.restype = D
        L.orc_first_step.argtypes = [I, I, D, D, D, I, U, P, P, P]
        L.orc_first_step.restype = I
        L.orc_step.argtypes = [I, I, D, D, D, I, U, P, P, P]
        L.orc_step.restype = I
        L.orc_steps.argtypes = [I, I, D, D, D, I, U, Lg, P, P]
        L.orc_steps.restype = I
        L.orc_run.argtypes = [I, I, D, D, D, I, U, Lg, P, P, P, P]
        L.orc_run.restype = I
        L.orc_norms.argtypes = [Lg, P, P, P]
        L.orc_norms.restype = None
        L.orc_set_scheme.argtypes = [I, I, I, P, P]
        L.orc_class_brackets.argtypes = [I, D, P, P, P]
        L.orc_class_brackets.restype = I
        L.orc_set_scheme.restype = I
        L.orc_set_threads.argtypes = [I]
        L.orc_set_threads.restype = None
        L.orc_get_threads.argtypes = []
        L.orc_get_threads.restype = I
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _grid(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2:
        raise ValueError("expected a 2-D array (ny, nx)")
    return a


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def brackets(scheme: int, lam: float):
    """(a[3], b[3], has_b) of the printed scheme at Courant number lam."""
    a = np.zeros(3)
    b = np.zeros(3)
    hb = ctypes.c_int(0)
    if lib().orc_brackets(int(scheme), float(lam), _ptr(a), _ptr(b), ctypes.byref(hb)):
        raise ValueError(f"unknown scheme {scheme}")
    return a, b, bool(hb.value)


CUSTOM_DEG = 12

# Node classes of a symmetric stencil up to three lines from the centre, in
# the C oracle's order: class (q1, q2) holds (+-q1, +-q2) and (+-q2, +-q1).
CLASSES = ((1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1), (3, 2), (3, 3))


def class_nodes(q1: int, q2: int):
    """The nodes of class (q1, q2): four on an axis or diagonal, else eight."""
    return sorted({(sx * a, sy * b) for (a, b) in ((q1, q2), (q2, q1)) for sx in (1, -1) for sy in (1, -1)})


def register_scheme(scheme_id: int, weights) -> None:
    """Make scheme_id (1000..1015) run the scheme with these node weights:
    {node: (A, B / tau)} as polynomials in lambda ({power: coefficient}),
    e.g. from ``derive.node_weights_for``.  Every node of a class must carry
    the same weights, and a class with weight must have all its nodes;
    nodes more than three lines from the centre must carry none.  First
    step eq. A1, two-step update eq. A2."""
    a = np.zeros((len(CLASSES), CUSTOM_DEG + 1))
    b = np.zeros((len(CLASSES), CUSTOM_DEG + 1))
    index = {c: k for k, c in enumerate(CLASSES)}
    per_class = {}
    for q, (A, B) in weights.items():
        key = tuple(sorted((abs(q[0]), abs(q[1])), reverse=True))
        if key == (0, 0):
            continue  # the centre weight is one minus the others (eq. A1, A2 as class sums)
        has = any(A.values()) or any(B.values())
        if key not in index:
            if has:
                raise ValueError(f"node {q} carries weight more than three lines from the centre")
            continue
        per_class.setdefault(key, []).append((tuple(q), dict(A), dict(B), has))
    for key, nodes in per_class.items():
        if not any(n[3] for n in nodes):
            continue
        if sorted(n[0] for n in nodes) != class_nodes(*key):
            raise ValueError(f"class {key} carries weight but the stencil lacks some of its nodes")
        ref = nodes[0]
        for n in nodes[1:]:
            if n[1] != ref[1] or n[2] != ref[2]:
                raise ValueError(f"node {n[0]} has other weights than {ref[0]} of the same class")
        c = index[key]
        for p_, v in ref[1].items():
            a[c, p_] = float(v)
        for p_, v in ref[2].items():
            b[c, p_] = float(v)
    if lib().orc_set_scheme(int(scheme_id), len(CLASSES), CUSTOM_DEG, _ptr(a), _ptr(b)):
        raise ValueError(f"bad custom scheme id {scheme_id}")


def class_brackets(scheme: int, lam: float):
    """(a[9], b[9], has_b): brackets of every class of CLASSES, normalised as
    in ``brackets`` (zero for the classes a scheme does not use)."""
    a = np.zeros(len(CLASSES))
    b = np.zeros(len(CLASSES))
    hb = ctypes.c_int(0)
    if lib().orc_class_brackets(int(scheme), float(lam), _ptr(a), _ptr(b), ctypes.byref(hb)):
        raise ValueError(f"unknown scheme {scheme}")
    return a, b, bool(hb.value)


def lambda_max(scheme: int) -> float:
    v = lib().orc_lambda_max(int(scheme))
    if v < 0:
        raise ValueError(f"unknown scheme {scheme}")
    return v


def first_step(u0, v0, h, tau, c, scheme, flags=0) -> np.ndarray:
    u0 = _grid(u0)
    v0 = _grid(v0)
    if u0.shape != v0.shape:
        raise ValueError("u0 and v0 differ in shape")
    ny, nx = u0.shape
    u1 = np.empty_like(u0)
    if lib().orc_first_step(nx, ny, h, tau, c, scheme, flags, _ptr(u0), _ptr(v0), _ptr(u1)):
        raise ValueError("oracle rejected the first-step arguments")
    return u1


def step(um1, u, h, tau, c, scheme, flags=0) -> np.ndarray:
    um1 = _grid(um1)
    u = _grid(u)
    ny, nx = u.shape
    up1 = np.empty_like(u)
    if lib().orc_step(nx, ny, h, tau, c, scheme, flags, _ptr(um1), _ptr(u), _ptr(up1)):
        raise ValueError("oracle rejected the step arguments")
    return up1


def steps(um1, u, h, tau, c, scheme, nsteps, flags=0):
    """Advance (u^{k-1}, u^k) by nsteps two-step updates; returns new copies."""
    um1 = _grid(um1).copy()
    u = _grid(u).copy()
    ny, nx = u.shape
    if lib().orc_steps(nx, ny, h, tau, c, scheme, flags, int(nsteps), _ptr(um1), _ptr(u)):
        raise ValueError("oracle rejected the steps arguments")
    return um1, u


def run(u0, v0, h, tau, c, scheme, nsteps, flags=0):
    """First step then nsteps-1 two-step updates: returns (u^{n-1}, u^n)."""
    u0 = _grid(u0)
    v0 = _grid(v0)
    ny, nx = u0.shape
    up = np.empty_like(u0)
    uo = np.empty_like(u0)
    if lib().orc_run(nx, ny, h, tau, c, scheme, flags, int(nsteps), _ptr(u0), _ptr(v0),
                     _ptr(up), _ptr(uo)):
        raise ValueError("oracle rejected the run arguments")
    return up, uo


def norms(a, b):
    """{max|a-b|, max|b|, sum (a-b)^2, sum b^2} in FP64, index order."""
    a = np.ascontiguousarray(a, dtype=np.float64).ravel()
    b = np.ascontiguousarray(b, dtype=np.float64).ravel()
    if a.size != b.size:
        raise ValueError("size mismatch")
    out = np.zeros(4)
    lib().orc_norms(a.size, _ptr(a), _ptr(b), _ptr(out))
    return out


def rel_max_err(a, b) -> float:
    """max|a-b| / max|b| (the tolerance measure used for GPU parity).

    Raises ValueError when either array holds a NaN or an infinity: a result
    that was never written (the GPU tests pre-fill outputs with NaN) or that
    blew up must fail a parity check, never pass it."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    for name, x in (("result", a), ("reference", b)):
        if not np.isfinite(x).all():
            bad = int(x.size - np.count_nonzero(np.isfinite(x)))
            raise ValueError(f"{name} holds {bad} non-finite value(s) of {x.size}")
    n = norms(a, b)
    return float(n[0] / n[1]) if n[1] > 0 else float(n[0])


def paper_error(u0, v0, h, tau, c, scheme, n_t, exact, flags=0, wrap=False) -> float:
    """Relative L2 error E(n, n_t) of Sec. 6.1.2 (eq. error): the sums run over
    levels k = 1..n_t and over every grid node, boundary included.

    ``exact(k)`` returns the exact solution sampled on the same nodes at
    t = k*tau.  With ``wrap`` (periodic runs on the n unique nodes) the sums
    run over the n+1 nodes 0..n of each line, node n being node 0 again."""
    um1 = _grid(u0)
    u = first_step(u0, v0, h, tau, c, scheme, flags)
    if not (flags & PERIODIC):
        um1 = um1.copy()
        um1[0, :] = 0.0; um1[-1, :] = 0.0; um1[:, 0] = 0.0; um1[:, -1] = 0.0
    num = 0.0
    den = 0.0
    for k in range(1, n_t + 1):
        if k > 1:
            um1, u = u, step(um1, u, h, tau, c, scheme, flags)
        uk = u
        ue = exact(k)
        if wrap:
            uk = np.pad(uk, ((0, 1), (0, 1)), mode="wrap")
            ue = np.pad(ue, ((0, 1), (0, 1)), mode="wrap")
        nr = norms(uk, ue)
        num += nr[2]
        den += nr[3]
    return float(np.sqrt(num / den))

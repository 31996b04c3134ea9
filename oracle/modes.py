"""Closed-form discrete solution of the schemes for sine-series data.

TEST INFRASTRUCTURE (part of the oracle; see ``oracle/__init__.py``).

On a grid of nx x ny nodes with the Dirichlet-zero / odd-reflection rule of
the oracle (or the periodic rule), a discrete sine mode

    e_m(i, j) = sin(p_m pi i / (nx-1)) * sin(q_m pi j / (ny-1))

is an eigenvector of every rotation sum of Sec. 6.2.1 (eq. notations2): with
theta = p pi/(nx-1), phi = q pi/(ny-1) and s_x = sin(theta/2), s_y =
sin(phi/2),

    delta(1,0) -> -4 (s_x^2 + s_y^2)
    delta(1,1) -> 4 (cos theta cos phi - 1) = -8 (s_x^2 + s_y^2) + 16 s_x^2 s_y^2
    delta(2,0) -> -4 (sin^2 theta + sin^2 phi).

So each mode amplitude obeys the scalar form of eq. A1 and A2:

    a_1     = (1 + sA) a_0 + tau (1 + sB) b_0
    a_{k+1} = 2 (1 + sA) a_k - a_{k-1},

with sA = lambda^2/2 * (a . delta) and sB = lambda^2/6 * (b . delta) the mode
symbols of A - 1 and B/tau - 1 (sB = 0 for the conventional first step).
Writing 1 + sA = cos w (sin(w/2) = sqrt(-sA/2), accurate for small w) gives

    a_k = a_0 cos(k w) + tau (1 + sB) b_0 sin(k w) / sin(w).

The weights come from the oracle's own printed brackets.  This holds at any
grid size and step count, which is what lets the tests check runs that are
too large for the full-grid oracle.  It is pinned against the full-grid
oracle on small grids by the test suite.
"""
from __future__ import annotations

import math

import numpy as np

from . import brackets, FIRST_CONVENTIONAL


def symbols(scheme, lam, theta, phi, conventional=False):
    a, b, has_b = brackets(scheme, lam)
    sx2 = math.sin(theta / 2) ** 2
    sy2 = math.sin(phi / 2) ** 2
    d10 = -4.0 * (sx2 + sy2)
    d11 = -8.0 * (sx2 + sy2) + 16.0 * sx2 * sy2
    d20 = -4.0 * (math.sin(theta) ** 2 + math.sin(phi) ** 2)
    l2 = lam * lam
    sA = l2 / 2.0 * (a[0] * d10 + a[1] * d11 + a[2] * d20)
    sB = 0.0
    if has_b and not conventional:
        sB = l2 / 6.0 * (b[0] * d10 + b[1] * d11 + b[2] * d20)
    return sA, sB


def amplitude(scheme, lam, tau, theta, phi, a0, b0, k, conventional=False):
    """Mode amplitude at level k (k >= 0)."""
    sA, sB = symbols(scheme, lam, theta, phi, conventional)
    if k == 0:
        return a0
    x = -sA / 2.0
    if not (0.0 < x <= 1.0):
        # Outside the stable range (or a zero symbol): iterate the recurrence.
        am1, ak = a0, (1.0 + sA) * a0 + tau * (1.0 + sB) * b0
        for _ in range(k - 1):
            am1, ak = ak, 2.0 * (1.0 + sA) * ak - am1
        return ak
    w = 2.0 * math.asin(math.sqrt(x))
    return a0 * math.cos(k * w) + tau * (1.0 + sB) * b0 * math.sin(k * w) / math.sin(w)


def solution(modes, nx, ny, h, tau, c, scheme, k, flags=0):
    """Grid function at level k for data u0 = sum_m A_m e_m, v0 = sum_m B_m e_m.

    ``modes`` is a list of (p, q, A, B) with integer p, q >= 1.  Returns a
    float64 array of shape (ny, nx)."""
    lam = c * tau / h
    conv = bool(flags & FIRST_CONVENTIONAL)
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    out = np.zeros((ny, nx))
    for (p, q, A, B) in modes:
        theta = p * math.pi / (nx - 1)
        phi = q * math.pi / (ny - 1)
        amp = amplitude(scheme, lam, tau, theta, phi, A, B, k, conv)
        out += amp * np.outer(np.sin(q * math.pi * y / (ny - 1)), np.sin(p * math.pi * x / (nx - 1)))
    return out


def solution_at(modes, nx, ny, h, tau, c, scheme, k, ii, jj, flags=0):
    """Level-k values at the sampled nodes (ii[s], jj[s]) only."""
    lam = c * tau / h
    conv = bool(flags & FIRST_CONVENTIONAL)
    ii = np.asarray(ii, dtype=np.float64)
    jj = np.asarray(jj, dtype=np.float64)
    out = np.zeros(ii.shape)
    for (p, q, A, B) in modes:
        theta = p * math.pi / (nx - 1)
        phi = q * math.pi / (ny - 1)
        amp = amplitude(scheme, lam, tau, theta, phi, A, B, k, conv)
        out += amp * np.sin(p * math.pi * ii / (nx - 1)) * np.sin(q * math.pi * jj / (ny - 1))
    return out

"""A conservation law of the two-step update, pinned on the oracle.

The two-step update (eq. A2) has the form u^{k+1} - 2u^k + u^{k-1} = A u^k
with A the scheme's stencil operator.  Every scheme's stencil is symmetric
(opposite nodes carry equal weights), and both boundary rules keep A
symmetric on the grid's nodes: Dirichlet boundary nodes are held at zero,
the 13-point ghost line (the odd reflection of the line inside) only adds to
the diagonal, and the periodic operator is circulant.  For such A the
quantity

    E_k = |u^{k+1} - u^k|^2 - <u^{k+1}, A u^k>

is exactly conserved: E_k - E_{k-1} = <A u^k, u^{k+1} - u^{k-1}>
- <u^{k+1}, A u^k> + <u^k, A u^{k-1}> = 0.  It holds at any grid size, so
it also checks full-size GPU runs (tests/test_gpu_fullsize.py).  A u is
obtained from the oracle's own update with a zero previous level:
step(0, u) = 2u + A u.  The Dirichlet rule's case, with a direct check of
the symmetry of A, is in tests/test_oracle_pins.py; this file adds the
periodic rule and a planted mistake.

A dropped or one-sided stencil term, or a boundary rule that is not an odd
reflection, breaks the symmetry and the conservation; the planted-mistake
case below shows the check notices a one-sided weight.
"""
import numpy as np
import pytest

import oracle

SCHEMES = (5, 9, 13, 109)  # the Poisson schemes and the conventional 9-point one


def apply_a(u, h, tau, c, scheme, flags=0):
    return oracle.step(np.zeros_like(u), u, h, tau, c, scheme, flags) - 2.0 * u


def energy(um, u, h, tau, c, scheme, flags=0):
    d = u - um
    return float(np.sum(d * d) - np.sum(u * apply_a(um, h, tau, c, scheme, flags)))


def _data(nx, ny, seed, periodic):
    rng = np.random.default_rng(seed)
    u0 = rng.standard_normal((ny, nx))
    v0 = rng.standard_normal((ny, nx))
    if not periodic:
        for a in (u0, v0):
            a[0, :] = a[-1, :] = a[:, 0] = a[:, -1] = 0.0
    return u0, v0


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("periodic", [True], ids=["periodic"])
def test_energy_is_conserved(scheme, periodic):
    nx, ny = 23, 17
    flags = oracle.PERIODIC if periodic else 0
    h = 1.0 / (nx - 1)
    tau = 0.9 * oracle.lambda_max(scheme) * h
    u0, v0 = _data(nx, ny, scheme, periodic)
    um, u = oracle.run(u0, v0, h, tau, 1.0, scheme, 2, flags)
    e0 = energy(um, u, h, tau, 1.0, scheme, flags)
    assert e0 > 0.0  # stable Courant number: E is a norm
    for _ in range(6):
        um, u = oracle.steps(um, u, h, tau, 1.0, scheme, 97, flags)
        e = energy(um, u, h, tau, 1.0, scheme, flags)
        assert abs(e - e0) <= 1e-12 * e0, (scheme, e, e0)


def test_energy_notices_a_one_sided_weight():
    # Plant a mistake in a copy of the update: the east neighbour weighted
    # 1% more than the west one.  The conservation law fails at once.
    nx, ny = 23, 17
    h = 1.0 / (nx - 1)
    tau = 0.6 * h
    u0, v0 = _data(nx, ny, 1, False)
    um, u = oracle.run(u0, v0, h, tau, 1.0, 5, 2)

    def bad_step(um, u):
        up = oracle.step(um, u, h, tau, 1.0, 5)
        lam2 = (tau / h) ** 2
        up[1:-1, 1:-1] += 0.01 * lam2 * u[1:-1, 2:]
        return up

    e0 = energy(um, u, h, tau, 1.0, 5)
    for _ in range(20):
        um, u = u, bad_step(um, u)
    assert abs(energy(um, u, h, tau, 1.0, 5) - e0) > 1e-6 * e0

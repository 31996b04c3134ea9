"""GPU runs of a scheme whose stencil reaches three lines out (Sec. 4-5).

The complete monomial set of degree 6 (Q_28, M*_{<=28}) gives a 25-node
scheme with weight on the classes (1,0), (1,1), (2,0), (2,1) and (3,0).  The
library builds it with its own floating-point construction and runs it with
its LDS-tiled one-level kernels; the oracle runs the exact weights.  FP64
results match to 1e-12 and compensated FP32 to 1e-5 of max|u|, on both
boundary rules, on grids from 3 x 3 (one updated node, ghosts reflected two
lines out) through ragged multi-tile sizes and padded rows.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1904_04048_amd as w
from oracle import derive
from tests.gpu_util import dev_grid, empty_like_grid, padding_intact, rough_data, smooth_data

pytestmark = pytest.mark.gpu

ORC_DEG6 = 1002


@pytest.fixture(scope="module")
def deg6():
    oracle.register_scheme(ORC_DEG6, derive.node_weights(28))
    return w.wave2d_scheme_create(derive.stencil(28), derive.monomials(28))


SHAPES = [(3, 3), (4, 7), (7, 7), (8, 9), (70, 13), (131, 97), (200, 129), (65, 260)]


# A periodic grid needs 7 x 7 nodes for a radius-3 stencil.
CASES = [(s, p) for s in SHAPES for p in (False, True) if not (p and min(s) < 7)]


@pytest.mark.parametrize("shape,periodic", CASES,
                         ids=[f"{s[0]}x{s[1]}-{'periodic' if p else 'dirichlet'}" for s, p in CASES])
@pytest.mark.parametrize("conv", [False, True], ids=["poisson", "conventional"])
def test_wide_scheme_matches_oracle(deg6, shape, periodic, conv):
    nx, ny = shape
    u0, v0 = rough_data(nx, ny, nx * 5 + ny)
    h = 1.0 / max(nx, ny)
    tau = 0.95 * w.wave2d_lambda_max(deg6) * h
    steps = 23
    f = (w.PERIODIC if periodic else 0) | (w.FIRST_CONVENTIONAL if conv else 0)
    of = (oracle.PERIODIC if periodic else 0) | (oracle.FIRST_CONVENTIONAL if conv else 0)
    print(f"wide scheme {nx}x{ny} periodic={periodic} conventional={conv}", flush=True)
    o1 = oracle.first_step(u0, v0, h, tau, 1.0, ORC_DEG6, of)
    rp, rc = oracle.run(u0, v0, h, tau, 1.0, ORC_DEG6, steps, of)
    U0, V0 = dev_grid(u0), dev_grid(v0)
    U1 = torch.full_like(U0, float("nan"))
    w.wave2d_first_step(U0, V0, U1, h, tau, 1.0, deg6, f)
    assert oracle.rel_max_err(U1.cpu().numpy(), o1) <= 1e-12
    P, C = torch.full_like(U0, float("nan")), torch.full_like(U0, float("nan"))
    w.wave2d_run(U0, V0, P, C, h, tau, 1.0, deg6, steps, f)
    assert oracle.rel_max_err(C.cpu().numpy(), rc) <= 1e-12
    assert oracle.rel_max_err(P.cpu().numpy(), rp) <= 1e-12
    u = torch.full(U0.shape, float("nan"), dtype=torch.float32, device=U0.device)
    lo, d = torch.full_like(u, float("nan")), torch.full_like(u, float("nan"))
    w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, deg6, steps, f)
    out = torch.empty_like(U0)
    w.wave2d_f32c_export(u, lo, out)
    assert oracle.rel_max_err(out.cpu().numpy(), rc) <= 1e-5


def test_wide_first_step_of_an_impulse_is_the_derived_weights(deg6):
    """Node by node: A phi_q and B phi_q / tau of the exact construction."""
    n = 15
    lam = 0.4
    h = 0.1
    tau = lam * h
    e = np.zeros((n, n))
    e[n // 2, n // 2] = 1.0
    E, Z = dev_grid(e), dev_grid(np.zeros((n, n)))
    RA, RB = torch.empty_like(E), torch.empty_like(E)
    w.wave2d_first_step(E, Z, RA, h, tau, 1.0, deg6)
    w.wave2d_first_step(Z, E, RB, h, tau, 1.0, deg6)
    rA, rB = RA.cpu().numpy(), RB.cpu().numpy()
    c = n // 2
    mask = np.zeros((n, n), dtype=bool)
    for (q1, q2), (A, B) in derive.node_weights(28).items():
        assert abs(rA[c - q2, c - q1] - derive.evaluate(A, lam)) < 1e-13, (q1, q2)
        assert abs(rB[c - q2, c - q1] / tau - derive.evaluate(B, lam)) < 1e-12, (q1, q2)
        mask[c - q2, c - q1] = True
    assert np.all(rA[~mask] == 0) and np.all(rB[~mask] == 0)


@pytest.mark.parametrize("ld", [131, 160])
def test_wide_padded_rows(deg6, ld):
    nx, ny = 131, 70
    (u0, v0), _ = smooth_data(nx, ny, 3)
    h = 1.0 / (nx - 1)
    tau = 0.9 * w.wave2d_lambda_max(deg6) * h
    rp, rc = oracle.run(u0, v0, h, tau, 1.0, ORC_DEG6, 30)
    U0, V0 = dev_grid(u0, ld), dev_grid(v0, ld)
    P, C = empty_like_grid(U0), empty_like_grid(U0)
    w.wave2d_run(U0, V0, P, C, h, tau, 1.0, deg6, 30)
    assert oracle.rel_max_err(C.cpu().numpy(), rc) <= 1e-12
    assert padding_intact(P) and padding_intact(C)
    u = empty_like_grid(U0, torch.float32)
    lo, d = empty_like_grid(U0, torch.float32), empty_like_grid(U0, torch.float32)
    w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, deg6, 30)
    out = empty_like_grid(U0)
    w.wave2d_f32c_export(u, lo, out)
    assert oracle.rel_max_err(out.cpu().numpy(), rc) <= 1e-5
    assert padding_intact(u) and padding_intact(lo) and padding_intact(d)


def test_wide_long_compensated_run(deg6):
    """1500 levels of smooth data at 0.9 of the limit: compensated FP32
    within 1e-5 of max|u| of the FP64 oracle, FP64 within 1e-12."""
    nx, ny = 97, 80
    (u0, v0), _ = smooth_data(nx, ny, 8)
    h = 1.0 / (nx - 1)
    tau = 0.9 * w.wave2d_lambda_max(deg6) * h
    steps = 1500
    _, rc = oracle.run(u0, v0, h, tau, 1.0, ORC_DEG6, steps)
    U0, V0 = dev_grid(u0), dev_grid(v0)
    P, C = torch.empty_like(U0), torch.empty_like(U0)
    w.wave2d_run(U0, V0, P, C, h, tau, 1.0, deg6, steps)
    assert oracle.rel_max_err(C.cpu().numpy(), rc) <= 1e-12
    u = torch.empty(U0.shape, dtype=torch.float32, device=U0.device)
    lo, d = torch.empty_like(u), torch.empty_like(u)
    w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, deg6, steps)
    out = torch.empty_like(U0)
    w.wave2d_f32c_export(u, lo, out)
    err = oracle.rel_max_err(out.cpu().numpy(), rc)
    print(f"wide compensated FP32 after {steps} levels: {err:.3g} of max|u|", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("split", [1, 7, 12])
def test_wide_steps_resume_bitwise(deg6, split):
    """Stepping in two calls (library buffer, then a caller workspace)
    equals one call, in FP64 and compensated FP32, for odd and even counts."""
    nx, ny = 90, 75
    u0, v0 = rough_data(nx, ny, 21)
    h = 1.0 / 89
    tau = 0.8 * w.wave2d_lambda_max(deg6) * h
    U0, V0 = dev_grid(u0), dev_grid(v0)
    P, C = torch.empty_like(U0), torch.empty_like(U0)
    w.wave2d_run(U0, V0, P, C, h, tau, 1.0, deg6, 1)
    P2, C2 = P.clone(), C.clone()
    w.wave2d_step(P, C, h, tau, 1.0, deg6, 13)
    work = torch.empty(w.wave2d_work_bytes(w.F64, nx, ny), dtype=torch.uint8, device=U0.device)
    w.wave2d_step(P2, C2, h, tau, 1.0, deg6, split)
    w.wave2d_step(P2, C2, h, tau, 1.0, deg6, 13 - split, work=work)
    assert torch.equal(P, P2) and torch.equal(C, C2)
    u = torch.empty(U0.shape, dtype=torch.float32, device=U0.device)
    lo, d = torch.empty_like(u), torch.empty_like(u)
    w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, deg6, 1)
    a = [t.clone() for t in (u, lo, d)]
    w.wave2d_f32c_step(u, lo, d, h, tau, 1.0, deg6, 13)
    wk = torch.empty(w.wave2d_work_bytes(w.F32C, nx, ny), dtype=torch.uint8, device=U0.device)
    w.wave2d_f32c_step(*a, h, tau, 1.0, deg6, split)
    w.wave2d_f32c_step(*a, h, tau, 1.0, deg6, 13 - split, work=wk)
    assert all(torch.equal(x, y) for x, y in zip((u, lo, d), a))


def test_wide_scheme_refused_by_batch_server_and_autotune(deg6):
    nx = ny = 64
    dev = torch.device("cuda:0")
    U0 = torch.zeros((ny, nx), dtype=torch.float64, device=dev)
    u = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    inst = dict(nx=nx, ny=ny, h=1.0 / 63, tau=0.3 / 63, c=1.0, scheme=deg6, steps=5, flags=0,
                u0=U0, v0=U0.clone(), u=u, lo=torch.empty_like(u), d=torch.empty_like(u))
    with pytest.raises(w.Wave2dError) as e:
        w.wave2d_batch_create([inst])
    assert "three lines" in str(e.value)
    sv = w.wave2d_server_create(64 << 20)
    try:
        with pytest.raises(w.Wave2dError):
            w.wave2d_server_submit(sv, nx, ny, 1.0 / 63, 0.3 / 63, 1.0, deg6, 5, 0, u0=U0, v0=U0)
    finally:
        w.wave2d_server_destroy(sv)
    with pytest.raises(w.Wave2dError):
        w.wave2d_autotune(w.F32C, deg6, 256, 256)


@pytest.mark.parametrize("shape", [(4097, 4097), (8193, 4097)], ids=["4097x4097", "8193x4097"])
def test_wide_compensated_on_large_grids(deg6, shape):
    """Grids large enough that the compensated kernel's segment rule picks
    segments of several turns of its seven-row register ring (on MI355X,
    14 rows at 4097^2 and 28 at 8193 x 4097), against the oracle after a
    few levels, with FP64 alongside."""
    nx, ny = shape
    (u0, v0), _ = smooth_data(nx, ny, 3)
    h = 1.0 / (nx - 1)
    tau = 0.9 * w.wave2d_lambda_max(deg6) * h
    steps = 5
    print(f"wide scheme {nx}x{ny}, {steps} levels", flush=True)
    _, rc = oracle.run(u0, v0, h, tau, 1.0, ORC_DEG6, steps)
    U0, V0 = dev_grid(u0), dev_grid(v0)
    del u0, v0
    u = torch.full(U0.shape, float("nan"), dtype=torch.float32, device=U0.device)
    lo, d = torch.full_like(u, float("nan")), torch.full_like(u, float("nan"))
    w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, deg6, steps)
    out = torch.empty_like(U0)
    w.wave2d_f32c_export(u, lo, out)
    assert oracle.rel_max_err(out.cpu().numpy(), rc) <= 1e-5
    P, C = torch.empty_like(U0), torch.empty_like(U0)
    w.wave2d_run(U0, V0, P, C, h, tau, 1.0, deg6, steps)
    assert oracle.rel_max_err(C.cpu().numpy(), rc) <= 1e-12

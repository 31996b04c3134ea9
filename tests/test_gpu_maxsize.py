"""The largest grids the library accepts.

* A square grid just below the node limit (ld * ny < 2^31: 46300^2 nodes,
  17 GB per FP64 array), both precisions, all three Poisson schemes run in
  the launch shapes the library picks: sampled outputs (corners, edges,
  interior, random) against the oracle run on a window around each sample
  that holds the sample's domain of dependence (R nodes per level); where
  the window meets the grid's boundary, the window's edge is the grid's
  edge, so the boundary rule applies unchanged, and the other edges are far
  enough that their own rule cannot reach the sample.
* The periodic rule on the same grid (too large for one buffer range, so
  the one-node-per-thread kernels run it): windows wrap around the grid.
* Sides at the limit (2^18 x 3 and 3 x 2^18): against the full-grid oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1904_04048_amd as w
from tests.gpu_util import rough_data

pytestmark = pytest.mark.gpu

N = 46300
STEPS = 5


def _radius(scheme):
    return 2 if scheme == w.P13 else 1


def _samples(nx, ny, rng):
    pts = [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1), (1, 1), (2, nx // 2), (nx - 2, ny // 3),
           (nx // 2, ny - 3), (nx // 2, ny // 2), (127, 4097), (nx - 129, 63)]
    pts += [(int(rng.integers(0, nx)), int(rng.integers(0, ny))) for _ in range(8)]
    return pts


def _window(x, y, nx, ny, hw, periodic):
    """Index ranges of the window around (x, y): clipped at the grid's edges
    (Dirichlet) or wrapped (periodic)."""
    if periodic:
        xs = np.arange(x - hw, x + hw + 1) % nx
        ys = np.arange(y - hw, y + hw + 1) % ny
        return xs, ys, hw, hw
    x0, x1 = max(0, x - hw), min(nx, x + hw + 1)
    y0, y1 = max(0, y - hw), min(ny, y + hw + 1)
    return np.arange(x0, x1), np.arange(y0, y1), x - x0, y - y0


def _check_samples(U0, V0, out, scheme, h, tau, tol, periodic=False):
    ny, nx = U0.shape
    hw = _radius(scheme) * STEPS + 6
    rng = np.random.default_rng(scheme + (100 if periodic else 0))
    scale = float(torch.max(torch.abs(out)))
    assert scale > 0
    for (x, y) in _samples(nx, ny, rng):
        xs, ys, cx, cy = _window(x, y, nx, ny, hw, periodic)
        ix, iy = torch.from_numpy(xs).to(U0.device), torch.from_numpy(ys).to(U0.device)
        u0 = U0.index_select(0, iy).index_select(1, ix).cpu().numpy()
        v0 = V0.index_select(0, iy).index_select(1, ix).cpu().numpy()
        got = float(out[y, x])
        # The oracle runs the window with the Dirichlet rule: where the
        # window was clipped its edge is the grid's own; its other edges
        # (and every edge of a wrapped window) are too far to reach the
        # sample in STEPS levels.
        _, ref = oracle.run(u0, v0, h, tau, 1.0, scheme, STEPS)
        assert abs(got - ref[cy, cx]) <= tol * scale, (scheme, periodic, x, y, got, ref[cy, cx])


@pytest.fixture(scope="module")
def big_data():
    if torch.cuda.get_device_properties(0).total_memory < 200 * 2**30:
        pytest.skip("needs a device with 200 GiB")
    g = torch.Generator(device="cuda").manual_seed(2024)
    U0 = torch.rand((N, N), dtype=torch.float64, device="cuda", generator=g) - 0.5
    V0 = torch.rand((N, N), dtype=torch.float64, device="cuda", generator=g) - 0.5
    yield U0, V0
    del U0, V0
    torch.cuda.empty_cache()


@pytest.mark.parametrize("scheme", [w.P5, w.P9, w.P13])
@pytest.mark.parametrize("periodic", [False, True], ids=["dirichlet", "periodic"])
def test_max_grid_fp64(big_data, scheme, periodic):
    U0, V0 = big_data
    assert 0.99 * 2**31 < N * N < 2**31
    h = 1.0 / (N - 1)
    tau = 0.9 * w.wave2d_lambda_max(scheme) * h
    f = w.PERIODIC if periodic else 0
    P, C = torch.empty_like(U0), torch.empty_like(U0)
    work = torch.empty(w.wave2d_work_bytes(w.F64, N, N), dtype=torch.uint8, device="cuda")
    w.wave2d_run(U0, V0, P, C, h, tau, 1.0, scheme, STEPS, f, work=work)
    torch.cuda.synchronize()
    del P, work
    _check_samples(U0, V0, C, scheme, h, tau, 1e-12, periodic)
    del C
    torch.cuda.empty_cache()


@pytest.mark.parametrize("scheme", [w.P9, w.P13])
def test_max_grid_f32c(big_data, scheme):
    U0, V0 = big_data
    h = 1.0 / (N - 1)
    tau = 0.9 * w.wave2d_lambda_max(scheme) * h
    u = torch.empty((N, N), dtype=torch.float32, device="cuda")
    lo, d = torch.empty_like(u), torch.empty_like(u)
    work = torch.empty(w.wave2d_work_bytes(w.F32C, N, N), dtype=torch.uint8, device="cuda")
    w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, scheme, STEPS, work=work)
    del work
    out = torch.empty_like(U0)
    w.wave2d_f32c_export(u, lo, out)
    torch.cuda.synchronize()
    del u, lo, d
    _check_samples(U0, V0, out, scheme, h, tau, 1e-5)
    del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("shape", [(1 << 18, 3), (3, 1 << 18), (1 << 18, 7)], ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("scheme", [w.P9, w.P13])
def test_longest_sides(shape, scheme):
    nx, ny = shape
    u0, v0 = rough_data(nx, ny, nx + ny)
    h = 1.0 / (max(nx, ny) - 1)
    tau = 0.9 * w.wave2d_lambda_max(scheme) * h
    steps = 21
    _, rc = oracle.run(u0, v0, h, tau, 1.0, scheme, steps)
    U0 = torch.from_numpy(u0).cuda()
    V0 = torch.from_numpy(v0).cuda()
    P, C = torch.empty_like(U0), torch.empty_like(U0)
    w.wave2d_run(U0, V0, P, C, h, tau, 1.0, scheme, steps)
    assert oracle.rel_max_err(C.cpu().numpy(), rc) <= 1e-12
    u = torch.empty(U0.shape, dtype=torch.float32, device="cuda")
    lo, d = torch.empty_like(u), torch.empty_like(u)
    w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, scheme, steps)
    out = torch.empty_like(U0)
    w.wave2d_f32c_export(u, lo, out)
    assert oracle.rel_max_err(out.cpu().numpy(), rc) <= 1e-5

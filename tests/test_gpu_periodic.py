"""GPU tests of the periodic boundary rule (WAVE2D_PERIODIC, the rule of the
paper's Table 3, Sec. 6.3).

* FP64 runs against the oracle's periodic rule (index mod n, every node
  updated) to 1e-12, compensated FP32 runs to 1e-5, on even widths (the
  temporally blocked kernels) and odd widths (one-node-per-thread kernels).
* The temporally blocked kernels give the same values as the
  one-node-per-thread kernels for every depth and segment height.
* Table 3 on periodic grids is in test_gpu_tables.py.
* Batches take periodic instances of even width and reject odd widths.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1904_04048_amd as w
from tests.gpu_util import dev_grid, rough_data

pytestmark = pytest.mark.gpu

SCHEMES = [w.P5, w.P9, w.P13, w.C9]
SHAPES = [(8, 8), (16, 12), (33, 20), (64, 64), (130, 70), (257, 200), (260, 131), (6, 40)]


@pytest.fixture(autouse=True)
def _reset_tuning():
    yield
    for p in (w.F64, w.F32C):
        for s in (w.P5, w.P9, w.P13, w.C9):
            w.wave2d_set_tuning(p, s)


def _flags(scheme):
    return w.PERIODIC | (w.FIRST_CONVENTIONAL if scheme == w.C9 else 0)


def _periodic_data(nx, ny, seed):
    # Smooth periodic data: sums of Fourier modes of the n-node torus.
    rng = np.random.default_rng(seed)
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    X, Y = np.meshgrid(x, y)
    u0 = np.zeros((ny, nx))
    v0 = np.zeros((ny, nx))
    for _ in range(4):
        kx, ky = rng.integers(0, 3, size=2)
        ph = rng.uniform(0, 2 * math.pi, size=2)
        u0 += rng.standard_normal() * np.cos(2 * math.pi * (kx * X + ky * Y) + ph[0])
        v0 += rng.standard_normal() * np.cos(2 * math.pi * (kx * X + ky * Y) + ph[1])
    return u0, v0


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_periodic_fp64_and_f32c_match_oracle(scheme, shape):
    nx, ny = shape
    if scheme == w.P13 and min(nx, ny) < 5:
        pytest.skip("13-point periodic grids need 5 x 5 nodes")
    u0, v0 = _periodic_data(nx, ny, nx * 100 + ny)
    h = 1.0 / max(nx, ny)
    tau = 0.9 * w.wave2d_lambda_max(scheme) * h
    steps = 37
    f = _flags(scheme)
    rp, rc = oracle.run(u0, v0, h, tau, 1.0, scheme, steps, f)
    U0, V0 = dev_grid(u0), dev_grid(v0)
    P, C = torch.empty_like(U0), torch.empty_like(U0)
    w.wave2d_run(U0, V0, P, C, h, tau, 1.0, scheme, steps, f)
    assert oracle.rel_max_err(C.cpu().numpy(), rc) <= 1e-12
    assert oracle.rel_max_err(P.cpu().numpy(), rp) <= 1e-12
    u = torch.empty(U0.shape, dtype=torch.float32, device=U0.device)
    lo, d = torch.empty_like(u), torch.empty_like(u)
    w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, scheme, steps, f)
    out = torch.empty_like(U0)
    w.wave2d_f32c_export(u, lo, out)
    assert oracle.rel_max_err(out.cpu().numpy(), rc) <= 1e-5


@pytest.mark.parametrize("scheme", [w.P5, w.P9, w.P13])
@pytest.mark.parametrize("depth", [1, 2, 3, 4, 6, 8])
def test_periodic_stream_equals_simple(scheme, depth):
    for (nx, ny) in [(260, 131), (128, 9), (6, 40), (64, 64)]:
        u0, v0 = rough_data(nx, ny, nx + ny)
        h = 1.0 / max(nx, ny)
        tau = 0.9 * w.wave2d_lambda_max(scheme) * h
        U0, V0 = dev_grid(u0), dev_grid(v0)
        for rows in (8, 13):
            outs = []
            for simple in (True, False):
                fl = w.PERIODIC | (w.KERNEL_SIMPLE if simple else 0)
                if not simple:
                    w.wave2d_set_tuning(w.F64, scheme, depth, rows)
                    w.wave2d_set_tuning(w.F32C, scheme, depth, rows)
                P, C = torch.empty_like(U0), torch.empty_like(U0)
                w.wave2d_run(U0, V0, P, C, h, tau, 1.0, scheme, 2 * depth + 3, fl)
                u = torch.empty(U0.shape, dtype=torch.float32, device=U0.device)
                lo, d = torch.empty_like(u), torch.empty_like(u)
                w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, scheme, 2 * depth + 3, fl)
                outs.append((P.clone(), C.clone(), u.clone(), lo.clone(), d.clone()))
            for a, b in zip(outs[0], outs[1]):
                assert torch.equal(a, b), (nx, ny, rows)


def test_periodic_batch_equals_solo_and_odd_width_rejected():
    dev = torch.device("cuda:0")
    insts = []
    for k, (nx, ny, scheme, steps) in enumerate([(64, 64, w.P9, 21), (130, 70, w.P13, 17), (8, 40, w.P5, 9)]):
        u0, v0 = _periodic_data(nx, ny, k)
        h = 1.0 / max(nx, ny)
        tau = 0.8 * w.wave2d_lambda_max(scheme) * h
        u = torch.empty((ny, nx), dtype=torch.float32, device=dev)
        insts.append(dict(nx=nx, ny=ny, h=h, tau=tau, c=1.0, scheme=scheme, steps=steps, flags=w.PERIODIC,
                          u0=dev_grid(u0), v0=dev_grid(v0), u=u, lo=torch.empty_like(u), d=torch.empty_like(u)))
    b = w.wave2d_batch_create(insts)
    try:
        w.wave2d_batch_run(b)
        torch.cuda.synchronize()
    finally:
        w.wave2d_batch_destroy(b)
    for t in insts:
        u = torch.empty_like(t["u"])
        lo, d = torch.empty_like(u), torch.empty_like(u)
        w.wave2d_f32c_run(t["u0"], t["v0"], u, lo, d, t["h"], t["tau"], 1.0, t["scheme"], t["steps"], w.PERIODIC)
        assert torch.equal(t["u"], u) and torch.equal(t["lo"], lo) and torch.equal(t["d"], d)
    odd = dict(insts[0])
    u0, v0 = _periodic_data(33, 20, 7)
    odd.update(nx=33, ny=20, u0=dev_grid(u0), v0=dev_grid(v0))
    odd["u"] = torch.empty((20, 33), dtype=torch.float32, device=dev)
    odd["lo"], odd["d"] = torch.empty_like(odd["u"]), torch.empty_like(odd["u"])
    with pytest.raises(w.Wave2dError):
        w.wave2d_batch_create([odd])

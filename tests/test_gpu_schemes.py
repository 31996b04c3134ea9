"""GPU runs of schemes built from a stencil and a monomial set (Sec. 4-5).

The "cross" scheme (centre and axis nodes at distance 1 and 2; monomials 1,
x^k, y^k for k <= 4) is a 13-point-class scheme with no diagonal weights.
The library builds its weights with its own construction, the oracle with
the exact rational one; the runs are compared like the paper's schemes:
FP64 to 1e-12 and compensated FP32 to 1e-5 of max|u|, on both boundary
rules; the temporally blocked kernels are bitwise equal to the
one-node-per-thread kernels; batches equal solo runs.  The paper's own
13-point set built at run time reproduces the built-in 13-point scheme.
"""
import time

import numpy as np
import pytest
import torch

import oracle
import paper_1904_04048_amd as w
from oracle import derive
from tests.gpu_util import dev_grid, rough_data

pytestmark = pytest.mark.gpu

C0 = [(0, 0)]
AX1 = [(1, 0), (-1, 0), (0, 1), (0, -1)]
AX2 = [(2, 0), (-2, 0), (0, 2), (0, -2)]
CROSS_NODES = C0 + AX1 + AX2
CROSS_EXPS = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (3, 0), (0, 3), (4, 0), (0, 4)]
ORC_CROSS = 1000


@pytest.fixture(scope="module")
def cross():
    oracle.register_scheme(ORC_CROSS, derive.node_weights_for(CROSS_NODES, CROSS_EXPS))
    return w.wave2d_scheme_create(CROSS_NODES, CROSS_EXPS)


@pytest.fixture(autouse=True)
def _reset_tuning(cross):
    yield
    for p in (w.F64, w.F32C):
        for s in (w.P5, w.P9, w.P13, w.C9):
            w.wave2d_set_tuning(p, s)


@pytest.mark.parametrize("shape", [(5, 5), (19, 7), (67, 131), (200, 129), (131, 300)], ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("periodic", [False, True], ids=["dirichlet", "periodic"])
@pytest.mark.parametrize("conv", [False, True], ids=["poisson", "conventional"])
def test_cross_scheme_matches_oracle(cross, shape, periodic, conv):
    nx, ny = shape
    u0, v0 = rough_data(nx, ny, nx * 7 + ny)
    h = 1.0 / max(nx, ny)
    tau = 0.95 * w.wave2d_lambda_max(cross) * h
    steps = 23
    f = (w.PERIODIC if periodic else 0) | (w.FIRST_CONVENTIONAL if conv else 0)
    of = (oracle.PERIODIC if periodic else 0) | (oracle.FIRST_CONVENTIONAL if conv else 0)
    rp, rc = oracle.run(u0, v0, h, tau, 1.0, ORC_CROSS, steps, of)
    U0, V0 = dev_grid(u0), dev_grid(v0)
    P, C = torch.empty_like(U0), torch.empty_like(U0)
    w.wave2d_run(U0, V0, P, C, h, tau, 1.0, cross, steps, f)
    assert oracle.rel_max_err(C.cpu().numpy(), rc) <= 1e-12
    assert oracle.rel_max_err(P.cpu().numpy(), rp) <= 1e-12
    u = torch.empty(U0.shape, dtype=torch.float32, device=U0.device)
    lo, d = torch.empty_like(u), torch.empty_like(u)
    w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, cross, steps, f)
    out = torch.empty_like(U0)
    w.wave2d_f32c_export(u, lo, out)
    assert oracle.rel_max_err(out.cpu().numpy(), rc) <= 1e-5


@pytest.mark.parametrize("depth", [1, 2, 3, 4, 6, 8])
def test_cross_scheme_stream_equals_simple(cross, depth):
    for (nx, ny) in [(260, 131), (131, 70), (64, 64)]:
        u0, v0 = rough_data(nx, ny, nx + 3 * ny)
        h = 1.0 / max(nx, ny)
        tau = 0.9 * w.wave2d_lambda_max(cross) * h
        U0, V0 = dev_grid(u0), dev_grid(v0)
        for rows in (8, 13):
            outs = []
            for simple in (True, False):
                fl = w.KERNEL_SIMPLE if simple else 0
                if not simple:
                    w.wave2d_set_tuning(w.F64, cross, depth, rows)
                    w.wave2d_set_tuning(w.F32C, cross, depth, rows)
                P, C = torch.empty_like(U0), torch.empty_like(U0)
                w.wave2d_run(U0, V0, P, C, h, tau, 1.0, cross, 2 * depth + 5, fl)
                u = torch.empty(U0.shape, dtype=torch.float32, device=U0.device)
                lo, d = torch.empty_like(u), torch.empty_like(u)
                w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, cross, 2 * depth + 5, fl)
                outs.append((P.clone(), C.clone(), u.clone(), lo.clone(), d.clone()))
            for a, b in zip(outs[0], outs[1]):
                assert torch.equal(a, b), (nx, ny, rows, depth)


def test_cross_scheme_in_batch(cross):
    dev = torch.device("cuda:0")
    insts = []
    for k, (nx, ny, scheme, steps) in enumerate([(300, 257, cross, 31), (129, 64, w.P9, 17), (70, 90, cross, 9)]):
        u0, v0 = rough_data(nx, ny, 11 + k)
        h = 1.0 / max(nx, ny)
        tau = 0.8 * w.wave2d_lambda_max(scheme) * h
        u = torch.empty((ny, nx), dtype=torch.float32, device=dev)
        insts.append(dict(nx=nx, ny=ny, h=h, tau=tau, c=1.0, scheme=scheme, steps=steps, flags=0,
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
        w.wave2d_f32c_run(t["u0"], t["v0"], u, lo, d, t["h"], t["tau"], 1.0, t["scheme"], t["steps"])
        assert torch.equal(t["u"], u) and torch.equal(t["lo"], lo) and torch.equal(t["d"], d)


def test_paper_13_point_set_built_at_run_time():
    sid = w.wave2d_scheme_create(derive.stencil(15), derive.monomials(15))
    nx, ny = 140, 97
    u0, v0 = rough_data(nx, ny, 5)
    h = 1.0 / 139
    tau = 0.9 * w.wave2d_lambda_max(w.P13) * h
    U0, V0 = dev_grid(u0), dev_grid(v0)
    out = []
    for s in (w.P13, sid):
        P, C = torch.empty_like(U0), torch.empty_like(U0)
        w.wave2d_run(U0, V0, P, C, h, tau, 1.0, s, 40)
        out.append(C.cpu().numpy())
    assert oracle.rel_max_err(out[1], out[0]) <= 1e-13


def test_cross_scheme_served(cross):
    # Served requests of a built scheme equal the same solve run alone.
    sv = w.wave2d_server_create(256 << 20)
    try:
        items = []
        for k, (nx, ny, steps, periodic) in enumerate([(200, 150, 41, False), (64, 96, 9, True), (131, 77, 25, False)]):
            u0, v0 = rough_data(nx, ny, 40 + k)
            U0, V0 = dev_grid(u0), dev_grid(v0)
            h = 1.0 / max(nx, ny)
            tau = 0.9 * w.wave2d_lambda_max(cross) * h
            f = w.PERIODIC if periodic else 0
            rid = w.wave2d_server_submit(sv, nx, ny, h, tau, 1.0, cross, steps, f, u0=U0, v0=V0)
            items.append((rid, U0, V0, h, tau, steps, f))
        for rid, U0, V0, h, tau, steps, f in items:
            t0 = time.time()
            r = None
            while r is None:
                r = w.wave2d_server_poll(sv, rid)
                assert time.time() - t0 < 60
                time.sleep(0.001)
            assert r["status"] == 0
            u = torch.empty(U0.shape, dtype=torch.float32, device="cuda")
            lo, d = torch.empty_like(u), torch.empty_like(u)
            w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, cross, steps, f)
            out = torch.empty_like(U0)
            w.wave2d_f32c_export(u, lo, out)
            assert torch.equal(w.result_tensor(r), out)
            w.wave2d_server_release(sv, rid)
    finally:
        w.wave2d_server_destroy(sv)

"""GPU tests of the request server.

Each served result must equal the same solve run alone (compensated FP32,
exported to FP64), bit for bit, whatever else was in flight; requests that
do not fit wait for memory; impossible requests are rejected; released
results return their memory.
"""
import time

import numpy as np
import pytest
import torch

import oracle
import paper_1904_04048_amd as w
from tests.gpu_util import smooth_data

pytestmark = pytest.mark.gpu


def _solo(u0, v0, h, tau, scheme, steps, flags=0):
    u = torch.empty(u0.shape, dtype=torch.float32, device="cuda")
    lo, d = torch.empty_like(u), torch.empty_like(u)
    w.wave2d_f32c_run(u0, v0, u, lo, d, h, tau, 1.0, scheme, steps, flags)
    out = torch.empty_like(u0)
    w.wave2d_f32c_export(u, lo, out)
    return out


def _wait(sv, ids, timeout=60.0):
    res = {}
    t0 = time.time()
    while len(res) < len(ids):
        for i in ids:
            if i not in res:
                r = w.wave2d_server_poll(sv, i)
                if r is not None:
                    res[i] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(res)} of {len(ids)} requests done")
        time.sleep(0.001)
    return res


SPECS = [  # (nx, ny, scheme, steps, lambda fraction, flags)
    (64, 64, w.P5, 40, 0.9, 0), (257, 129, w.P9, 130, 0.9, 0), (131, 300, w.P13, 77, 0.8, 0),
    (400, 400, w.P9, 13, 0.5, w.FIRST_CONVENTIONAL), (90, 70, w.C9, 55, 0.7, w.FIRST_CONVENTIONAL),
    (513, 257, w.P5, 1, 0.9, 0), (700, 333, w.P13, 23, 0.9, 0), (33, 45, w.P9, 200, 0.95, 0),
]


def _submit_all(sv, seed=0, with_modes=True):
    items = []
    for k, (nx, ny, scheme, steps, frac, flags) in enumerate(SPECS):
        h = 1.0 / (max(nx, ny) - 1)
        tau = frac * w.wave2d_lambda_max(scheme) * h
        if with_modes and k % 2 == 0:
            rng = np.random.default_rng(seed + k)
            modes = [(p, q, float(rng.standard_normal()) / (p * p + q * q), float(rng.standard_normal()))
                     for p, q in ((1, 1), (2, 3), (3, 1))]
            U0 = torch.empty((ny, nx), dtype=torch.float64, device="cuda")
            V0 = torch.empty_like(U0)
            w.wave2d_sine_series(U0, V0, modes)  # the same sampling the server does
            rid = w.wave2d_server_submit(sv, nx, ny, h, tau, 1.0, scheme, steps, flags, modes=modes)
        else:
            (u0, v0), _ = smooth_data(nx, ny, seed + k)
            U0, V0 = torch.from_numpy(u0).cuda(), torch.from_numpy(v0).cuda()
            rid = w.wave2d_server_submit(sv, nx, ny, h, tau, 1.0, scheme, steps, flags, u0=U0, v0=V0)
        items.append((rid, U0, V0, h, tau, scheme, steps, flags))
    return items


@pytest.mark.parametrize("budget_mb", [1024, 24])
def test_served_results_equal_solo(budget_mb):
    sv = w.wave2d_server_create(budget_mb << 20)
    try:
        items = _submit_all(sv)
        res = _wait(sv, [it[0] for it in items])
        for (rid, U0, V0, h, tau, scheme, steps, flags) in items:
            r = res[rid]
            assert r["status"] == 0
            assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
            got = w.result_tensor(r)
            ref = _solo(U0, V0, h, tau, scheme, steps, flags)
            assert torch.equal(got, ref), (rid, scheme, steps)
        st = w.wave2d_server_stats_get(sv)
        assert st["completed"] == len(SPECS) and st["failed"] == 0
        for it in items:
            w.wave2d_server_release(sv, it[0])
        st = w.wave2d_server_stats_get(sv)
        assert st["bytes_in_use"] == 0
    finally:
        w.wave2d_server_destroy(sv)


def test_served_accuracy_against_oracle():
    sv = w.wave2d_server_create(512 << 20)
    try:
        nx, ny, scheme, steps = 201, 151, w.P9, 300
        (u0, v0), _ = smooth_data(nx, ny, 42)
        h = 1.0 / 200
        tau = 0.9 * w.wave2d_lambda_max(scheme) * h
        U0, V0 = torch.from_numpy(u0).cuda(), torch.from_numpy(v0).cuda()
        rid = w.wave2d_server_submit(sv, nx, ny, h, tau, 1.0, scheme, steps, u0=U0, v0=V0)
        r = _wait(sv, [rid])[rid]
        got = w.result_tensor(r).cpu().numpy()
        _, ref = oracle.run(u0, v0, h, tau, 1.0, scheme, steps)
        assert oracle.rel_max_err(got, ref) <= 1e-5
    finally:
        w.wave2d_server_destroy(sv)


def test_server_rejects():
    sv = w.wave2d_server_create(8 << 20)
    try:
        with pytest.raises(w.Wave2dError):   # never fits in 8 MiB
            w.wave2d_server_submit(sv, 1025, 1025, 1e-3, 5e-4, 1.0, w.P9, 10, modes=[(1, 1, 1.0, 0.0)])
        with pytest.raises(w.Wave2dError):   # unstable
            w.wave2d_server_submit(sv, 65, 65, 1.0 / 64, 1.0 / 64, 1.0, w.P9, 10, modes=[(1, 1, 1.0, 0.0)])
        with pytest.raises(w.Wave2dError):   # no initial data
            w.wave2d_server_submit(sv, 65, 65, 1.0 / 64, 0.5 / 64, 1.0, w.P9, 10)
        with pytest.raises(w.Wave2dError):
            w.wave2d_server_poll(sv, 12345)
    finally:
        w.wave2d_server_destroy(sv)

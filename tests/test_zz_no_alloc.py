"""The allocation-free entry point (wave2d_f32c_step_noalloc) against the
existing wave2d_f32c_step, bit for bit, through the C ABI.

Two calls in a row on one device (the second on a smaller grid, so the
fixed array keeps the first call's contents when the second starts), odd and
even step counts (the odd pass count ends with a copy out of the array),
every stencil class, and the size limit.
"""
import pytest
import torch

import paper_1904_04048_amd as w
from tests.gpu_util import dev_grid, empty_like_grid, smooth_data

pytestmark = pytest.mark.gpu


def _state(nx, ny, ld, scheme, seed, steps=5):
    (u0, v0), _ = smooth_data(nx, ny, seed)
    h = 1.0 / (max(nx, ny) - 1)
    tau = 0.9 * w.wave2d_lambda_max(scheme) * h
    U0, V0 = dev_grid(u0, ld), dev_grid(v0, ld)
    u = empty_like_grid(U0, torch.float32)
    lo, d = empty_like_grid(U0, torch.float32), empty_like_grid(U0, torch.float32)
    w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, scheme, steps)
    return (u, lo, d), h, tau


def _clone(st):
    out = []
    for t in st:
        c = empty_like_grid(t)
        c.copy_(t)
        out.append(c)
    return out


@pytest.mark.parametrize("scheme", [w.P5, w.P9, w.P13])
def test_noalloc_equals_f32c_step_two_calls(scheme):
    # First call on the larger grid, then on a smaller one.
    cases = [(1031, 777, 1040, 37), (300, 257, 300, 20)]
    for k, (nx, ny, ld, steps) in enumerate(cases):
        st, h, tau = _state(nx, ny, ld, scheme, 100 + k)
        a = _clone(st)
        b = _clone(st)
        print(f"noalloc scheme {scheme} grid {nx}x{ny} ld {ld} steps {steps}", flush=True)
        w.wave2d_f32c_step(a[0], a[1], a[2], h, tau, 1.0, scheme, steps)
        w.wave2d_f32c_step_noalloc(b[0], b[1], b[2], h, tau, 1.0, scheme, steps)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.isfinite(y).all()
            assert torch.equal(x, y)


def test_noalloc_odd_pass_count_and_zero_steps():
    st, h, tau = _state(517, 263, 517, w.P9, 7)
    for steps in (0, 1, 3, 9, 17):
        a = _clone(st)
        b = _clone(st)
        w.wave2d_f32c_step(a[0], a[1], a[2], h, tau, 1.0, w.P9, steps)
        w.wave2d_f32c_step_noalloc(b[0], b[1], b[2], h, tau, 1.0, w.P9, steps)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.equal(x, y), steps


def test_noalloc_periodic_matches():
    st, h, tau = _state(256, 130, 256, w.P13, 9)
    a = _clone(st)
    b = _clone(st)
    w.wave2d_f32c_step(a[0], a[1], a[2], h, tau, 1.0, w.P13, 14, w.PERIODIC)
    w.wave2d_f32c_step_noalloc(b[0], b[1], b[2], h, tau, 1.0, w.P13, 14, w.PERIODIC)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_noalloc_rejects_grids_beyond_the_array():
    # 2400^2 needs 3 x 23.04 MB > 64 MiB: rejected before anything is enqueued.
    n = 2400
    assert w.wave2d_work_bytes(w.F32C, n, n) > w.NOALLOC_MAX_BYTES
    u = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    lo, d = torch.zeros_like(u), torch.zeros_like(u)
    with pytest.raises(w.Wave2dError) as ei:
        w.wave2d_f32c_step_noalloc(u, lo, d, 1.0 / (n - 1), 0.5 / (n - 1), 1.0, w.P9, 4)
    assert ei.value.status == -1  # WAVE2D_EINVAL
    assert not u.any() and not lo.any() and not d.any()
    # The largest square grid that fits still runs.
    m = 2364
    assert w.wave2d_work_bytes(w.F32C, m, m) <= w.NOALLOC_MAX_BYTES
    st, h, tau = _state(m, m, m, w.P9, 3, steps=2)
    a = _clone(st)
    b = _clone(st)
    w.wave2d_f32c_step(a[0], a[1], a[2], h, tau, 1.0, w.P9, 8)
    w.wave2d_f32c_step_noalloc(b[0], b[1], b[2], h, tau, 1.0, w.P9, 8)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)

"""wave2d for MI355X: the Poisson-formula explicit schemes for the 2D wave
equation (Khutoryansky, arXiv:1904.04048) as hand-written gfx950 kernels
behind a C ABI (include/wave2d.h).

This module is the thin Python binding: each function has the name of the C
entry point it calls and only marshals arguments.  Grids are torch tensors
on the GPU of shape (ny, nx) with unit stride along x; the row stride is
passed as the leading dimension.  Work is enqueued on the current torch
stream of the tensors' device.

Importing the package does not load the library; the first call does, and
fails loudly if libwave2d.so has not been built.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (ALLOW_UNSTABLE, BATCH_GRAPH, BATCH_ROUNDS, C9, F32C, F64, FIRST_CONVENTIONAL, KERNEL_SIMPLE, NOALLOC_MAX_BYTES, P5,
                   P9, P13, PERIODIC, BatchStats, Instance, Request, Result, ServerStats, Tuning, Wave2dError)

__all__ = [
    "P5", "P9", "P13", "C9", "F64", "F32C", "FIRST_CONVENTIONAL", "ALLOW_UNSTABLE", "KERNEL_SIMPLE", "PERIODIC",
    "Wave2dError", "wave2d_lambda_max", "wave2d_weights", "wave2d_class_weights", "CLASSES", "wave2d_work_bytes", "wave2d_first_step",
    "wave2d_step", "wave2d_run", "wave2d_f32c_init", "wave2d_f32c_step", "wave2d_f32c_step_noalloc",
    "NOALLOC_MAX_BYTES", "wave2d_f32c_export",
    "wave2d_f32c_run", "wave2d_norms", "wave2d_f32c_norms", "wave2d_set_tuning", "wave2d_get_tuning",
    "wave2d_release", "wave2d_autotune", "wave2d_batch_create", "wave2d_batch_run", "wave2d_batch_stats_get", "wave2d_batch_autotune",
    "wave2d_batch_set_rows_cap", "wave2d_batch_destroy", "BATCH_GRAPH", "BATCH_ROUNDS", "wave2d_sine_series", "wave2d_server_create", "wave2d_server_submit",
    "wave2d_server_poll", "wave2d_server_release", "wave2d_server_stats_get", "wave2d_server_destroy",
]


def _grid(*tensors, dtypes):
    import torch
    t0 = tensors[0]
    ny, nx = t0.shape
    ld = t0.stride(0)
    dev = t0.device
    for t, dt in zip(tensors, dtypes):
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("grids must be GPU tensors")
        if t.dtype != dt:
            raise ValueError(f"expected {dt}, got {t.dtype}")
        if t.dim() != 2 or tuple(t.shape) != (ny, nx):
            raise ValueError("all grids must have the same shape (ny, nx)")
        if t.stride(1) != 1 or t.stride(0) != ld:
            raise ValueError("grids need unit x stride and a common row stride")
        if t.device != dev:
            raise ValueError("grids on different devices")
    stream = torch.cuda.current_stream(dev).cuda_stream
    return nx, ny, ld, ctypes.c_void_p(stream)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _work(work):
    if work is None:
        return ctypes.c_void_p(0), 0
    return ctypes.c_void_p(work.data_ptr()), work.numel() * work.element_size()


def wave2d_lambda_max(scheme: int) -> float:
    v = _lib.load().wave2d_lambda_max(scheme)
    if v < 0:
        raise ValueError(f"unknown scheme {scheme}")
    return v


def wave2d_scheme_create(nodes, exps) -> int:
    """Scheme id built from m stencil nodes (q1, q2) and m monomial
    exponents (a1, a2) (Sec. 4-5)."""
    nodes = [int(v) for q in nodes for v in q]
    exps = [int(v) for e in exps for v in e]
    if len(nodes) != len(exps):
        raise ValueError("nodes and exps must have the same length")
    m = len(nodes) // 2
    nb = (ctypes.c_int32 * max(1, 2 * m))(*nodes)
    eb = (ctypes.c_int32 * max(1, 2 * m))(*exps)
    sid = ctypes.c_int(0)
    _lib.check(_lib.load().wave2d_scheme_create(m, nb, eb, ctypes.byref(sid)))
    return sid.value


def wave2d_weights(scheme: int, lam: float, flags: int = 0):
    """(w2, wa, wb): two-step weights and first-step A / (B/tau) node weights."""
    w2, wa, wb = (ctypes.c_double * 3)(), (ctypes.c_double * 3)(), (ctypes.c_double * 3)()
    _lib.check(_lib.load().wave2d_weights(scheme, flags, lam, w2, wa, wb))
    return list(w2), list(wa), list(wb)


CLASSES = ((1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1), (3, 2), (3, 3))


def wave2d_class_weights(scheme: int, lam: float, flags: int = 0, nclass: int = 9):
    """(w2, wa, wb) for the first nclass node classes of CLASSES."""
    w2, wa, wb = (ctypes.c_double * nclass)(), (ctypes.c_double * nclass)(), (ctypes.c_double * nclass)()
    _lib.check(_lib.load().wave2d_class_weights(scheme, flags, lam, nclass, w2, wa, wb))
    return list(w2), list(wa), list(wb)


def wave2d_work_bytes(precision: int, nx: int, ny: int, ld: int | None = None) -> int:
    return int(_lib.load().wave2d_work_bytes(precision, nx, ny, nx if ld is None else ld))


def wave2d_first_step(u0, v0, u1, h, tau, c, scheme, flags=0):
    import torch
    nx, ny, ld, s = _grid(u0, v0, u1, dtypes=(torch.float64,) * 3)
    _lib.check(_lib.load().wave2d_first_step(nx, ny, ld, h, tau, c, scheme, flags, _p(u0), _p(v0), _p(u1), s))


def wave2d_step(u_prev, u_cur, h, tau, c, scheme, steps, flags=0, work=None):
    import torch
    nx, ny, ld, s = _grid(u_prev, u_cur, dtypes=(torch.float64,) * 2)
    wp, wb = _work(work)
    _lib.check(_lib.load().wave2d_step(nx, ny, ld, h, tau, c, scheme, flags, steps, _p(u_prev), _p(u_cur),
                                       wp, wb, s))


def wave2d_run(u0, v0, u_prev_out, u_out, h, tau, c, scheme, steps, flags=0, work=None):
    import torch
    nx, ny, ld, s = _grid(u0, v0, u_prev_out, u_out, dtypes=(torch.float64,) * 4)
    wp, wb = _work(work)
    _lib.check(_lib.load().wave2d_run(nx, ny, ld, h, tau, c, scheme, flags, steps, _p(u0), _p(v0),
                                      _p(u_prev_out), _p(u_out), wp, wb, s))


def wave2d_f32c_init(u_prev, u_cur, u, lo, d):
    import torch
    nx, ny, ld, s = _grid(u_prev, u_cur, u, lo, d, dtypes=(torch.float64,) * 2 + (torch.float32,) * 3)
    _lib.check(_lib.load().wave2d_f32c_init(nx, ny, ld, _p(u_prev), _p(u_cur), _p(u), _p(lo), _p(d), s))


def wave2d_f32c_step(u, lo, d, h, tau, c, scheme, steps, flags=0, work=None):
    import torch
    nx, ny, ld, s = _grid(u, lo, d, dtypes=(torch.float32,) * 3)
    wp, wb = _work(work)
    _lib.check(_lib.load().wave2d_f32c_step(nx, ny, ld, h, tau, c, scheme, flags, steps, _p(u), _p(lo), _p(d),
                                            wp, wb, s))


def wave2d_f32c_step_noalloc(u, lo, d, h, tau, c, scheme, steps, flags=0):
    """wave2d_f32c_step with the second state in the library's fixed device
    array (no allocation; grids up to NOALLOC_MAX_BYTES of workspace)."""
    import torch
    nx, ny, ld, s = _grid(u, lo, d, dtypes=(torch.float32,) * 3)
    _lib.check(_lib.load().wave2d_f32c_step_noalloc(nx, ny, ld, h, tau, c, scheme, flags, steps, _p(u), _p(lo),
                                                    _p(d), s))


def wave2d_f32c_export(u, lo, out):
    import torch
    nx, ny, ld, s = _grid(u, lo, out, dtypes=(torch.float32, torch.float32, torch.float64))
    _lib.check(_lib.load().wave2d_f32c_export(nx, ny, ld, _p(u), _p(lo), _p(out), s))


def wave2d_f32c_run(u0, v0, u, lo, d, h, tau, c, scheme, steps, flags=0, work=None):
    import torch
    nx, ny, ld, s = _grid(u0, v0, u, lo, d, dtypes=(torch.float64,) * 2 + (torch.float32,) * 3)
    wp, wb = _work(work)
    _lib.check(_lib.load().wave2d_f32c_run(nx, ny, ld, h, tau, c, scheme, flags, steps, _p(u0), _p(v0), _p(u),
                                           _p(lo), _p(d), wp, wb, s))


def wave2d_norms(a, b):
    """[max|a-b|, max|b|, sum (a-b)^2, sum b^2] (synchronous)."""
    import torch
    nx, ny, ld, s = _grid(a, b, dtypes=(torch.float64,) * 2)
    out = (ctypes.c_double * 4)()
    _lib.check(_lib.load().wave2d_norms(nx, ny, ld, _p(a), _p(b), out, s))
    return list(out)


def wave2d_f32c_norms(u, lo, b):
    import torch
    nx, ny, ld, s = _grid(u, lo, b, dtypes=(torch.float32, torch.float32, torch.float64))
    out = (ctypes.c_double * 4)()
    _lib.check(_lib.load().wave2d_f32c_norms(nx, ny, ld, _p(u), _p(lo), _p(b), out, s))
    return list(out)


def wave2d_set_tuning(precision: int, scheme: int, depth: int | None = None, rows: int | None = None):
    """Override the launch shape for (precision, scheme); no arguments resets it."""
    L = _lib.load()
    if depth is None:
        _lib.check(L.wave2d_set_tuning(precision, scheme, None))
        return
    t = Tuning(depth, rows if rows is not None else 64)
    _lib.check(L.wave2d_set_tuning(precision, scheme, ctypes.byref(t)))


def wave2d_get_tuning(precision: int, scheme: int, nx: int = 0, ny: int = 0):
    t = Tuning()
    _lib.check(_lib.load().wave2d_get_tuning(precision, scheme, nx, ny, ctypes.byref(t)))
    return t.depth, t.rows


def wave2d_release():
    _lib.check(_lib.load().wave2d_release())


def wave2d_autotune(precision: int, scheme: int, nx: int, ny: int):
    """Time every register-resident launch shape on an nx x ny grid, select
    the fastest for this process and return (depth, rows)."""
    import torch
    t = Tuning()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(_lib.load().wave2d_autotune(precision, scheme, nx, ny, s, ctypes.byref(t)))
    return t.depth, t.rows


def wave2d_batch_create(instances, flags: int = 0):
    """instances: list of dicts with keys nx, ny, ld, h, tau, c, scheme, flags,
    steps and tensors u0, v0 (float64) and u, lo, d (float32).  Returns an
    opaque handle (keep the tensors alive while the batch exists)."""
    arr = (Instance * len(instances))()
    for k, it in enumerate(instances):
        u0 = it["u0"]
        ny, nx = u0.shape
        arr[k] = Instance(nx, ny, u0.stride(0), it["h"], it["tau"], it.get("c", 1.0), it["scheme"],
                          it.get("flags", 0), it["steps"], u0.data_ptr(), it["v0"].data_ptr(),
                          it["u"].data_ptr(), it["lo"].data_ptr(), it["d"].data_ptr())
    h = ctypes.c_void_p()
    _lib.check(_lib.load().wave2d_batch_create(arr, len(instances), flags, ctypes.byref(h)))
    return h


def wave2d_batch_run(batch):
    import torch
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(_lib.load().wave2d_batch_run(batch, s))


def wave2d_batch_stats_get(batch):
    st = BatchStats()
    _lib.check(_lib.load().wave2d_batch_stats_get(batch, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in BatchStats._fields_}


def wave2d_batch_autotune(batch):
    """Time the batch with each candidate segment cap; keep and return the fastest."""
    import torch
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    cap = ctypes.c_int32(0)
    _lib.check(_lib.load().wave2d_batch_autotune(batch, s, ctypes.byref(cap)))
    return cap.value


def wave2d_batch_set_rows_cap(batch, rows_cap):
    """Re-plan the batch's persistent items for segments of at most rows_cap rows."""
    import torch
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(_lib.load().wave2d_batch_set_rows_cap(batch, rows_cap, s))


def wave2d_batch_destroy(batch):
    _lib.check(_lib.load().wave2d_batch_destroy(batch))


def wave2d_sine_series(u0, v0, modes):
    """Sample u0, v0 (float64 GPU grids) from modes [(p, q, A, B), ...] on the device."""
    import torch
    nx, ny, ld, s = _grid(u0, v0, dtypes=(torch.float64,) * 2)
    arr = (ctypes.c_double * (4 * len(modes)))(*[float(v) for m in modes for v in m])
    _lib.check(_lib.load().wave2d_sine_series(nx, ny, ld, len(modes), arr, _p(u0), _p(v0), s))


def wave2d_server_create(mem_budget: int = 0, flags: int = 0):
    h = ctypes.c_void_p()
    _lib.check(_lib.load().wave2d_server_create(mem_budget, flags, ctypes.byref(h)))
    return h


def wave2d_server_submit(server, nx, ny, h, tau, c, scheme, steps, flags=0, modes=None, u0=None, v0=None):
    """Queue a request; initial data as sine modes [(p, q, A, B), ...] or as
    GPU float64 grids u0, v0 (kept alive by the caller until completion)."""
    rq = Request(nx, ny, h, tau, c, scheme, flags, steps, 0, None, None, None)
    keep = None
    if modes:
        keep = (ctypes.c_double * (4 * len(modes)))(*[float(v) for m in modes for v in m])
        rq.nmodes = len(modes)
        rq.modes = ctypes.cast(keep, ctypes.c_void_p)
    else:
        rq.u0 = u0.data_ptr() if u0 is not None else None
        rq.v0 = v0.data_ptr() if v0 is not None else None
        if u0 is not None or v0 is not None:
            # The server reads the grids on its own stream: work queued on
            # this one that writes them must be complete first.
            import torch
            torch.cuda.current_stream().synchronize()
    rid = ctypes.c_uint64()
    _lib.check(_lib.load().wave2d_server_submit(server, ctypes.byref(rq), ctypes.byref(rid)))
    return rid.value


def wave2d_server_poll(server, rid):
    """None while the request is queued or running, else a dict."""
    r = Result()
    st = _lib.load().wave2d_server_poll(server, rid, ctypes.byref(r))
    if st == _lib.EBUSY:
        return None
    _lib.check(st)
    return {k: getattr(r, k) for k, _ in Result._fields_}


def wave2d_server_release(server, rid):
    _lib.check(_lib.load().wave2d_server_release(server, rid))


def wave2d_server_stats_get(server):
    s = ServerStats()
    _lib.check(_lib.load().wave2d_server_stats_get(server, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in ServerStats._fields_}


def wave2d_server_destroy(server):
    _lib.check(_lib.load().wave2d_server_destroy(server))


def result_tensor(res):
    """View a served FP64 result (device pointer owned by the server until
    release) as a torch tensor copy."""
    import torch
    n = res["ld"] * res["ny"]
    buf = torch.empty(n, dtype=torch.float64, device="cuda")
    _lib.load()
    import ctypes as C
    hip = C.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    rc = hip.hipMemcpy(C.c_void_p(buf.data_ptr()), C.c_void_p(res["u"]), n * 8, 3)  # device to device
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
    return buf.view(res["ny"], res["ld"])[:, :res["nx"]]

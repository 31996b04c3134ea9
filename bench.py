"""Benchmark of the wave2d hot path on one MI355X.

One step = one run of the batched workload: 512 seeded instances (sides
log-uniform in [64, 2048] nodes, schemes uniform over the 5-, 9- and
13-point schemes, Courant numbers in [0.3, 0.9] of each scheme's limit,
100-2000 levels, 8 random sine modes of initial data), each solved in the
compensated-FP32 form from its FP64 first step: first steps, remainder
passes, one persistent launch per stencil class for all full passes, final
copies (about 15 launches, enqueued eagerly so that HIP events bracket the
persistent launches; the same batch replayed as one captured graph is
reported beside it).  Inputs are resident on the GPU before the timed
region.  The same JSON line carries the single-grid workloads (9-point
4097^2, 13-point 8193^2 Gaussian pulse, 5-point 257^2 FP64 standing wave,
an untabulated 6001^2 grid), the served workload (Poisson arrivals), errors
against the FP64 oracle, and the oracle's own rate on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
    python bench.py --mode profile     # short run for rocprofv3 counter passes
    python bench.py --mode summarize   # write profiles/ from the rocprofv3 output
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid-point updates/s (GLUP/s) + % HBM roofline; served p50/p99 latency at fixed error"
HBM_PEAK_GBS = 8000.0
# Vector ALU issue available to these kernels: 256 CUs x 4 SIMDs x one wave64
# instruction per 4 cycles (16 lanes per cycle) x 2.4 GHz = 39.3e12 lane
# operations/s (78.6 TFLOP/s counting a fused multiply-add as two).  The
# published 157.3 TFLOP/s FP32 figure needs packed FP32 instructions, which
# the library is compiled not to emit.
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
STATE_BYTES_PER_NODE = 24  # compensated state (u, lo, d): 12 B read + 12 B written per node per pass
PROFILES = os.path.join(ROOT, "profiles")
XCDS = 8
BATCH_COUNTERS = os.path.join(PROFILES, "k_stream_persist_batch512_counters.md")
BATCH_STATS = os.path.join(PROFILES, "k_stream_persist_batch512_kernel_stats.md")
C2_COUNTERS = os.path.join(PROFILES, "k_stream_fused_f32c_9pt_4097_counters.md")
C3_COUNTERS = os.path.join(PROFILES, "k_stream_fused_f32c_13pt_8193_counters.md")
WIDE_COUNTERS = os.path.join(PROFILES, "k_wide_step_f32c_deg6_4097_counters.md")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", choices=["bench", "profile", "summarize"], default="bench")
    ap.add_argument("--prof-dir", default=os.path.join(ROOT, "gpurun_out"),
                    help="summarize: directory holding the rocprofv3 csv output")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serve", action="store_true", help="skip the served workload")
    ap.add_argument("--no-single", action="store_true", help="skip the single-grid workloads")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--kernel-launches", type=int, default=60)
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---- source hashes and committed counter records --------------------------------

def kernel_source_hash():
    """Hash of the sources the step kernels are built from: a counter record
    taken on other sources no longer describes the kernel."""
    import hashlib
    h = hashlib.sha256()
    for f in ("stream.hip", "point.h", "w2d.h"):
        h.update(open(os.path.join(ROOT, "paper_1904_04048_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def wide_source_hash():
    """Hash of the sources the wide-scheme kernels are built from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("wide.hip", "wide.h", "point.h", "w2d.h"):
        h.update(open(os.path.join(ROOT, "paper_1904_04048_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def counter_record(path):
    """The JSON record of a committed rocprofv3 counter summary, or None."""
    try:
        text = open(path).read()
        return json.loads(text.split("```json")[1].split("```")[0])
    except (OSError, ValueError, IndexError):
        return None


def traffic_record(path, kernel_cfg):
    """Measured HBM bytes per launch of a kernel from a committed counter
    summary, if it was taken on this kernel configuration and sources."""
    rec = counter_record(path)
    if rec is None or rec.get("kernel_cfg") != kernel_cfg:
        return None
    return rec.get("hbm_bytes_per_launch")


def roofline_hbm(alg_bytes, t_launch, lup, traffic, kernel, extra):
    """HBM roofline of one kernel: algorithmic bytes (the compensated state
    read and written once per pass) per launch over the launch time, against
    8 TB/s."""
    gbs = alg_bytes / t_launch / 1e9
    out = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
           "launch_us": round(t_launch * 1e6, 2), "bytes_per_launch": int(alg_bytes), "lup_per_launch": int(lup),
           "kernel_glups": round(lup / t_launch / 1e9, 1)}
    out.update(extra)
    return out


def alu_view(path):
    """The same kernel on the vector-ALU view, from its committed counters."""
    rec = counter_record(path) or {}
    return {"peak_lane_ops": round(VALU_LANE_OPS / 1e12, 1), "unit": "T lane-ops/s",
            "valu_issue_frac": rec.get("valu_issue_frac"), "lane_ops_per_lup": rec.get("lane_ops_per_lup")}


# ---- the batched workload (headline) ---------------------------------------------

def make_batch(dev, flags=0, host_data=False):
    """The 512 instances and their batch.  host_data: sample the initial data
    on the host and copy it over (no device kernels: the counter-collection
    runs keep their dispatch count small)."""
    import torch

    import paper_1904_04048_amd as w
    from paper_1904_04048_amd import workloads as W
    probs = W.c4()
    insts = []
    for pr in probs:
        if host_data:
            u0, v0 = W.sine_series_matmul(pr.nx, pr.ny, pr.modes)
            U0, V0 = torch.from_numpy(u0).to(dev), torch.from_numpy(v0).to(dev)
        else:
            U0, V0 = W.sine_series_torch(pr.nx, pr.ny, pr.modes, dev)
        u = torch.empty((pr.ny, pr.nx), dtype=torch.float32, device=dev)
        insts.append(dict(nx=pr.nx, ny=pr.ny, h=pr.h, tau=pr.tau, c=pr.c, scheme=pr.scheme, steps=pr.steps,
                          flags=0, u0=U0, v0=V0, u=u, lo=torch.empty_like(u), d=torch.empty_like(u)))
    return probs, insts, w.wave2d_batch_create(insts, flags)


def batch_errors(probs, insts, budget_s=20.0):
    """Errors of the batch's results against the FP64 oracle: the oracle's
    closed-form discrete solution of the sine-series data (any size) on every
    4th instance and on the 16 smallest-and-longest ones, and the full-grid C
    oracle on the 4 smallest-and-longest ones."""
    import oracle
    from oracle import modes as M
    from paper_1904_04048_amd import workloads as W
    hard = sorted(range(len(probs)), key=lambda k: (probs[k].nx, -probs[k].steps))[:16]
    sample = sorted(set(range(0, len(probs), 4)) | set(hard))
    worst_cf, worst_full, n_cf, n_full = 0.0, 0.0, 0, 0
    t0 = time.perf_counter()
    for k in sample:
        if time.perf_counter() - t0 > budget_s and k not in hard:
            continue
        pr, t = probs[k], insts[k]
        got = t["u"].double().cpu().numpy() + t["lo"].double().cpu().numpy()
        ref = M.solution(pr.modes, pr.nx, pr.ny, pr.h, pr.tau, pr.c, pr.scheme, pr.steps)
        worst_cf = max(worst_cf, oracle.rel_max_err(got, ref))
        n_cf += 1
        if k in hard[:4]:
            u0, v0 = W.sine_series(pr.nx, pr.ny, pr.modes)
            _, full = oracle.run(u0, v0, pr.h, pr.tau, pr.c, pr.scheme, pr.steps)
            worst_full = max(worst_full, oracle.rel_max_err(got, full))
            n_full += 1
    return {"max_rel_vs_oracle_closed_form": worst_cf, "instances_closed_form": n_cf,
            "max_rel_vs_oracle_full_grid": worst_full, "instances_full_grid": n_full,
            "sample": "closed form: every 4th instance and the 16 smallest-and-longest; "
                      "full-grid oracle: the 4 smallest-and-longest",
            "hardest": [{"side": probs[k].nx, "scheme": probs[k].scheme, "steps": probs[k].steps} for k in hard[:4]]}


def batch_bench(args, dev):
    import torch

    import paper_1904_04048_amd as w
    probs, insts, b = make_batch(dev)
    try:
        log("batch: autotune")
        cap = w.wave2d_batch_autotune(b)
        st = w.wave2d_batch_stats_get(b)
        for _ in range(max(1, args.warmup)):
            w.wave2d_batch_run(b)
        torch.cuda.synchronize()
        log("batch: timed")
        ms_persist = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            w.wave2d_batch_run(b)
            s2 = w.wave2d_batch_stats_get(b)  # waits for the run; reads its persistent-launch events
            ms_persist.append(s2["last_persistent_ms"])
            if s2["stalled_waits"]:
                raise RuntimeError(f"persistent launch: {s2['stalled_waits']} waits gave up")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        log("batch: errors")
        errs = batch_errors(probs, insts)
    finally:
        w.wave2d_batch_destroy(b)
    # The same batch replayed as one captured graph (not timed per launch).
    bg = w.wave2d_batch_create(insts, w.BATCH_GRAPH)
    try:
        w.wave2d_batch_set_rows_cap(bg, cap)
        w.wave2d_batch_run(bg)
        torch.cuda.synchronize()
        reps = max(2, min(5, args.steps))
        t0 = time.perf_counter()
        for _ in range(reps):
            w.wave2d_batch_run(bg)
        torch.cuda.synchronize()
        graph_glups = st["lup"] * reps / (time.perf_counter() - t0) / 1e9
    finally:
        w.wave2d_batch_destroy(bg)
    t_launch = sum(ms_persist) / len(ms_persist) / 1e3
    cfg = {"kernel": "k_stream_persist", "source": kernel_source_hash()}
    crec = counter_record(BATCH_COUNTERS) or {}
    roof = roofline_hbm(st["persistent_bytes"], t_launch, st["persistent_lup"], traffic_record(BATCH_COUNTERS, cfg),
                        "k_stream_persist (every full pass of all 512 instances: three concurrent per-class "
                        "launches per step, timed together)",
                        {"pass_depths": {"5": 8, "9": 8, "13": 6}, "rows_cap": cap,
                         "traffic_rows_cap": crec.get("rows_cap") if crec.get("kernel_cfg") == cfg else None,
                         "launches_timed": len(ms_persist), "alu": alu_view(BATCH_COUNTERS)})
    return {"value": round(st["lup"] * args.steps / elapsed / 1e9, 2),
            "ms_per_step": round(elapsed / args.steps * 1e3, 3), "graph_replay_value": round(graph_glups, 2),
            "stats": {k: st[k] for k in ("instances", "rounds", "launches", "lup", "state_bytes", "items",
                                         "persistent_items", "persistent_lup")},
            "mean_segment_rows": round(st["item_rows"] / max(1, st["items"]), 1),
            "roofline": roof, "error": errs}


# ---- single-grid workloads ------------------------------------------------------

def pass_time(w, p, u, lo, d, work, depth, launches):
    """Average time of one pass (one launch) of the streaming kernel, from
    HIP events on the stream the kernel runs on, after an untimed run of the
    same launches (a device idle for a while first runs at lower clocks)."""
    import torch
    stream = torch.cuda.current_stream()
    L = max(2, launches - launches % 2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w.wave2d_f32c_step(u, lo, d, p.h, p.tau, p.c, p.scheme, depth * L, work=work)
    e0.record(stream)
    w.wave2d_f32c_step(u, lo, d, p.h, p.tau, p.c, p.scheme, depth * L, work=work)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / L


def median_time(f, reps):
    import torch
    f()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        f()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2]


def exact_c2(p, k):
    """Exact solution of the PDE for the 9-point workload's data at t = k tau."""
    import numpy as np
    t = k * p.tau
    x = np.arange(p.nx) * p.h
    y = np.arange(p.ny) * p.h
    a = math.cos(math.sqrt(13.0) * math.pi * t)
    b = math.sin(math.sqrt(2.0) * math.pi * t) / (math.sqrt(2.0) * math.pi)
    return a * np.outer(np.sin(3 * math.pi * y), np.sin(2 * math.pi * x)) + \
        b * np.outer(np.sin(math.pi * y), np.sin(math.pi * x))


def c2_bench(args, dev):
    """9-point 4097^2, 2000 levels: compensated FP32 and FP64, errors
    against the oracle's closed-form discrete solution and the exact PDE
    solution, and the per-pass roofline of its fused pass kernel."""
    import torch

    import paper_1904_04048_amd as w
    from oracle import modes as M
    from paper_1904_04048_amd import workloads as W
    p = W.c2()
    u0, v0 = p.data()
    U0, V0 = torch.from_numpy(u0).to(dev), torch.from_numpy(v0).to(dev)
    del u0, v0
    u = torch.empty((p.ny, p.nx), dtype=torch.float32, device=dev)
    lo, d = torch.empty_like(u), torch.empty_like(u)
    work = torch.empty(w.wave2d_work_bytes(w.F32C, p.nx, p.ny), dtype=torch.uint8, device=dev)
    t = median_time(lambda: w.wave2d_f32c_run(U0, V0, u, lo, d, p.h, p.tau, p.c, p.scheme, p.steps, work=work), 5)
    got = torch.empty_like(U0)
    w.wave2d_f32c_export(u, lo, got)
    ref = torch.from_numpy(M.solution(p.modes, p.nx, p.ny, p.h, p.tau, p.c, p.scheme, p.steps)).to(dev)
    nr = w.wave2d_norms(got, ref)
    ne = w.wave2d_norms(got, torch.from_numpy(exact_c2(p, p.steps)).to(dev))
    work64 = torch.empty(w.wave2d_work_bytes(w.F64, p.nx, p.ny), dtype=torch.uint8, device=dev)
    P, C = torch.empty_like(U0), torch.empty_like(U0)
    t64 = median_time(lambda: w.wave2d_run(U0, V0, P, C, p.h, p.tau, p.c, p.scheme, p.steps, work=work64), 3)
    n64 = w.wave2d_norms(C, ref)
    del P, C, work64, ref, got
    depth, rows = w.wave2d_get_tuning(w.F32C, p.scheme, p.nx, p.ny)
    t_launch = pass_time(w, p, u, lo, d, work, depth, args.kernel_launches)
    cfg = {"kernel": "k_stream_fused<PF32C,KIND9>", "depth": depth, "rows": rows, "grid": [p.nx, p.ny],
           "source": kernel_source_hash()}
    roof = roofline_hbm(STATE_BYTES_PER_NODE * p.nx * p.ny, t_launch, p.interior * depth,
                        traffic_record(C2_COUNTERS, cfg), "k_stream_fused<PF32C,KIND9> (one pass)",
                        {"depth": depth, "rows": rows, "alu": alu_view(C2_COUNTERS)})
    return {"workload": "9-point, 4097x4097, 2000 levels, compensated FP32 (FP64 first step)",
            "value": round(p.lup / t / 1e9, 2), "unit": "GLUP/s", "ms_per_solve": round(t * 1e3, 2),
            "roofline": roof,
            "error": {"max_rel_vs_oracle_closed_form": nr[0] / nr[1], "max_rel_vs_exact_pde": ne[0] / ne[1]},
            "fp64_path": {"value": round(p.lup / t64 / 1e9, 2), "ms_per_solve": round(t64 * 1e3, 2),
                          "max_rel_vs_oracle_closed_form": n64[0] / n64[1],
                          "depth": w.wave2d_get_tuning(w.F64, p.scheme, p.nx, p.ny)[0]}}


def c3_bench(args, dev):
    """13-point Gaussian pulse on 8193^2, 3000 levels (compensated and FP64),
    and the same problem on a 1025^2 copy against the full-grid oracle."""
    import torch

    import oracle
    import paper_1904_04048_amd as w
    from paper_1904_04048_amd import workloads as W
    p = W.c3()
    u0, v0 = p.data()
    U0, V0 = torch.from_numpy(u0).to(dev), torch.from_numpy(v0).to(dev)
    del u0, v0
    u = torch.empty((p.ny, p.nx), dtype=torch.float32, device=dev)
    lo, d = torch.empty_like(u), torch.empty_like(u)
    work = torch.empty(w.wave2d_work_bytes(w.F32C, p.nx, p.ny), dtype=torch.uint8, device=dev)
    t = median_time(lambda: w.wave2d_f32c_run(U0, V0, u, lo, d, p.h, p.tau, p.c, p.scheme, p.steps, work=work), 3)
    P, C = torch.empty_like(U0), torch.empty_like(U0)
    t0 = time.perf_counter()
    w.wave2d_run(U0, V0, P, C, p.h, p.tau, p.c, p.scheme, p.steps)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    nr = w.wave2d_f32c_norms(u, lo, C)
    del P, C, U0, V0
    depth, rows = w.wave2d_get_tuning(w.F32C, p.scheme, p.nx, p.ny)
    t_launch = pass_time(w, p, u, lo, d, work, depth, max(2, args.kernel_launches // 4))
    cfg = {"kernel": "k_stream_fused<PF32C,KIND13>", "depth": depth, "rows": rows, "grid": [p.nx, p.ny],
           "source": kernel_source_hash()}
    roof = roofline_hbm(STATE_BYTES_PER_NODE * p.nx * p.ny, t_launch, p.interior * depth,
                        traffic_record(C3_COUNTERS, cfg), "k_stream_fused<PF32C,KIND13> (one pass)",
                        {"depth": depth, "rows": rows, "alu": alu_view(C3_COUNTERS)})
    del u, lo, d, work
    torch.cuda.empty_cache()
    # The 1025^2 copy: same pulse and Courant number, h = 1/1024.
    q = W.c3(n=1024)
    a0, b0 = q.data()
    A0, B0 = torch.from_numpy(a0).to(dev), torch.from_numpy(b0).to(dev)
    cu = torch.empty((q.ny, q.nx), dtype=torch.float32, device=dev)
    clo, cd = torch.empty_like(cu), torch.empty_like(cu)
    w.wave2d_f32c_run(A0, B0, cu, clo, cd, q.h, q.tau, q.c, q.scheme, q.steps)
    cp, cc = torch.empty_like(A0), torch.empty_like(A0)
    w.wave2d_run(A0, B0, cp, cc, q.h, q.tau, q.c, q.scheme, q.steps)
    got32 = (cu.double() + clo.double()).cpu().numpy()
    got64 = cc.cpu().numpy()
    tc = time.perf_counter()
    _, ref = oracle.run(a0, b0, q.h, q.tau, q.c, q.scheme, q.steps)
    tc = time.perf_counter() - tc
    return {"workload": "13-point, 8193x8193, 3000 levels, Gaussian pulse, compensated FP32",
            "value": round(p.lup / t / 1e9, 2), "unit": "GLUP/s", "ms_per_solve": round(t * 1e3, 2),
            "fp64_value": round(p.lup / t64 / 1e9, 2), "roofline": roof,
            "error": {"max_rel_vs_gpu_fp64": nr[0] / nr[1],
                      "copy_1025": {"max_rel_f32c_vs_oracle": oracle.rel_max_err(got32, ref),
                                    "max_rel_fp64_vs_oracle": oracle.rel_max_err(got64, ref),
                                    "oracle_s": round(tc, 1)}}}


def c1_bench(dev):
    """5-point FP64 standing wave on 257^2, 400 levels (launch-latency bound)."""
    import numpy as np
    import torch

    import oracle
    import paper_1904_04048_amd as w
    from paper_1904_04048_amd import workloads as W
    p = W.c1()
    u0, v0 = p.data()
    U0, V0 = torch.from_numpy(u0).to(dev), torch.from_numpy(v0).to(dev)
    P, C = torch.empty_like(U0), torch.empty_like(U0)
    # The launch shape from the library's autotuner for this grid (a small
    # grid's passes are latency bound: short segments give more waves).
    depth, rows = w.wave2d_autotune(w.F64, p.scheme, p.nx, p.ny)
    t = median_time(lambda: w.wave2d_run(U0, V0, P, C, p.h, p.tau, p.c, p.scheme, p.steps), 7)
    w.wave2d_set_tuning(w.F64, p.scheme)
    _, ref = oracle.run(u0, v0, p.h, p.tau, p.c, p.scheme, p.steps)
    got = C.cpu().numpy()
    x = np.arange(p.nx) * p.h
    ex = math.cos(math.sqrt(2.0) * math.pi * p.steps * p.tau) * np.outer(np.sin(math.pi * x), np.sin(math.pi * x))
    return {"workload": "5-point, 257x257, 400 levels, FP64, u0 = sin pi x sin pi y",
            "ms_per_solve": round(t * 1e3, 3), "value": round(p.lup / t / 1e9, 2), "unit": "GLUP/s",
            "depth": depth, "rows": rows,
            "error": {"max_rel_vs_oracle": oracle.rel_max_err(got, ref),
                      "max_rel_vs_exact_pde": oracle.rel_max_err(got, ex)}}


def off_table_bench(dev):
    """An untabulated size (6001^2, 9-point, compensated, 1000 levels): the
    library's size rule picks its launch shape, no measured table entry."""
    import torch

    import paper_1904_04048_amd as w
    from paper_1904_04048_amd import workloads as W
    p = W.c2(n=6000, steps=1000)
    U0, V0 = W.sine_series_torch(p.nx, p.ny, p.modes, dev)
    u = torch.empty((p.ny, p.nx), dtype=torch.float32, device=dev)
    lo, d = torch.empty_like(u), torch.empty_like(u)
    work = torch.empty(w.wave2d_work_bytes(w.F32C, p.nx, p.ny), dtype=torch.uint8, device=dev)
    t = median_time(lambda: w.wave2d_f32c_run(U0, V0, u, lo, d, p.h, p.tau, p.c, p.scheme, p.steps, work=work), 3)
    depth, rows = w.wave2d_get_tuning(w.F32C, p.scheme, p.nx, p.ny)
    return {"workload": "9-point, 6001x6001, 1000 levels, compensated FP32 (shape from the size rule)",
            "value": round(p.lup / t / 1e9, 2), "unit": "GLUP/s", "ms_per_solve": round(t * 1e3, 2),
            "depth": depth, "rows": rows}


def wide_bench(dev):
    """A built scheme reaching three lines out (the complete degree-6 set of
    Sec. 4-5, 25 nodes), 4097^2, 200 levels at 0.9 of its stability limit,
    FP64 and compensated FP32: one level per launch (FP64 through LDS-staged
    tiles, compensated by waves streaming down column strips), 24
    algorithmic bytes per update in both precisions (FP64: u^k and u^{k-1}
    read, u^{k+1} written; compensated: u, lo, d read and written)."""
    import torch

    import oracle
    import paper_1904_04048_amd as w
    from oracle import derive
    from paper_1904_04048_amd import workloads as W
    sid = w.wave2d_scheme_create(*W.complete_set(6))
    n, steps = 4097, 200
    h = 1.0 / (n - 1)
    tau = 0.9 * w.wave2d_lambda_max(sid) * h
    modes = [(2, 3, 1.0, 0.0), (1, 1, 0.0, 1.0)]
    U0, V0 = W.sine_series_torch(n, n, modes, dev)
    lup = (n - 2) * (n - 2) * steps
    P, C = torch.empty_like(U0), torch.empty_like(U0)
    t64 = median_time(lambda: w.wave2d_run(U0, V0, P, C, h, tau, 1.0, sid, steps), 3)
    u = torch.empty((n, n), dtype=torch.float32, device=dev)
    lo, d = torch.empty_like(u), torch.empty_like(u)
    work = torch.empty(w.wave2d_work_bytes(w.F32C, n, n), dtype=torch.uint8, device=dev)
    t32 = median_time(lambda: w.wave2d_f32c_run(U0, V0, u, lo, d, h, tau, 1.0, sid, steps, work=work), 3)
    # Errors: compensated FP32 against the GPU FP64 path at full size (both
    # after `steps` levels), and both paths against the oracle on a 257^2
    # copy of the workload.
    out = torch.empty_like(U0)
    w.wave2d_f32c_export(u, lo, out)
    f32_vs_f64 = float((out - C).abs().max() / C.abs().max())
    # One level of the compensated kernel, timed with HIP events on the
    # current stream (the state runs on past the compared level).
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    w.wave2d_f32c_step(u, lo, d, h, tau, 1.0, sid, 100, work=work)
    e1.record(stream)
    torch.cuda.synchronize()
    t_level = e0.elapsed_time(e1) / 1e3 / 100
    m = 257
    oracle.register_scheme(1010, derive.node_weights(28))
    u0s, v0s = W.sine_series(m, m, modes)
    hs = 1.0 / (m - 1)
    taus = 0.9 * w.wave2d_lambda_max(sid) * hs
    _, ref = oracle.run(u0s, v0s, hs, taus, 1.0, 1010, 400)
    U0s, V0s = torch.from_numpy(u0s).to(dev), torch.from_numpy(v0s).to(dev)
    us = torch.empty((m, m), dtype=torch.float32, device=dev)
    los, ds = torch.empty_like(us), torch.empty_like(us)
    w.wave2d_f32c_run(U0s, V0s, us, los, ds, hs, taus, 1.0, sid, 400)
    outs = torch.empty_like(U0s)
    w.wave2d_f32c_export(us, los, outs)
    Ps, Cs = torch.empty_like(U0s), torch.empty_like(U0s)
    w.wave2d_run(U0s, V0s, Ps, Cs, hs, taus, 1.0, sid, 400)
    alg = STATE_BYTES_PER_NODE * n * n
    cfg = {"kernel": "k_wide_step_f32c", "grid": [n, n], "source": wide_source_hash()}
    return {"workload": "built scheme, complete degree-6 set (25 nodes, radius 3), 4097x4097, 200 levels",
            "value": round(lup / t32 / 1e9, 2), "unit": "GLUP/s", "ms_per_solve": round(t32 * 1e3, 2),
            "fp64_value": round(lup / t64 / 1e9, 2), "fp64_ms_per_solve": round(t64 * 1e3, 2),
            "roofline": roofline_hbm(alg, t_level, (n - 2) * (n - 2), traffic_record(WIDE_COUNTERS, cfg),
                                     "k_wide_step_f32c (one level per launch)", {"alu": alu_view(WIDE_COUNTERS)}),
            "error": {"max_rel_f32c_vs_gpu_fp64": f32_vs_f64,
                      "copy_257_400_levels": {"max_rel_f32c_vs_oracle": oracle.rel_max_err(outs.cpu().numpy(), ref),
                                              "max_rel_fp64_vs_oracle": oracle.rel_max_err(Cs.cpu().numpy(), ref)}}}


# ---- served workload ------------------------------------------------------------

def serve_bench(args):
    """Requests drawn like the batch (sides up to 4096, 100-5000 levels)
    arriving as a Poisson process at 70% of the server's measured saturation
    throughput; latency = completion - submission.  Errors against the FP64
    oracle's closed form on every 8th request and on every request of side
    <= 512, and against the GPU FP64 path on every 32nd."""
    import threading

    import numpy as np
    import torch

    import oracle
    import paper_1904_04048_amd as w
    from oracle import modes as M
    from paper_1904_04048_amd import workloads as W

    n_meas = args.serve_requests
    n_warm = 32
    probs = W.c5_requests(n_warm + n_meas + 64)
    sv = w.wave2d_server_create(48 << 30)
    try:
        def submit(pr):
            return w.wave2d_server_submit(sv, pr.nx, pr.ny, pr.h, pr.tau, pr.c, pr.scheme, pr.steps, modes=pr.modes)

        burst = probs[-64:]
        t0 = time.perf_counter()
        ids = [submit(pr) for pr in burst]
        done = set()
        while len(done) < len(ids):
            for i in ids:
                if i not in done and w.wave2d_server_poll(sv, i) is not None:
                    done.add(i)
            time.sleep(0.0005)
        sat = sum(pr.lup for pr in burst) / (time.perf_counter() - t0) / 1e9
        for i in ids:
            w.wave2d_server_release(sv, i)
        mean_lup = float(np.mean([pr.lup for pr in probs[:n_warm + n_meas]]))
        qps = 0.7 * sat * 1e9 / mean_lup
        arrivals = W.poisson_arrivals(n_warm + n_meas, qps)
        sub_ids = [None] * len(arrivals)
        start = time.perf_counter()

        def client():
            for k, t in enumerate(arrivals):
                dt = start + t - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                sub_ids[k] = submit(probs[k])

        th = threading.Thread(target=client)
        th.start()
        # Results are checked and released as they finish, so the arena never
        # fills up with finished results.
        res = {}
        checked = {"closed_form": 0, "gpu_fp64": 0}
        worst = {"closed_form": 0.0, "gpu_fp64": 0.0}
        last_log = time.perf_counter()
        while len(res) < len(arrivals):
            progressed = False
            for k in range(len(arrivals)):
                if k in res or sub_ids[k] is None:
                    continue
                r = w.wave2d_server_poll(sv, sub_ids[k])
                if r is None:
                    continue
                progressed = True
                res[k] = {kk: r[kk] for kk in ("t_submit", "t_admit", "t_done", "status")}
                pr = probs[k]
                if k >= n_warm and (k % 8 == 0 or pr.nx <= 512):
                    got = w.result_tensor(r).cpu().numpy()
                    ref = M.solution(pr.modes, pr.nx, pr.ny, pr.h, pr.tau, pr.c, pr.scheme, pr.steps)
                    worst["closed_form"] = max(worst["closed_form"], oracle.rel_max_err(got, ref))
                    checked["closed_form"] += 1
                if k >= n_warm and k % 32 == 0:
                    U0 = torch.empty((pr.ny, pr.nx), dtype=torch.float64, device="cuda")
                    V0 = torch.empty_like(U0)
                    w.wave2d_sine_series(U0, V0, pr.modes)
                    P, C = torch.empty_like(U0), torch.empty_like(U0)
                    w.wave2d_run(U0, V0, P, C, pr.h, pr.tau, pr.c, pr.scheme, pr.steps)
                    nr = w.wave2d_norms(w.result_tensor(r).contiguous(), C)
                    worst["gpu_fp64"] = max(worst["gpu_fp64"], nr[0] / nr[1])
                    checked["gpu_fp64"] += 1
                    del U0, V0, P, C
                w.wave2d_server_release(sv, sub_ids[k])
            if time.perf_counter() - last_log > 5:
                log(f"serve: {len(res)} of {len(arrivals)} done")
                last_log = time.perf_counter()
            if not progressed:
                time.sleep(0.0005)
        th.join()
        makespan = time.perf_counter() - start
        meas = [res[k] for k in range(n_warm, len(arrivals))]
        assert all(r["status"] == 0 for r in meas)
        lat = np.array([r["t_done"] - r["t_submit"] for r in meas])
        t_first = min(r["t_submit"] for r in meas)
        t_last = max(r["t_done"] for r in meas)
        lup_meas = sum(probs[k].lup for k in range(n_warm, len(arrivals)))
        st = w.wave2d_server_stats_get(sv)
    finally:
        w.wave2d_server_destroy(sv)
    return {"workload": "Poisson arrivals of requests: sides 64-4096, schemes 5/9/13, 100-5000 levels, "
                        "compensated FP32, FP64 results",
            "requests": n_meas, "warmup_requests": n_warm, "qps": round(qps, 2),
            "saturation_glups": round(sat, 1), "value": round(lup_meas / (t_last - t_first) / 1e9, 1),
            "unit": "GLUP/s", "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "mean_ms": round(float(lat.mean()) * 1e3, 2), "makespan_s": round(makespan, 2),
            "quanta": st["quanta"],
            "error": {"max_rel_vs_oracle_closed_form": worst["closed_form"],
                      "requests_closed_form": checked["closed_form"],
                      "max_rel_vs_gpu_fp64": worst["gpu_fp64"], "requests_gpu_fp64": checked["gpu_fp64"],
                      "sample": "closed form: every 8th request and every request of side <= 512; "
                                "GPU FP64: every 32nd"}}


# ---- CPU baseline ----------------------------------------------------------------

def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(budget_s=12.0):
    """The FP64 CPU oracle (plain C loops, unchanged) on a bounded sample of
    the batched workload: its instances in order, each for up to 200 levels,
    until about budget_s seconds of work, on one thread and on every host
    thread it is given."""
    import oracle
    from paper_1904_04048_amd import workloads as W
    probs = W.c4()
    threads_all = oracle.get_threads()

    def run(threads):
        oracle.set_threads(threads)
        lup, t_tot, n = 0, 0.0, 0
        for pr in probs:
            if t_tot > budget_s:
                break
            u0, v0 = W.sine_series(pr.nx, pr.ny, pr.modes)
            steps = min(pr.steps, 200)
            t0 = time.perf_counter()
            oracle.run(u0, v0, pr.h, pr.tau, pr.c, pr.scheme, steps)
            t_tot += time.perf_counter() - t0
            lup += pr.interior * steps
            n += 1
        return lup / t_tot / 1e9, n, t_tot

    v1, n1, t1 = run(1)
    va, na, ta = run(threads_all)
    oracle.set_threads(threads_all)
    return {"value": round(va, 5), "unit": "GLUP/s", "cores": threads_all, "kind": "oracle",
            "sample": f"the first {na} instances of the 512-instance batch, up to 200 levels each "
                      f"({ta:.1f} s on {threads_all} threads)",
            "single_thread": {"value": round(v1, 5), "unit": "GLUP/s",
                              "sample": f"the first {n1} instances, up to 200 levels each ({t1:.1f} s)"},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


# ---- profile and summarize modes ----------------------------------------------------

def profile_run(dev):
    """Short run for rocprofv3 counter passes: a 256 MiB device copy (the
    counters' calibration), one run of the batch, ten passes each of the
    4097^2 9-point and 8193^2 13-point single-grid kernels, and ten levels of
    the degree-6 built scheme's compensated kernel at 4097^2."""
    import torch

    import paper_1904_04048_amd as w
    from paper_1904_04048_amd import workloads as W
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)  # 256 MiB
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    del a, b
    probs, insts, bt = make_batch(dev, host_data=True)
    try:
        cap = w.wave2d_batch_autotune(bt)
        w.wave2d_batch_run(bt)
        torch.cuda.synchronize()
        st = w.wave2d_batch_stats_get(bt)
    finally:
        w.wave2d_batch_destroy(bt)
    del insts
    torch.cuda.empty_cache()
    shapes = {}
    for p in (W.c2(), W.c3()):
        u0, v0 = p.data()
        U0, V0 = torch.from_numpy(u0).to(dev), torch.from_numpy(v0).to(dev)
        del u0, v0
        u = torch.empty((p.ny, p.nx), dtype=torch.float32, device=dev)
        lo, d = torch.empty_like(u), torch.empty_like(u)
        work = torch.empty(w.wave2d_work_bytes(w.F32C, p.nx, p.ny), dtype=torch.uint8, device=dev)
        depth, rows = w.wave2d_get_tuning(w.F32C, p.scheme, p.nx, p.ny)
        w.wave2d_f32c_run(U0, V0, u, lo, d, p.h, p.tau, p.c, p.scheme, 1, work=work)
        w.wave2d_f32c_step(u, lo, d, p.h, p.tau, p.c, p.scheme, depth * 10, work=work)
        torch.cuda.synchronize()
        shapes[str(p.scheme)] = {"depth": depth, "rows": rows, "grid": [p.nx, p.ny]}
        del U0, V0, u, lo, d, work
        torch.cuda.empty_cache()
    import numpy as np
    sid = w.wave2d_scheme_create(*W.complete_set(6))
    n = 4097
    rng = np.random.default_rng(0)
    u, lo, d = (torch.from_numpy(rng.uniform(-0.5, 0.5, (n, n)).astype(np.float32) * s).to(dev)
                for s in (1.0, 1e-8, 1e-3))
    h = 1.0 / (n - 1)
    w.wave2d_f32c_step(u, lo, d, h, 0.9 * w.wave2d_lambda_max(sid) * h, 1.0, sid, 10)
    torch.cuda.synchronize()
    del u, lo, d
    print(json.dumps({"profile": "done", "rows_cap": cap, "shapes": shapes, "source": kernel_source_hash(),
                      "wide": {"grid": [n, n], "source": wide_source_hash()},
                      "batch": {"persistent_bytes": st["persistent_bytes"], "persistent_lup": st["persistent_lup"]},
                      "copy_bytes": 2 * 256 * 1024 * 1024}), flush=True)


PROFILE_CMDS = [
    "    rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch -o fetch "
    "-- python3 bench.py --mode profile",
    "    rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write -o write "
    "-- python3 bench.py --mode profile",
    "    rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_ANY "
    "SQ_INSTS_VMEM_RD SQ_INSTS_SALU --output-format csv -d gpurun_out/pmc_sq -o sq "
    "-- python3 bench.py --mode profile",
    "    rocprofv3 --pmc GRBM_GUI_ACTIVE GRBM_COUNT --output-format csv -d gpurun_out/pmc_grbm -o grbm "
    "-- python3 bench.py --mode profile",
    "    python3 bench.py --mode summarize   (the profile run's JSON line in gpurun_out/pmc_fetch.log)"]


def summarize(prof_dir):
    """Write the profiles/ summaries from rocprofv3 csv output: FETCH_SIZE and
    WRITE_SIZE of the three step kernels (scaled by what the same counters
    read for a plain 256 MiB copy), their vector-instruction issue, and the
    kernel trace of a bench run."""
    import csv
    import statistics

    from paper_1904_04048_amd import workloads as W
    rec = None
    for line in open(os.path.join(prof_dir, "pmc_fetch.log")):
        if line.startswith("{") and '"profile"' in line:
            rec = json.loads(line)
    assert rec is not None, "no profile record in pmc_fetch.log"
    assert rec["source"] == kernel_source_hash(), "profiles were taken on other kernel sources"

    def per_kernel(path, multi=False):
        """(dispatch id, value) lists per kernel name (and counter name)."""
        out = {}
        if not os.path.exists(path):
            return out
        for r in csv.DictReader(open(path)):
            key = (r["Kernel_Name"], r["Counter_Name"]) if multi else r["Kernel_Name"]
            out.setdefault(key, []).append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
        return out

    def pick(vals, how):
        """The median over a kernel's dispatches, or its last dispatch."""
        return statistics.median(v for _, v in vals) if how == "median" else max(vals)[1]

    fetch = per_kernel(os.path.join(prof_dir, "pmc_fetch", "fetch_counter_collection.csv"))
    write = per_kernel(os.path.join(prof_dir, "pmc_write", "write_counter_collection.csv"))
    sq = per_kernel(os.path.join(prof_dir, "pmc_sq", "sq_counter_collection.csv"), True)
    gr = per_kernel(os.path.join(prof_dir, "pmc_grbm", "grbm_counter_collection.csv"), True)
    copy_bytes = 256 * 1024 * 1024
    # The calibration copies are the three largest copy-kernel dispatches
    # (host-to-device uploads of the batch's data also run as copy kernels).
    cf = statistics.median(sorted(v for _, v in [v for k, v in fetch.items() if "copyBuffer" in k][0])[-3:])
    cw = statistics.median(sorted(v for _, v in [v for k, v in write.items() if "copyBuffer" in k][0])[-3:])
    f_scale = copy_bytes / (cf * 1024)
    w_scale = copy_bytes / (cw * 1024)
    simds = 256 * 4

    def one(title, path, match, cfg, alg, lup, how="median", nk=1, note="", extra=None):
        """Counters of one launch of a kernel, or summed over the `nk`
        kernels that `match` selects (the batch's per-class launches)."""
        extra = extra or {}
        kf = [pick(v, how) for k, v in fetch.items() if match(k)]
        kw = [pick(v, how) for k, v in write.items() if match(k)]
        assert len(kf) == nk and len(kw) == nk, (title, len(kf), len(kw))
        rd = sum(kf) * 1024 * f_scale
        wr = sum(kw) * 1024 * w_scale
        out = {"kernel_cfg": cfg, **extra, "hbm_bytes_per_launch": int(rd + wr), "read_bytes_per_launch": int(rd),
               "write_bytes_per_launch": int(wr), "algorithmic_bytes_per_launch": int(alg),
               "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4)}
        issue_md = []
        v = {c: [pick(x, how) for (k, cn), x in sq.items() if match(k) and cn == c]
             for c in ("SQ_INSTS_VALU", "SQ_WAVES", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_WAIT_INST_ANY",
                       "SQ_WAVE_CYCLES")}
        g = [pick(x, how) for (k, cn), x in gr.items() if match(k) and cn == "GRBM_GUI_ACTIVE"]
        if all(len(x) == nk for x in v.values()) and len(g) == nk:
            v = {c: [sum(x)] for c, x in v.items()}
            g = [sum(g)]
            cycles = g[0] / XCDS  # the counter sums the 8 XCDs' clocks
            valu = v["SQ_INSTS_VALU"][0]
            issue = valu * 4 / (simds * cycles)
            out["valu_issue_frac"] = round(issue, 4)
            out["lane_ops_per_lup"] = round(valu * 64 / lup, 2)
            out["wait_frac"] = round(v["SQ_WAIT_INST_ANY"][0] / max(1.0, v["SQ_WAVE_CYCLES"][0]), 4)
            issue_md = ["", "| waves | VALU insts | SALU insts | VMEM reads | cycles | us | VALU issue | "
                            "lane-ops per update | wait / wave cycles |",
                        "|---|---|---|---|---|---|---|---|---|",
                        f"| {v['SQ_WAVES'][0]:.0f} | {valu:.4g} | {v['SQ_INSTS_SALU'][0]:.4g} | "
                        f"{v['SQ_INSTS_VMEM_RD'][0]:.4g} | {cycles:.0f} | {cycles / 2.4e3:.1f} | {issue:.3f} | "
                        f"{valu * 64 / lup:.1f} | {out['wait_frac']:.3f} |", "",
                        "VALU issue = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x cycles), the fraction of SIMD "
                        "cycles that issue a wave64 vector instruction (one per 4 cycles per SIMD without "
                        "packed FP32); GRBM_GUI_ACTIVE sums the clocks of the 8 XCDs, so the kernel's cycles "
                        "are that / 8.  Lane operations per update = VALU instructions x 64 / grid-point "
                        "updates of the launch (useful updates only)."]
        md = [f"# {title}", "", "Commands (from the repository root, one MI355X, one counter group per run):", ""] + \
            PROFILE_CMDS + ["",
                            f"Copy calibration (256 MiB device copy): FETCH_SIZE reads {cf:.0f} "
                            f"KiB (scale {f_scale:.3f}), WRITE_SIZE reads {cw:.0f} KiB "
                            f"(scale {w_scale:.3f}).", "",
                            f"One launch{note}: FETCH_SIZE {sum(kf):.0f} KiB, WRITE_SIZE {sum(kw):.0f} KiB; "
                            f"scaled: read {rd / 1e6:.1f} MB, write {wr / 1e6:.1f} MB against {alg / 1e6:.1f} MB "
                            f"algorithmic ({(rd + wr) / alg:.2f}x)."] + issue_md + \
            ["", "```json", json.dumps(out, indent=1), "```", ""]
        open(path, "w").write("\n".join(md))
        print(title, json.dumps(out))

    bst = rec["batch"]
    one("HBM traffic and issue of the persistent batch launches (512 instances, compensated FP32)",
        BATCH_COUNTERS, lambda k: "k_stream_persist" in k,
        {"kernel": "k_stream_persist", "source": rec["source"]},
        bst["persistent_bytes"], bst["persistent_lup"], how="last", nk=3, extra={"rows_cap": rec["rows_cap"]},
        note=(f" (the three per-class launches of the run after autotuning, segments of at most "
              f"{rec['rows_cap']} rows, summed; under counter collection the launches run one at a time)"))
    for scheme, path, kind, p in ((9, C2_COUNTERS, 1, W.c2()), (13, C3_COUNTERS, 2, W.c3())):
        sh = rec["shapes"][str(scheme)]
        tag = f"PF32C, {kind}, {sh['depth']}, 2>"
        name = "KIND9" if kind == 1 else "KIND13"
        one(f"HBM traffic and issue of one {scheme}-point compensated pass, {p.nx} x {p.ny}",
            path, lambda k, tag=tag: "k_stream_fused" in k and tag in k,
            {"kernel": f"k_stream_fused<PF32C,{name}>", "depth": sh["depth"], "rows": sh["rows"],
             "grid": [p.nx, p.ny], "source": rec["source"]},
            STATE_BYTES_PER_NODE * p.nx * p.ny, p.interior * sh["depth"])
    if "wide" in rec:
        n = rec["wide"]["grid"][0]
        one(f"HBM traffic and issue of one level of the degree-6 built scheme's compensated kernel, {n} x {n}",
            WIDE_COUNTERS, lambda k: "k_wide_step_f32c" in k,
            {"kernel": "k_wide_step_f32c", "grid": [n, n], "source": rec["wide"]["source"]},
            STATE_BYTES_PER_NODE * n * n, (n - 2) * (n - 2))

    tpath = os.path.join(prof_dir, "prof_bench", "bench_kernel_stats.csv")
    if os.path.exists(tpath):
        stats = list(csv.DictReader(open(tpath)))
        lines = ["# Kernel statistics of a benchmark run (batch headline and single grids)", "",
                 "Command (from the repository root, on one MI355X):", "",
                 "    rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_bench -o bench \\",
                 "        -- python3 bench.py --steps 3 --warmup 1 --no-cpu --no-serve > gpurun_out/prof_bench.log",
                 "",
                 "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
        for r in stats[:14]:
            name = r["Name"].replace("w2d::(anonymous namespace)::", "").replace("|", "/")
            if len(name) > 90:
                name = name[:90] + "..."
            lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs'])/1e3:.1f} | "
                         f"{float(r['MinNs'])/1e3:.1f} | {float(r['MaxNs'])/1e3:.1f} | {float(r['Percentage']):.1f} |")
        lines += batch_spans(prof_dir)
        open(BATCH_STATS, "w").write("\n".join(lines) + "\n")
        print(open(BATCH_STATS).read())


AUTOTUNE_RUNS = 7 * 3  # wave2d_batch_autotune: 7 candidate heights x (1 warm-up + 2 timed runs)


def batch_spans(prof_dir):
    """The persistent phase of each batch run in the kernel trace: from the
    first start to the last end of its three concurrent per-class launches.
    Runs in trace order: autotuning, warm-up, the timed steps, then the
    graph replays; the timed steps' mean is set beside the bench line's own
    HIP-event figure of the same run."""
    import csv
    import statistics
    tpath = os.path.join(prof_dir, "prof_bench", "bench_kernel_trace.csv")
    lpath = os.path.join(prof_dir, "prof_bench.log")
    if not (os.path.exists(tpath) and os.path.exists(lpath)):
        return []
    line = [x for x in open(lpath) if x.startswith("{") and '"metric"' in x][-1]
    b = json.loads(line)
    ds = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"])
                for r in csv.DictReader(open(tpath)) if "k_stream_persist" in r["Kernel_Name"])
    runs = [ds[i:i + 3] for i in range(0, len(ds), 3)]
    reps = max(2, min(5, b["steps"]))
    assert len(runs) == AUTOTUNE_RUNS + b["warmup"] + b["steps"] + 1 + reps, len(runs)
    assert all(len({k for _, _, k in r}) == 3 for r in runs)
    timed = runs[AUTOTUNE_RUNS + b["warmup"]:AUTOTUNE_RUNS + b["warmup"] + b["steps"]]
    spans = [(max(e for _, e, _ in r) - min(t for t, _, _ in r)) / 1e3 for r in timed]
    mean = statistics.mean(spans)
    ev = b["roofline"]["launch_us"]
    return ["", "Persistent phase of the timed batch runs (three concurrent per-class launches, first start "
                "to last end in the trace):", "",
            "| run | span us |", "|---|---|"] + [f"| {k} | {x:.0f} |" for k, x in enumerate(spans)] + \
           ["", f"Mean {mean:.0f} us; the bench line of the same run measured {ev:.0f} us with HIP events "
                f"around the three launches ({(ev - mean) / mean * 100:+.1f}%).  Bench line: value "
                f"{b['value']} GLUP/s, roofline frac {b['roofline']['frac']}, segments of at most "
                f"{b['roofline']['rows_cap']} rows."]


def main():
    args = parse()
    if args.mode == "summarize":
        summarize(args.prof_dir)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs on one GPU; a multi-GPU decomposition is described but not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    dev = torch.device("cuda:0")
    if args.mode == "profile":
        profile_run(dev)
        return

    log("batch")
    bt = batch_bench(args, dev)
    torch.cuda.empty_cache()
    out = {
        "metric": METRIC, "value": bt["value"], "unit": "GLUP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": bt["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "512-instance batch: sides 64-2048, schemes 5/9/13, lambda 0.3-0.9 of the limit, "
                               "100-2000 levels, 8 sine modes, compensated FP32 (FP64 first steps)",
                   "instances": bt["stats"]["instances"], "lup_per_step": bt["stats"]["lup"],
                   "parallelism": "single GPU", "seed": 0},
        "roofline": bt["roofline"],
        "error": bt["error"],
        "batch": {k: bt[k] for k in ("stats", "mean_segment_rows", "graph_replay_value")},
    }
    if not args.no_single:
        log("single grids")
        single = {"c2_9pt_4097": c2_bench(args, dev)}
        torch.cuda.empty_cache()
        single["c3_13pt_8193"] = c3_bench(args, dev)
        torch.cuda.empty_cache()
        single["c1_5pt_257_fp64"] = c1_bench(dev)
        single["off_table_9pt_6001"] = off_table_bench(dev)
        torch.cuda.empty_cache()
        single["wide_deg6_4097"] = wide_bench(dev)
        torch.cuda.empty_cache()
        out["single_grid"] = single
    if not args.no_serve:
        log("serving")
        out["serving"] = serve_bench(args)
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

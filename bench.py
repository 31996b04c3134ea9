"""Benchmark of the wave2d hot path on one MI355X.

One step = one whole solve of the 9-point workload on a 4097 x 4097 grid
(h = 1/4096, c = 1, lambda = 0.9 x the stability limit, 2000 time levels,
u0 = sin 2 pi x sin 3 pi y, v0 = sin pi x sin pi y): the FP64 first step
fused with the compensated-FP32 state split, 1999 temporally blocked
two-step updates, and the FP64 error norms of the result against an FP64
GPU solve of the same problem.  Inputs are resident on the GPU before the
timed region.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
    python bench.py --mode profile     # short run for rocprofv3 counter passes
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid-point updates/s (GLUP/s) + % HBM roofline; served p50/p99 latency at fixed error"
HBM_PEAK_GBS = 8000.0
# Vector ALU peak available to this build: 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops (fused multiply-add) x 2.4 GHz.  The published 157.3 TFLOP/s FP32
# figure needs packed FP32 instructions, which this build does not emit.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Floating-point operations of one compensated 9-point grid-point update as
# formulated (a fused multiply-add counts two): u stencil 8 sub + 6 add +
# mul + fma = 17; lo stencil 6 add + mul + 2 fma = 11; d += s, y = d + lo,
# s = su + slo and the 6-operation TwoSum = 9.
FLOPS_PER_LUP_F32C_9PT = 37
STATE_BYTES_PER_NODE = 24  # compensated state (u, lo, d): 12 B read + 12 B written per node per pass
KERNEL_NAME = "k_stream_fused<PF32C,KIND9> (one pass: boundary and interior work items)"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", choices=["bench", "profile", "summarize"], default="bench")
    ap.add_argument("--prof-dir", default=os.path.join(ROOT, "gpurun_out"),
                    help="summarize: directory holding the rocprofv3 csv output")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--kernel-launches", type=int, default=100)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 512-instance workload")
    ap.add_argument("--no-serve", action="store_true", help="skip the served workload")
    ap.add_argument("--serve-requests", type=int, default=300)
    return ap.parse_args()


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


def cpu_baseline(p, u0, v0, budget_s=20.0):
    """The FP64 CPU oracle on a bounded sample of the same solve: the first
    step and as many two-step updates as fit in about budget_s seconds."""
    import oracle
    threads = oracle.get_threads()
    t0 = time.perf_counter()
    um1, u = u0.copy(), oracle.first_step(u0, v0, p.h, p.tau, p.c, p.scheme)
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    um1, u = oracle.steps(um1, u, p.h, p.tau, p.c, p.scheme, 2)
    per = (time.perf_counter() - t0) / 2
    n = int(max(4, min(2000, (budget_s - t_first) / max(per, 1e-9))))
    t0 = time.perf_counter()
    oracle.steps(um1, u, p.h, p.tau, p.c, p.scheme, n)
    dt = time.perf_counter() - t0
    return {"value": round(p.interior * n / dt / 1e9, 5), "unit": "GLUP/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} two-step updates of the {p.nx}x{p.ny} 9-point FP64 solve ({dt:.1f} s timed)"}


COUNTERS_MD = os.path.join(ROOT, "profiles", "k_stream_f32c_9pt_4097_counters.md")
STATS_MD = os.path.join(ROOT, "profiles", "k_stream_f32c_9pt_4097_kernel_stats.md")
VALU_MD = os.path.join(ROOT, "profiles", "k_stream_f32c_9pt_4097_valu.md")
XCDS = 8


def kernel_source_hash():
    """Hash of the sources the step kernels are built from: a counter record
    taken on other sources no longer describes the kernel."""
    import hashlib
    h = hashlib.sha256()
    for f in ("stream.hip", "point.h", "w2d.h"):
        h.update(open(os.path.join(ROOT, "paper_1904_04048_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_record(kernel_cfg):
    """Measured HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on this kernel configuration."""
    try:
        text = open(COUNTERS_MD).read()
        rec = json.loads(text.split("```json")[1].split("```")[0])
    except (OSError, ValueError, IndexError):
        return None
    if rec.get("kernel_cfg") != kernel_cfg:
        return None
    return rec.get("hbm_bytes_per_launch")


def summarize(prof_dir):
    """Write the profiles/ summaries from rocprofv3 csv output: kernel-trace
    statistics of a bench run, and FETCH_SIZE / WRITE_SIZE of the dominant
    kernel scaled by what the same counters read for a plain copy."""
    import csv
    import statistics
    # The shape the profile runs used, as they printed it (the default height
    # depends on the device's occupancy, so it is not recomputed here).
    cfg = None
    for line in open(os.path.join(prof_dir, "pmc_fetch.log")):
        if line.startswith("{") and '"profile"' in line:
            cfg = json.loads(line)["kernel_cfg"]
    assert cfg is not None, "no profile record in pmc_fetch.log"
    depth, rows = cfg["depth"], cfg["rows"]
    stats = list(csv.DictReader(open(os.path.join(prof_dir, "prof_bench", "bench_kernel_stats.csv"))))
    lines = ["# Kernel statistics: 9-point compensated-FP32 workload, 4097 x 4097, 2000 levels", "",
             "Command (from the repository root, on one MI355X):", "",
             "    rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_bench -o bench \\",
             "        -- python3 bench.py --steps 2 --warmup 1 --no-cpu", "",
             "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in stats[:8]:
        name = r["Name"].replace("w2d::(anonymous namespace)::", "").replace("|", "/")
        if len(name) > 90:
            name = name[:90] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs'])/1e3:.1f} | {float(r['MinNs'])/1e3:.1f} | "
                     f"{float(r['MaxNs'])/1e3:.1f} | {float(r['Percentage']):.1f} |")
    # The headline pass kernels alone: the same kernels also run on other
    # grids (autotuning, batches), so their dispatches are told apart by grid
    # size; the 4097^2 solve is the grid with the most dispatches.
    per = {}
    for r in csv.DictReader(open(os.path.join(prof_dir, "prof_bench", "bench_kernel_trace.csv"))):
        n = r["Kernel_Name"]
        for kind in ("fused",):
            if f"k_stream_{kind}<" in n and f"PF32C, 1, {depth}, 2>" in n:
                dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                per.setdefault(kind, {}).setdefault(int(r["Grid_Size_X"]), []).append(dur)
    lines += ["", f"Headline pass kernels (9-point compensated, 4097 x 4097, depth {depth}, rows {rows}):",
              "", "| kernel | waves | dispatches | avg us | min us | max us |", "|---|---|---|---|---|---|"]
    for kind, by_grid in sorted(per.items()):
        g = max(by_grid, key=lambda k: len(by_grid[k]))
        v = by_grid[g]
        lines.append(f"| k_stream_{kind}<PF32C,KIND9,{depth}> | {g // 64} | {len(v)} | {sum(v)/len(v):.1f} | "
                     f"{min(v):.1f} | {max(v):.1f} |")
    lines += ["", "One launch per pass holds the boundary work items (first wave ids) and the interior ones.", ""]
    open(STATS_MD, "w").write("\n".join(lines) + "\n")

    def per_kernel(path):
        out = {}
        for r in csv.DictReader(open(path)):
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out
    fetch = per_kernel(os.path.join(prof_dir, "pmc_fetch", "fetch_counter_collection.csv"))
    write = per_kernel(os.path.join(prof_dir, "pmc_write", "write_counter_collection.csv"))
    copy_bytes = 256 * 1024 * 1024  # bench.py --mode profile copies 256 MiB per dispatch
    cf = [v for k, v in fetch.items() if "copyBuffer" in k][0]
    cw = [v for k, v in write.items() if "copyBuffer" in k][0]
    f_scale = copy_bytes / (statistics.median(cf) * 1024)
    w_scale = copy_bytes / (statistics.median(cw) * 1024)
    from paper_1904_04048_amd import workloads as W
    p = W.c2()
    # One pass = one launch of the fused kernel of this depth.
    tag = f"PF32C, 1, {depth}, 2>"
    kf = [statistics.median(v) for k, v in fetch.items() if "k_stream_fused" in k and tag in k]
    kw = [statistics.median(v) for k, v in write.items() if "k_stream_fused" in k and tag in k]
    assert len(kf) == 1 and len(kw) == 1, (len(kf), len(kw))
    rd = sum(kf) * 1024 * f_scale
    wr = sum(kw) * 1024 * w_scale
    assert cfg["source"] == kernel_source_hash(), "profiles were taken on other kernel sources"
    alg = STATE_BYTES_PER_NODE * p.nx * p.ny
    rec = {"kernel_cfg": cfg, "hbm_bytes_per_launch": int(rd + wr), "read_bytes_per_launch": int(rd),
           "write_bytes_per_launch": int(wr), "algorithmic_bytes_per_launch": alg,
           "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4)}
    md = ["# HBM traffic of the dominant kernel pass (compensated FP32, 9-point, 4097 x 4097)", "",
          "Commands (from the repository root, one MI355X, one counter per run):", "",
          "    rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch -o fetch -- python3 bench.py --mode profile",
          "    rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write -o write -- python3 bench.py --mode profile",
          "    python3 bench.py --mode summarize", "",
          f"Copy calibration (256 MiB device copy): FETCH_SIZE reads {statistics.median(cf):.0f} KiB "
          f"(scale {f_scale:.3f}), WRITE_SIZE reads {statistics.median(cw):.0f} KiB (scale {w_scale:.3f}).", "",
          f"One pass of the step kernel (boundary and interior items), depth {depth}, rows {rows}: FETCH_SIZE "
          f"{sum(kf):.0f} KiB, WRITE_SIZE {sum(kw):.0f} KiB per pass; scaled: read {rd/1e6:.1f} MB, "
          f"write {wr/1e6:.1f} MB per launch against {alg/1e6:.1f} MB algorithmic "
          f"({(rd + wr)/alg:.2f}x).", "", "```json", json.dumps(rec, indent=1), "```", ""]
    open(COUNTERS_MD, "w").write("\n".join(md))
    print(json.dumps(rec))

    # Instruction issue of the same pass, if the SQ and GRBM counter runs exist.
    sq_csv = os.path.join(prof_dir, "pmc_sq", "sq_counter_collection.csv")
    gr_csv = os.path.join(prof_dir, "pmc_grbm", "grbm_counter_collection.csv")
    if not (os.path.exists(sq_csv) and os.path.exists(gr_csv)):
        return

    def per_kernel_counter(path):
        out = {}
        for r in csv.DictReader(open(path)):
            if "k_stream_fused" in r["Kernel_Name"] and tag in r["Kernel_Name"]:
                out.setdefault(("pass", r["Counter_Name"]), []).append(float(r["Counter_Value"]))
        return {k: statistics.median(v) for k, v in out.items()}
    sq = per_kernel_counter(sq_csv)
    sq.update(per_kernel_counter(gr_csv))
    simds = 256 * 4
    lup = p.interior * depth
    rows_md = []
    for kind in ("pass",):
        v = {c: sq.get((kind, c)) for c in ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_SALU",
                                            "SQ_INSTS_VMEM_RD", "SQ_WAVES", "GRBM_GUI_ACTIVE")}
        if any(x is None for x in v.values()):
            continue
        cycles = v["GRBM_GUI_ACTIVE"] / XCDS  # the counter sums the 8 XCDs' clocks
        issue = v["SQ_INSTS_VALU"] * 4 / (simds * cycles)
        rows_md.append(f"| {kind} | {v['SQ_WAVES']:.0f} | {v['SQ_INSTS_VALU']:.4g} | {v['SQ_INSTS_SALU']:.4g} | "
                       f"{v['SQ_INSTS_VMEM_RD']:.4g} | {cycles:.0f} | {cycles / 2.4e3:.1f} | {issue:.3f} |")
    tot_valu = sq.get(("pass", "SQ_INSTS_VALU"), 0.0)
    md = ["# Vector instruction issue of the dominant kernel pass (compensated FP32, 9-point, 4097 x 4097)", "",
          "Commands (from the repository root, one MI355X, one counter group per run):", "",
          "    rocprofv3 --pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES "
          "SQ_WAIT_INST_ANY SQ_INSTS_VMEM_RD SQ_INSTS_SALU --output-format csv -d gpurun_out/pmc_sq -o sq "
          "-- python3 bench.py --mode profile",
          "    rocprofv3 --pmc GRBM_GUI_ACTIVE GRBM_COUNT --output-format csv -d gpurun_out/pmc_grbm -o grbm "
          "-- python3 bench.py --mode profile",
          "    python3 bench.py --mode summarize", "",
          f"Shape: depth {depth}, rows {rows}; one launch per pass (boundary and interior work items).  "
          "Medians over the dispatches of the profile run.  GRBM_GUI_ACTIVE sums the clocks of the 8 XCDs, so the kernel's "
          "cycles are that / 8 (us at 2.4 GHz shown beside them).  `issue` = SQ_INSTS_VALU x 4 cycles / "
          "(1024 SIMDs x cycles): the fraction of SIMD cycles that issue a wave64 vector instruction (one per "
          "4 cycles per SIMD without packed FP32).  SQ_ACTIVE_INST_VALU reads the same as SQ_INSTS_VALU on "
          "this device and adds nothing.", "",
          "| kernel | waves | VALU insts | SALU insts | VMEM reads | cycles | us | issue |",
          "|---|---|---|---|---|---|---|---|"] + rows_md + ["",
          f"VALU instructions per grid-point update of the pass (lane operations / useful updates): "
          f"{tot_valu * 64 / lup:.1f}", ""]
    open(VALU_MD, "w").write("\n".join(md))
    print(open(VALU_MD).read())


def other_workloads():
    """Throughput of the two other single-grid workloads (not the headline):
    the 5-point FP64 standing wave on 257^2 (400 levels, launch-latency
    bound) and the 13-point Gaussian pulse on 8193^2 (3000 levels,
    compensated, with its error against the FP64 GPU solve)."""
    import torch

    import paper_1904_04048_amd as w
    from paper_1904_04048_amd import workloads as W

    dev = torch.device("cuda:0")
    out = {}

    def timed(f, reps):
        f()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            f()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[len(ts) // 2]

    p = W.c1()
    u0, v0 = p.data()
    U0, V0 = torch.from_numpy(u0).to(dev), torch.from_numpy(v0).to(dev)
    P, C = torch.empty_like(U0), torch.empty_like(U0)
    t = timed(lambda: w.wave2d_run(U0, V0, P, C, p.h, p.tau, p.c, p.scheme, p.steps), 5)
    out["standing_wave_257_fp64"] = {"workload": "5-point, 257x257, 400 levels, FP64, u0 = sin pi x sin pi y",
                                     "ms_per_solve": round(t * 1e3, 3), "value": round(p.lup / t / 1e9, 2),
                                     "unit": "GLUP/s"}
    p = W.c3()
    u0, v0 = p.data()
    U0, V0 = torch.from_numpy(u0).to(dev), torch.from_numpy(v0).to(dev)
    u = torch.empty((p.ny, p.nx), dtype=torch.float32, device=dev)
    lo, d = torch.empty_like(u), torch.empty_like(u)
    t = timed(lambda: w.wave2d_f32c_run(U0, V0, u, lo, d, p.h, p.tau, p.c, p.scheme, p.steps), 2)
    P, C = torch.empty_like(U0), torch.empty_like(U0)
    t64 = timed(lambda: w.wave2d_run(U0, V0, P, C, p.h, p.tau, p.c, p.scheme, p.steps), 1)
    nr = w.wave2d_f32c_norms(u, lo, C)
    depth, rows = w.wave2d_get_tuning(w.F32C, p.scheme, p.nx, p.ny)
    out["gaussian_8193_13pt"] = {"workload": "13-point, 8193x8193, 3000 levels, Gaussian pulse, compensated FP32",
                                 "ms_per_solve": round(t * 1e3, 2), "value": round(p.lup / t / 1e9, 2),
                                 "unit": "GLUP/s", "depth": depth, "rows": rows,
                                 "fp64_value": round(p.lup / t64 / 1e9, 2),
                                 "max_rel_err_vs_gpu_fp64": nr[0] / nr[1]}
    del U0, V0, u, lo, d, P, C
    torch.cuda.empty_cache()
    return out


def batch_bench(args):
    """The batched workload: 512 seeded instances (sides log-uniform in
    [64, 2048], schemes uniform over 5/9/13-point, lambda in [0.3, 0.9] x
    limit, 100-2000 levels, 8 random sine modes), compensated FP32, the
    library's default depth per stencil class (the segment height is chosen
    per batched launch), the whole batch replayed as one graph.  (Tuning on
    a single 1025^2 grid is not used: single grids run one fused launch per
    pass, batches two launches on two streams, and their best depths
    differ.)"""
    import torch

    import paper_1904_04048_amd as w
    from paper_1904_04048_amd import workloads as W

    dev = torch.device("cuda:0")
    tuned = {sch: w.wave2d_get_tuning(w.F32C, sch) for sch in (w.P5, w.P9, w.P13)}
    probs = W.c4()
    insts = []
    for pr in probs:
        U0, V0 = W.sine_series_torch(pr.nx, pr.ny, pr.modes, dev)
        u = torch.empty((pr.ny, pr.nx), dtype=torch.float32, device=dev)
        insts.append(dict(nx=pr.nx, ny=pr.ny, h=pr.h, tau=pr.tau, c=pr.c, scheme=pr.scheme, steps=pr.steps,
                          flags=0, u0=U0, v0=V0, u=u, lo=torch.empty_like(u), d=torch.empty_like(u)))
    b = w.wave2d_batch_create(insts, w.BATCH_GRAPH)
    try:
        st = w.wave2d_batch_stats_get(b)
        w.wave2d_batch_run(b)  # captures the graph, warms up
        torch.cuda.synchronize()
        reps = max(1, min(3, args.steps))
        t0 = time.perf_counter()
        for _ in range(reps):
            w.wave2d_batch_run(b)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        # Accuracy on a sample: every 64th instance against its FP64 GPU solve.
        worst = 0.0
        for k in range(0, len(insts), 64):
            t = insts[k]
            P = torch.empty_like(t["u0"])
            C = torch.empty_like(t["u0"])
            w.wave2d_run(t["u0"], t["v0"], P, C, t["h"], t["tau"], t["c"], t["scheme"], t["steps"])
            nr = w.wave2d_f32c_norms(t["u"], t["lo"], C)
            worst = max(worst, nr[0] / nr[1])
    finally:
        w.wave2d_batch_destroy(b)
    return {"workload": "512 instances, sides 64-2048, schemes 5/9/13, 100-2000 levels, compensated FP32",
            "value": round(st["lup"] / dt / 1e9, 2), "unit": "GLUP/s", "ms_per_batch": round(dt * 1e3, 2),
            "lup": st["lup"], "rounds": st["rounds"], "launches_per_run": st["launches"],
            "state_bytes": st["state_bytes"], "graph": True,
            "shapes": {str(k): list(v) for k, v in tuned.items()},
            "work_items": st["items"], "mean_segment_rows": round(st["item_rows"] / max(1, st["items"]), 1),
            "max_rel_err_vs_gpu_fp64_sampled": worst, "sample": "every 64th instance"}


def serve_bench(args):
    """Served workload: requests drawn like the batch (sides up to 4096,
    100-5000 levels), arriving as a Poisson process at 70% of the server's
    measured saturation throughput; latency = completion - submission."""
    import threading

    import numpy as np
    import torch

    import paper_1904_04048_amd as w
    from paper_1904_04048_amd import workloads as W

    n_meas = args.serve_requests
    n_warm = 16
    probs = W.c5_requests(n_warm + n_meas + 64)
    sv = w.wave2d_server_create(48 << 30)
    try:
        def submit(pr):
            return w.wave2d_server_submit(sv, pr.nx, pr.ny, pr.h, pr.tau, pr.c, pr.scheme, pr.steps, modes=pr.modes)

        def drain(ids):
            out = {}
            while len(out) < len(ids):
                for i in ids:
                    if i not in out:
                        r = w.wave2d_server_poll(sv, i)
                        if r is not None:
                            out[i] = r
                time.sleep(0.0005)
            return out

        # Saturation: a burst of requests submitted at once.
        burst = probs[-64:]
        t0 = time.perf_counter()
        ids = [submit(pr) for pr in burst]
        drain(ids)
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
        th.join()
        res = drain(sub_ids)
        makespan = time.perf_counter() - start
        meas = [res[sub_ids[k]] for k in range(n_warm, len(sub_ids))]
        lat = np.array([r["t_done"] - r["t_submit"] for r in meas])
        t_first = min(r["t_submit"] for r in meas)
        t_last = max(r["t_done"] for r in meas)
        lup_meas = sum(probs[k].lup for k in range(n_warm, len(sub_ids)))
        # Error on a sample: served result against the FP64 GPU solve.
        worst = 0.0
        for k in range(n_warm, len(sub_ids), 50):
            pr = probs[k]
            U0 = torch.empty((pr.ny, pr.nx), dtype=torch.float64, device="cuda")
            V0 = torch.empty_like(U0)
            w.wave2d_sine_series(U0, V0, pr.modes)
            P, C = torch.empty_like(U0), torch.empty_like(U0)
            w.wave2d_run(U0, V0, P, C, pr.h, pr.tau, pr.c, pr.scheme, pr.steps)
            got = w.result_tensor(res[sub_ids[k]])
            nr = w.wave2d_norms(got.contiguous(), C)
            worst = max(worst, nr[0] / nr[1])
        st = w.wave2d_server_stats_get(sv)
        for i in sub_ids:
            w.wave2d_server_release(sv, i)
    finally:
        w.wave2d_server_destroy(sv)
    return {"workload": "Poisson arrivals of requests: sides 64-4096, schemes 5/9/13, 100-5000 levels, "
                        "compensated FP32, FP64 results",
            "requests": n_meas, "warmup_requests": n_warm, "qps": round(qps, 2),
            "saturation_glups": round(sat, 1), "value": round(lup_meas / (t_last - t_first) / 1e9, 1),
            "unit": "GLUP/s", "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "mean_ms": round(float(lat.mean()) * 1e3, 2), "makespan_s": round(makespan, 2),
            "quanta": st["quanta"], "max_rel_err_vs_gpu_fp64_sampled": worst, "sample": "every 50th request"}


def main():
    args = parse()
    if args.mode == "summarize":
        summarize(args.prof_dir)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU decomposition is a design note, not part of this build)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1904_04048_amd as w
    from paper_1904_04048_amd import workloads as W

    dev = torch.device("cuda:0")
    p = W.c2()
    u0, v0 = p.data()
    U0 = torch.from_numpy(u0).to(dev)
    V0 = torch.from_numpy(v0).to(dev)
    shape = (p.ny, p.nx)
    u = torch.empty(shape, dtype=torch.float32, device=dev)
    lo, d = torch.empty_like(u), torch.empty_like(u)
    work = torch.empty(w.wave2d_work_bytes(w.F32C, p.nx, p.ny), dtype=torch.uint8, device=dev)
    work64 = torch.empty(w.wave2d_work_bytes(w.F64, p.nx, p.ny), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    depth, rows = w.wave2d_get_tuning(w.F32C, p.scheme, p.nx, p.ny)
    kernel_cfg = {"kernel": KERNEL_NAME, "depth": depth, "rows": rows, "grid": [p.nx, p.ny],
                  "source": kernel_source_hash()}

    if args.mode == "profile":
        # Copy calibration for the memory counters, then the dominant kernel.
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)  # 256 MiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        w.wave2d_f32c_run(U0, V0, u, lo, d, p.h, p.tau, p.c, p.scheme, 1, work=work)
        w.wave2d_f32c_step(u, lo, d, p.h, p.tau, p.c, p.scheme, depth * 6, work=work)
        torch.cuda.synchronize()
        print(json.dumps({"profile": "done", "kernel_cfg": kernel_cfg, "copy_bytes": 2 * a.numel() * 4}))
        return

    # FP64 reference solve on the GPU (also the plain FP64 path's throughput).
    UP, UC = torch.empty_like(U0), torch.empty_like(U0)
    w.wave2d_run(U0, V0, UP, UC, p.h, p.tau, p.c, p.scheme, p.steps, work=work64)
    torch.cuda.synchronize()
    t64s = []
    for _ in range(3):
        t0 = time.perf_counter()
        w.wave2d_run(U0, V0, UP, UC, p.h, p.tau, p.c, p.scheme, p.steps, work=work64)
        torch.cuda.synchronize()
        t64s.append(time.perf_counter() - t0)
    t64 = sorted(t64s)[1]  # median of three solves
    ref = UC

    def one_solve():
        w.wave2d_f32c_run(U0, V0, u, lo, d, p.h, p.tau, p.c, p.scheme, p.steps, work=work)
        return w.wave2d_f32c_norms(u, lo, ref)  # synchronous

    for _ in range(args.warmup):
        one_solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nr = one_solve()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = elapsed / args.steps * 1e3
    glups = p.lup * args.steps / elapsed / 1e9
    err_fp64 = nr[0] / nr[1]

    U_ex = torch.from_numpy(exact_c2(p, p.steps)).to(dev)
    ne = w.wave2d_f32c_norms(u, lo, U_ex)
    err_exact = ne[0] / ne[1]

    # Dominant kernel: average launch time of the temporally blocked step
    # kernel, from events on the stream it is launched on.  The same L
    # launches run once untimed first: the host work just above leaves the
    # device idle long enough for its clocks to drop, and a short warm-up
    # measured ~8% slower passes than the solves (162 vs 150 us at 4097^2).
    L = max(2, args.kernel_launches - args.kernel_launches % 2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w.wave2d_f32c_step(u, lo, d, p.h, p.tau, p.c, p.scheme, depth * L, work=work)
    e0.record(stream)
    w.wave2d_f32c_step(u, lo, d, p.h, p.tau, p.c, p.scheme, depth * L, work=work)
    e1.record(stream)
    torch.cuda.synchronize()
    t_launch = e0.elapsed_time(e1) / 1e3 / L
    nodes = p.nx * p.ny
    alg_bytes = STATE_BYTES_PER_NODE * nodes
    achieved_gbs = alg_bytes / t_launch / 1e9
    kernel_glups = p.interior * depth / t_launch / 1e9
    traffic = traffic_record(kernel_cfg)
    # The pass is bound by vector instruction issue (SQ counters: the SIMDs
    # issue VALU work on 77% of the kernel's cycles), not by HBM: it advances
    # `depth` levels per read of the state.
    lup_launch = p.interior * depth
    achieved_tflops = FLOPS_PER_LUP_F32C_9PT * lup_launch / t_launch / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved_tflops, 2), "peak": round(VALU_PEAK_TFLOPS, 1),
                "unit": "TFLOP/s", "frac": round(achieved_tflops / VALU_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": kernel_cfg["kernel"], "depth": depth, "rows": rows,
                "launch_us": round(t_launch * 1e6, 2), "kernel_glups": round(kernel_glups, 1),
                "flops_per_lup": FLOPS_PER_LUP_F32C_9PT, "lup_per_launch": lup_launch,
                "hbm": {"achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": alg_bytes,
                        "traffic_gbs": round(traffic / t_launch / 1e9, 1) if traffic else None,
                        "single_level_equiv_gbs": round(kernel_glups * 24, 1)}}

    out = {
        "metric": METRIC, "value": round(glups, 2), "unit": "GLUP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "9-point, 4097x4097, 2000 levels, compensated FP32 (FP64 first step and norms)",
                   "scheme": p.scheme, "nx": p.nx, "ny": p.ny, "steps_per_solve": p.steps,
                   "lambda": p.lam, "lup_per_solve": p.lup, "parallelism": "single GPU"},
        "error": {"max_rel_vs_gpu_fp64": err_fp64, "max_rel_vs_exact_pde": err_exact},
        "fp64_path": {"value": round(p.lup / t64 / 1e9, 2), "unit": "GLUP/s", "ms_per_solve": round(t64 * 1e3, 2),
                      "depth": w.wave2d_get_tuning(w.F64, p.scheme, p.nx, p.ny)[0]},
        "roofline": roofline,
    }
    del u, lo, d, work, work64, UP, UC, U_ex
    torch.cuda.empty_cache()
    out["other_workloads"] = other_workloads()
    if not args.no_batch:
        out["batch"] = batch_bench(args)
        torch.cuda.empty_cache()
    if not args.no_serve:
        out["serving"] = serve_bench(args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, u0, v0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

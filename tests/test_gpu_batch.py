"""GPU tests of batches and the autotuner.

A batch advances many uneven instances with shared launches; each instance's
final state must be bit-identical to the same solve run alone
(wave2d_f32c_run), both when the batch is enqueued directly and when it is
replayed as a captured graph (several replays, with unrelated eager work and
synchronizations between them).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1904_04048_amd as w
from tests.gpu_util import smooth_data

pytestmark = pytest.mark.gpu

# (nx, ny, scheme, steps, flags, lambda fraction)
CASES = [
    (5, 7, w.P5, 3, 0, 0.9), (64, 64, w.P9, 1, 0, 0.5), (131, 97, w.P13, 20, 0, 0.9),
    (300, 257, w.P9, 33, 0, 0.9), (97, 300, w.P5, 12, w.FIRST_CONVENTIONAL, 0.7),
    (257, 257, w.C9, 17, w.FIRST_CONVENTIONAL, 0.8), (70, 450, w.P13, 9, 0, 0.6),
    (400, 130, w.P9, 2, 0, 0.3), (33, 33, w.P13, 40, 0, 0.95), (513, 300, w.P5, 25, 0, 0.9),
]


def _make(cases, seed=0):
    dev = torch.device("cuda:0")
    out = []
    for k, (nx, ny, scheme, steps, flags, frac) in enumerate(cases):
        (u0, v0), _ = smooth_data(nx, ny, seed + k)
        h = 1.0 / (max(nx, ny) - 1)
        tau = frac * w.wave2d_lambda_max(scheme) * h
        t = dict(nx=nx, ny=ny, h=h, tau=tau, c=1.0, scheme=scheme, steps=steps, flags=flags,
                 u0=torch.from_numpy(u0).to(dev), v0=torch.from_numpy(v0).to(dev),
                 u=torch.full((ny, nx), float("nan"), dtype=torch.float32, device=dev))
        t["lo"] = torch.full_like(t["u"], float("nan"))
        t["d"] = torch.full_like(t["u"], float("nan"))
        out.append(t)
    return out


def _solo(t):
    u = torch.empty_like(t["u"])
    lo, d = torch.empty_like(u), torch.empty_like(u)
    w.wave2d_f32c_run(t["u0"], t["v0"], u, lo, d, t["h"], t["tau"], t["c"], t["scheme"], t["steps"], t["flags"])
    return u, lo, d


@pytest.mark.parametrize("graph", [False, True])
def test_batch_bitwise_equals_solo(graph):
    insts = _make(CASES)
    refs = [_solo(t) for t in insts]
    b = w.wave2d_batch_create(insts, w.BATCH_GRAPH if graph else 0)
    try:
        st = w.wave2d_batch_stats_get(b)
        assert st["instances"] == len(CASES)
        assert st["lup"] == sum((nx - 2) * (ny - 2) * s for (nx, ny, _, s, _, _) in CASES)
        for rep in range(3 if graph else 1):
            for t in insts:
                t["u"].fill_(float("nan"))
                t["lo"].zero_()
                t["d"].zero_()
            torch.cuda.synchronize()
            w.wave2d_batch_run(b)
            torch.cuda.synchronize()
            for t, (u, lo, d) in zip(insts, refs):
                assert torch.equal(t["u"], u) and torch.equal(t["lo"], lo) and torch.equal(t["d"], d), rep
            # unrelated eager work between replays
            x = torch.randn(1000, 1000, device="cuda")
            (x @ x).sum().item()
    finally:
        w.wave2d_batch_destroy(b)


def test_batch_tall_segments_bitwise():
    # Enough work items per launch that taller segments than the tuned
    # floor are taken; results stay bit-identical to solo solves.
    cases = [(513, 385, (w.P5, w.P9, w.P13)[k % 3], 13 + k % 5, 0, 0.9) for k in range(48)]
    insts = _make(cases, seed=30)
    for s in (w.P5, w.P9, w.P13):
        w.wave2d_set_tuning(w.F32C, s, 3 if s == w.P13 else 6, 8)
    try:
        b = w.wave2d_batch_create(insts)
    finally:
        for s in (w.P5, w.P9, w.P13):
            w.wave2d_set_tuning(w.F32C, s)
    try:
        st = w.wave2d_batch_stats_get(b)
        assert st["items"] > 0 and st["item_rows"] / st["items"] > 8
        w.wave2d_batch_run(b)
        torch.cuda.synchronize()
    finally:
        w.wave2d_batch_destroy(b)
    for t in insts:
        u, lo, d = _solo(t)
        assert torch.equal(t["u"], u) and torch.equal(t["lo"], lo) and torch.equal(t["d"], d)


def test_batch_accuracy_against_oracle():
    insts = _make(CASES[:4], seed=10)
    b = w.wave2d_batch_create(insts)
    try:
        w.wave2d_batch_run(b)
        torch.cuda.synchronize()
    finally:
        w.wave2d_batch_destroy(b)
    for t in insts:
        _, ref = oracle.run(t["u0"].cpu().numpy(), t["v0"].cpu().numpy(), t["h"], t["tau"], 1.0, t["scheme"],
                            t["steps"], t["flags"])
        got = t["u"].double().cpu().numpy() + t["lo"].double().cpu().numpy()
        assert oracle.rel_max_err(got, ref) <= 1e-5


def test_batch_rejects_bad_instance_and_overlap():
    insts = _make(CASES[:3], seed=20)
    bad = dict(insts[1])
    bad["tau"] = 2.0 * bad["h"]
    with pytest.raises(w.Wave2dError):
        w.wave2d_batch_create([insts[0], bad])
    dup = dict(insts[0])  # same state arrays as insts[0]
    with pytest.raises(w.Wave2dError):
        w.wave2d_batch_create([insts[0], dup])


@pytest.mark.parametrize("prec", [w.F64, w.F32C])
@pytest.mark.parametrize("scheme", [w.P9, w.P13])
def test_autotune_picks_supported_shape_and_keeps_results(prec, scheme):
    try:
        depth, rows = w.wave2d_autotune(prec, scheme, 300, 257)
        assert depth in (1, 2, 3, 4, 6, 8) and rows >= 1
        assert w.wave2d_get_tuning(prec, scheme, 300, 257) == (depth, rows)
        if rows >= 8:
            assert w.wave2d_get_tuning(prec, scheme) == (depth, rows)
        else:
            # a short-segment pick stays with its grid size
            assert w.wave2d_get_tuning(prec, scheme)[1] >= 8
        (u0, v0), _ = smooth_data(300, 257, 3)
        U0 = torch.from_numpy(u0).cuda()
        V0 = torch.from_numpy(v0).cuda()
        h = 1.0 / 299
        tau = 0.9 * w.wave2d_lambda_max(scheme) * h
        if prec == w.F64:
            a = [torch.empty_like(U0) for _ in range(4)]
            w.wave2d_run(U0, V0, a[0], a[1], h, tau, 1.0, scheme, 19)
            w.wave2d_run(U0, V0, a[2], a[3], h, tau, 1.0, scheme, 19, w.KERNEL_SIMPLE)
            assert torch.equal(a[0], a[2]) and torch.equal(a[1], a[3])
        else:
            a = [torch.empty(U0.shape, dtype=torch.float32, device="cuda") for _ in range(6)]
            w.wave2d_f32c_run(U0, V0, a[0], a[1], a[2], h, tau, 1.0, scheme, 19)
            w.wave2d_f32c_run(U0, V0, a[3], a[4], a[5], h, tau, 1.0, scheme, 19, w.KERNEL_SIMPLE)
            assert all(torch.equal(a[k], a[k + 3]) for k in range(3))
    finally:
        w.wave2d_set_tuning(prec, scheme)


# Instances with enough levels that most passes run in the persistent
# launch (full passes of 8 levels, 6 for 13 points), plus remainders.
PCASES = [(nx, ny, (w.P5, w.P9, w.P13, w.C9)[k % 4], st, w.FIRST_CONVENTIONAL if k % 4 == 3 else 0, fr)
          for k, (nx, ny, st, fr) in enumerate([
              (64, 64, 101, 0.9), (640, 517, 77, 0.8), (129, 700, 150, 0.9), (300, 300, 64, 0.5),
              (97, 65, 203, 0.95), (1025, 257, 49, 0.9), (513, 513, 90, 0.7), (66, 1100, 31, 0.9),
              (200, 130, 121, 0.6), (777, 333, 58, 0.9), (45, 45, 300, 0.9), (1100, 90, 40, 0.85)])]


def _clear(insts):
    for t in insts:
        t["u"].fill_(float("nan"))
        t["lo"].fill_(float("nan"))
        t["d"].fill_(float("nan"))
    torch.cuda.synchronize()


@pytest.mark.parametrize("graph", [False, True])
def test_persistent_batch_bitwise_equals_rounds_and_solo(graph):
    insts = _make(PCASES, seed=40)
    refs = [_solo(t) for t in insts]
    bp = w.wave2d_batch_create(insts, w.BATCH_GRAPH if graph else 0)
    br = w.wave2d_batch_create(insts, w.BATCH_ROUNDS)
    try:
        sp = w.wave2d_batch_stats_get(bp)
        sr = w.wave2d_batch_stats_get(br)
        print(f"persistent: {sp}\nrounds: {sr}", flush=True)
        assert sp["persistent_items"] > 0 and sr["persistent_items"] == 0
        assert sp["launches"] < sr["launches"] and sp["lup"] == sr["lup"]
        for rep in range(3 if graph else 1):
            _clear(insts)
            w.wave2d_batch_run(bp)
            torch.cuda.synchronize()
            assert w.wave2d_batch_stats_get(bp)["stalled_waits"] == 0
            for k, (t, (u, lo, d)) in enumerate(zip(insts, refs)):
                assert torch.equal(t["u"], u) and torch.equal(t["lo"], lo) and torch.equal(t["d"], d), (rep, k)
            x = torch.randn(1000, 1000, device="cuda")
            (x @ x).sum().item()
        _clear(insts)
        w.wave2d_batch_run(br)
        torch.cuda.synchronize()
        for k, (t, (u, lo, d)) in enumerate(zip(insts, refs)):
            assert torch.equal(t["u"], u) and torch.equal(t["lo"], lo) and torch.equal(t["d"], d), k
    finally:
        w.wave2d_batch_destroy(bp)
        w.wave2d_batch_destroy(br)


def test_persistent_batch_wait_limit_ends_the_launch(monkeypatch):
    # A wait limit of zero polls (set from the host) makes items whose
    # previous pass is still running give up: the launch must still end,
    # and the batch must report the stalled waits.
    insts = _make([(1025, 1025, w.P9, 50, 0, 0.9)], seed=50)
    monkeypatch.setenv("WAVE2D_BATCH_WAIT_MS", "0")
    b = w.wave2d_batch_create(insts)
    monkeypatch.delenv("WAVE2D_BATCH_WAIT_MS")
    try:
        assert w.wave2d_batch_stats_get(b)["persistent_items"] > 0
        w.wave2d_batch_run(b)
        torch.cuda.synchronize()
        assert w.wave2d_batch_stats_get(b)["stalled_waits"] > 0
    finally:
        w.wave2d_batch_destroy(b)
    # A batch created afterwards uses the normal limit and is exact.
    b = w.wave2d_batch_create(insts)
    try:
        _clear(insts)
        w.wave2d_batch_run(b)
        torch.cuda.synchronize()
        assert w.wave2d_batch_stats_get(b)["stalled_waits"] == 0
    finally:
        w.wave2d_batch_destroy(b)
    u, lo, d = _solo(insts[0])
    assert torch.equal(insts[0]["u"], u) and torch.equal(insts[0]["lo"], lo) and torch.equal(insts[0]["d"], d)


def test_persistent_batch_autotune_keeps_results():
    # Autotuning re-plans the persistent tables for each candidate segment
    # height (queue membership follows the work model, so every per-queue
    # table changes); the batch must stay exact after it, eager and replayed.
    insts = _make(PCASES, seed=60)
    refs = [_solo(t) for t in insts]
    b = w.wave2d_batch_create(insts, w.BATCH_GRAPH)
    try:
        cap = w.wave2d_batch_autotune(b)
        assert cap in (64, 96, 128, 160, 224, 320, 512)
        st = w.wave2d_batch_stats_get(b)
        assert st["stalled_waits"] == 0 and st["last_persistent_ms"] > 0
        for rep in range(2):
            _clear(insts)
            w.wave2d_batch_run(b)
            torch.cuda.synchronize()
            assert w.wave2d_batch_stats_get(b)["stalled_waits"] == 0
            for k, (t, (u, lo, d)) in enumerate(zip(insts, refs)):
                assert torch.equal(t["u"], u) and torch.equal(t["lo"], lo) and torch.equal(t["d"], d), (rep, k)
    finally:
        w.wave2d_batch_destroy(b)
    # The tuned height applied to another batch of the same instances, and
    # other heights down to the smallest accepted, keep the results.
    b = w.wave2d_batch_create(insts, w.BATCH_GRAPH)
    try:
        with pytest.raises(w.Wave2dError):
            w.wave2d_batch_set_rows_cap(b, 7)
        with pytest.raises(w.Wave2dError):
            w.wave2d_batch_set_rows_cap(b, 4097)
        for c in (cap, 8, 1000):
            w.wave2d_batch_set_rows_cap(b, c)
            _clear(insts)
            w.wave2d_batch_run(b)
            torch.cuda.synchronize()
            assert w.wave2d_batch_stats_get(b)["stalled_waits"] == 0
            for k, (t, (u, lo, d)) in enumerate(zip(insts, refs)):
                assert torch.equal(t["u"], u) and torch.equal(t["lo"], lo) and torch.equal(t["d"], d), (c, k)
    finally:
        w.wave2d_batch_destroy(b)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_persistent_batch_random_mixes(seed):
    # Random mixes of sizes (including grids narrower than one strip and
    # taller than several segments), schemes, periodic instances, step
    # counts and segment heights: the persistent plan must equal the rounds
    # plan bit for bit, with no stalled waits.
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(14):
        nx = int(rng.integers(8, 700)) & ~1 if k % 3 == 0 else int(rng.integers(5, 700))
        ny = int(rng.integers(5, 900))
        scheme = (w.P5, w.P9, w.P13, w.C9)[int(rng.integers(0, 4))]
        steps = int(rng.integers(1, 120))
        cases.append((nx, ny, scheme, steps, w.FIRST_CONVENTIONAL if scheme == w.C9 else 0,
                      float(rng.uniform(0.3, 0.95))))
    insts = _make(cases, seed=100 + seed)
    # every third instance of even width runs on the periodic rule
    for k, t in enumerate(insts):
        if k % 3 == 0 and t["nx"] % 2 == 0 and t["nx"] >= 5 and t["ny"] >= 5:
            t["flags"] |= w.PERIODIC
    br = w.wave2d_batch_create(insts, w.BATCH_ROUNDS)
    try:
        _clear(insts)
        w.wave2d_batch_run(br)
        torch.cuda.synchronize()
        refs = [(t["u"].clone(), t["lo"].clone(), t["d"].clone()) for t in insts]
    finally:
        w.wave2d_batch_destroy(br)
    bp = w.wave2d_batch_create(insts)
    try:
        for cap in (int(rng.integers(8, 64)), 160, 777):
            w.wave2d_batch_set_rows_cap(bp, cap)
            _clear(insts)
            print(f"random mix seed {seed} rows cap {cap}", flush=True)
            w.wave2d_batch_run(bp)
            torch.cuda.synchronize()
            assert w.wave2d_batch_stats_get(bp)["stalled_waits"] == 0
            for k, (t, (u, lo, d)) in enumerate(zip(insts, refs)):
                assert torch.equal(t["u"], u) and torch.equal(t["lo"], lo) and torch.equal(t["d"], d), (cap, k)
    finally:
        w.wave2d_batch_destroy(bp)


def test_full_batch_repeats_bitwise():
    """The 512-instance batch of the benchmark (persistent launches, all
    three classes concurrently): ten runs give the first run's bits in every
    instance, outputs cleared to NaN before each run."""
    from paper_1904_04048_amd import workloads as W
    dev = torch.device("cuda:0")
    insts = []
    for pr in W.c4():
        U0, V0 = W.sine_series_torch(pr.nx, pr.ny, pr.modes, dev)
        u = torch.empty((pr.ny, pr.nx), dtype=torch.float32, device=dev)
        insts.append(dict(nx=pr.nx, ny=pr.ny, h=pr.h, tau=pr.tau, c=pr.c, scheme=pr.scheme, steps=pr.steps,
                          flags=0, u0=U0, v0=V0, u=u, lo=torch.empty_like(u), d=torch.empty_like(u)))
    bt = w.wave2d_batch_create(insts)
    try:
        w.wave2d_batch_run(bt)
        torch.cuda.synchronize()
        ref = [[t[k].clone() for k in ("u", "lo", "d")] for t in insts]
        for run in range(10):
            for t in insts:
                for k in ("u", "lo", "d"):
                    t[k].fill_(float("nan"))
            w.wave2d_batch_run(bt)
            torch.cuda.synchronize()
            for i, (t, r) in enumerate(zip(insts, ref)):
                assert all(torch.equal(t[k], x) for k, x in zip(("u", "lo", "d"), r)), (run, i)
            print(f"full batch run {run}: bitwise equal", flush=True)
    finally:
        w.wave2d_batch_destroy(bt)

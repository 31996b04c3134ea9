// Batches of compensated-FP32 solves and the launch-shape autotuner.
//
// A batch is planned once: instances are grouped by stencil class and tuned
// launch shape, and the run is cut into rounds.  In every round each
// unfinished instance advances by one pass of up to its class's depth; all
// instances of a class that take the same depth share one launch of the
// batched streaming kernels (their work items form one index space, so
// small and large grids load-balance inside the launch).  Boundary-strip
// items run on a side stream beside the interior items.  The tables of
// every launch are built on the host and uploaded once; with
// WAVE2D_BATCH_GRAPH the whole sequence is captured into one hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "host.h"

using namespace w2d;
using namespace w2d_host;

namespace {

struct Launch {
    int kind, depth;
    bool interior;
    size_t items_off, prefix_off;
    int count, total;
};

struct Round {
    size_t first, last;  // launches [first, last)
};

struct InstRec {
    Params p;
    wave2d_instance in;
    FirstW fw;
    float *bu, *bl, *bd;  // second state
    bool ends_in_b;
};

}  // namespace

struct wave2d_batch {
    int device = 0;
    uint32_t flags = 0;
    std::vector<InstRec> inst;
    std::vector<Launch> launches;
    std::vector<Round> rounds;
    void* tables = nullptr;
    size_t tables_bytes = 0;
    void* work = nullptr;
    size_t work_bytes = 0;
    wave2d_batch_stats st{};
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t capture = nullptr;  // private stream the graph is captured on
};

namespace {

int largest_supported(int d)
{
    static const int sup[] = {8, 6, 4, 3, 2, 1};
    for (int v : sup)
        if (v <= d && stream_depth_supported(v)) return v;
    return 1;
}

int enqueue(wave2d_batch* b, hipStream_t s)
{
    // First steps (fused with the state split), one launch per instance.
    for (const InstRec& r : b->inst)
        W2D_HIP(simple_first_step_f32c(r.p.g, r.p.kind, r.fw, r.in.u0, r.in.v0, r.in.u, r.in.lo, r.in.d, s));
    const Fork* fk = nullptr;
    int rc;
    if ((rc = side_of(s, &fk))) return rc;
    const char* base = (const char*)b->tables;
    for (const Round& rd : b->rounds) {
        bool any_gen = false;
        for (size_t k = rd.first; k < rd.last; ++k) any_gen |= !b->launches[k].interior;
        if (any_gen) {
            W2D_HIP(hipEventRecord(fk->ev_fork, s));
            W2D_HIP(hipStreamWaitEvent(fk->side, fk->ev_fork, 0));
        }
        for (size_t k = rd.first; k < rd.last; ++k) {
            const Launch& L = b->launches[k];
            W2D_HIP(batch_launch(WAVE2D_F32C, L.kind, L.depth, L.interior, base + L.items_off,
                                 (const int*)(base + L.prefix_off), L.count, L.total, L.interior ? s : fk->side));
        }
        if (any_gen) {
            W2D_HIP(hipEventRecord(fk->ev_join, fk->side));
            W2D_HIP(hipStreamWaitEvent(s, fk->ev_join, 0));
        }
    }
    for (const InstRec& r : b->inst)
        if (r.ends_in_b) W2D_HIP(copy_f32x3(r.p.g, r.bu, r.bl, r.bd, r.in.u, r.in.lo, r.in.d, s));
    return WAVE2D_OK;
}

}  // namespace

extern "C" {

int wave2d_batch_create(const wave2d_instance* inst, int64_t count, uint32_t flags, wave2d_batch** out)
{
    if (!out) return fail(WAVE2D_EINVAL, "out is NULL");
    *out = nullptr;
    if (!inst || count < 1 || count > (1 << 20)) return fail(WAVE2D_EINVAL, "need 1..2^20 instances");
    if (flags & ~WAVE2D_BATCH_GRAPH) return fail(WAVE2D_EINVAL, "unknown batch flag bits 0x%x", flags);
    wave2d_batch* b = new wave2d_batch();
    b->flags = flags;
    int r;
    if ((r = get_device(&b->device))) {
        delete b;
        return r;
    }
    // Validate every instance and check that no two arrays of the batch overlap.
    std::vector<std::pair<const char*, size_t>> spans;
    for (int64_t i = 0; i < count; ++i) {
        const wave2d_instance& in = inst[i];
        InstRec rec{};
        rec.in = in;
        if ((r = validate(in.nx, in.ny, in.ld, in.h, in.tau, in.c, in.scheme,
                          in.flags & ~(uint32_t)WAVE2D_KERNEL_SIMPLE, &rec.p))) {
            delete b;
            return fail(r, "instance %lld: %s", (long long)i, wave2d_last_error());
        }
        if (in.steps < 1) {
            delete b;
            return fail(WAVE2D_EINVAL, "instance %lld: steps must be >= 1", (long long)i);
        }
        if (!stream_ok(rec.p.g, sizeof(float))) {
            delete b;
            return fail(WAVE2D_EINVAL, "instance %lld: periodic batch instances need an even nx and ld*ny*4 < 2^31",
                        (long long)i);
        }
        if ((r = check_ptrs(rec.p.g, {{in.u0, 8}, {in.v0, 8}, {in.u, 4}, {in.lo, 4}, {in.d, 4}}))) {
            delete b;
            return fail(r, "instance %lld: %s", (long long)i, wave2d_last_error());
        }
        rec.fw = first_w(rec.p, in.flags, in.tau);
        spans.push_back({(const char*)in.u, grid_bytes(rec.p.g, 4)});
        spans.push_back({(const char*)in.lo, grid_bytes(rec.p.g, 4)});
        spans.push_back({(const char*)in.d, grid_bytes(rec.p.g, 4)});
        b->inst.push_back(rec);
    }
    std::sort(spans.begin(), spans.end());
    for (size_t k = 1; k < spans.size(); ++k)
        if (spans[k - 1].first + spans[k - 1].second > spans[k].first) {
            delete b;
            return fail(WAVE2D_EINVAL, "state arrays of two batch instances overlap");
        }

    // Second state of every instance in one allocation.
    size_t wb = 0;
    std::vector<size_t> woff(b->inst.size());
    for (size_t i = 0; i < b->inst.size(); ++i) {
        woff[i] = wb;
        wb += 3 * align256((size_t)b->inst[i].p.g.ld * b->inst[i].p.g.ny * sizeof(float));
    }
    hipError_t e = hipMalloc(&b->work, wb);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return fail(WAVE2D_ENOMEM, "batch workspace of %zu bytes: %s", wb, hipGetErrorString(e));
    }
    b->work_bytes = wb;
    for (size_t i = 0; i < b->inst.size(); ++i) {
        InstRec& rc = b->inst[i];
        const size_t st = align256((size_t)rc.p.g.ld * rc.p.g.ny * sizeof(float));
        char* p0 = (char*)b->work + woff[i];
        rc.bu = (float*)p0;
        rc.bl = (float*)(p0 + st);
        rc.bd = (float*)(p0 + 2 * st);
    }

    // Classes: (stencil class, tuned depth, rows).
    struct Cls {
        int kind, depth, rows;
        std::vector<size_t> members;
    };
    std::vector<Cls> classes;
    for (size_t i = 0; i < b->inst.size(); ++i) {
        const InstRec& rc = b->inst[i];
        const wave2d_tuning tn = tuning_for(WAVE2D_F32C, rc.p.scheme, 0, 0);
        auto it = std::find_if(classes.begin(), classes.end(), [&](const Cls& c) {
            return c.kind == rc.p.kind && c.depth == tn.depth && c.rows == tn.rows;
        });
        if (it == classes.end()) {
            classes.push_back(Cls{rc.p.kind, tn.depth, tn.rows, {}});
            it = classes.end() - 1;
        }
        it->members.push_back(i);
    }

    // Rounds.
    std::vector<int64_t> left(b->inst.size());
    std::vector<bool> in_b(b->inst.size(), false);
    for (size_t i = 0; i < b->inst.size(); ++i) left[i] = b->inst[i].in.steps - 1;
    std::vector<unsigned char> host;
    auto align_host = [&]() { host.resize(align256(host.size())); };
    BatchTables gen, inr;
    int64_t lup = 0, sbytes = 0;
    for (const InstRec& rc : b->inst) {
        lup += (int64_t)(rc.p.g.nx - 2) * (rc.p.g.ny - 2) * rc.in.steps;
        sbytes += 12 * (int64_t)rc.p.g.nx * rc.p.g.ny;
    }
    for (;;) {
        Round rd{b->launches.size(), b->launches.size()};
        bool active = false;
        for (const Cls& c : classes) {
            std::map<int, std::vector<size_t>> by_depth;
            for (size_t i : c.members)
                if (left[i] > 0) by_depth[largest_supported((int)std::min<int64_t>(c.depth, left[i]))].push_back(i);
            for (auto& kv : by_depth) {
                const int dep = kv.first;
                std::vector<BatchInst> bi;
                for (size_t i : kv.second) {
                    const InstRec& rc = b->inst[i];
                    BatchInst x{};
                    x.g = rc.p.g;
                    x.kind = rc.p.kind;
                    const bool src_b = in_b[i];
                    x.in_w0 = src_b ? rc.bu : rc.in.u;
                    x.in_w1 = src_b ? rc.bl : rc.in.lo;
                    x.in_p = src_b ? rc.bd : rc.in.d;
                    x.out_w0 = src_b ? rc.in.u : rc.bu;
                    x.out_w1 = src_b ? rc.in.lo : rc.bl;
                    x.out_p = src_b ? rc.in.d : rc.bd;
                    x.w32 = step_w32(rc.p);
                    bi.push_back(x);
                    left[i] -= dep;
                    in_b[i] = !in_b[i];
                }
                batch_tables(WAVE2D_F32C, c.kind, dep, c.rows, bi, gen, inr);
                for (int pass = 0; pass < 2; ++pass) {
                    const BatchTables& t = pass ? inr : gen;
                    if (t.count == 0) continue;
                    Launch L{c.kind, dep, pass == 1, 0, 0, t.count, t.prefix.back()};
                    b->st.items += t.prefix.back();
                    b->st.item_rows += (int64_t)t.prefix.back() * t.rows;
                    align_host();
                    L.items_off = host.size();
                    host.insert(host.end(), t.items.begin(), t.items.end());
                    align_host();
                    L.prefix_off = host.size();
                    const unsigned char* pp = (const unsigned char*)t.prefix.data();
                    host.insert(host.end(), pp, pp + t.prefix.size() * sizeof(int));
                    b->launches.push_back(L);
                }
                active = true;
            }
        }
        rd.last = b->launches.size();
        if (!active) break;
        b->rounds.push_back(rd);
    }
    for (size_t i = 0; i < b->inst.size(); ++i) b->inst[i].ends_in_b = in_b[i];
    align_host();
    if (!host.empty()) {
        e = hipMalloc(&b->tables, host.size());
        if (e != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(b->work);
            delete b;
            return fail(WAVE2D_ENOMEM, "batch tables of %zu bytes: %s", host.size(), hipGetErrorString(e));
        }
        b->tables_bytes = host.size();
        e = hipMemcpy(b->tables, host.data(), host.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(b->tables);
            (void)hipFree(b->work);
            delete b;
            return hip_fail(e, "hipMemcpy(batch tables)");
        }
    }
    int64_t copies = 0;
    for (const InstRec& rc : b->inst) copies += rc.ends_in_b ? 1 : 0;
    b->st.instances = (int64_t)b->inst.size();
    b->st.rounds = (int64_t)b->rounds.size();
    b->st.launches = (int64_t)b->inst.size() + (int64_t)b->launches.size() + copies;
    b->st.lup = lup;
    b->st.state_bytes = sbytes;
    b->st.work_bytes = (int64_t)b->work_bytes;
    *out = b;
    return WAVE2D_OK;
}

int wave2d_batch_run(wave2d_batch* b, void* stream)
{
    if (!b) return fail(WAVE2D_EINVAL, "batch is NULL");
    hipStream_t s = (hipStream_t)stream;
    const Fork* fk = nullptr;
    if (!(b->flags & WAVE2D_BATCH_GRAPH)) {
        int rs = side_of(s, &fk);
        if (rs) return rs;
        return enqueue(b, s);
    }
    if (!b->exec) {
        // The caller's stream may be the null stream, which cannot be
        // captured: capture on a private stream and launch on the caller's.
        if (!b->capture) W2D_HIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
        int rs = side_of(b->capture, &fk);  // created outside the capture
        if (rs) return rs;
        W2D_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed));
        int r = enqueue(b, b->capture);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->capture, &g);
        if (r) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        b->graph = g;
        W2D_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    }
    W2D_HIP(hipGraphLaunch(b->exec, s));
    return WAVE2D_OK;
}

int wave2d_batch_stats_get(const wave2d_batch* b, wave2d_batch_stats* st)
{
    if (!b || !st) return fail(WAVE2D_EINVAL, "NULL argument");
    *st = b->st;
    return WAVE2D_OK;
}

int wave2d_batch_destroy(wave2d_batch* b)
{
    if (!b) return WAVE2D_OK;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->tables) (void)hipFree(b->tables);
    if (b->work) (void)hipFree(b->work);
    delete b;
    return WAVE2D_OK;
}

int wave2d_autotune(int precision, int scheme, int64_t nx, int64_t ny, void* stream, wave2d_tuning* best)
{
    if (precision != WAVE2D_F64 && precision != WAVE2D_F32C) return fail(WAVE2D_EINVAL, "unknown precision");
    if (!best) return fail(WAVE2D_EINVAL, "best is NULL");
    Params p;
    const double lam = 0.5 * wave2d_lambda_max(scheme);
    int r = validate(nx, ny, nx, 1.0, lam, 1.0, scheme, 0, &p);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)nx * ny;
    const size_t elt = precision == WAVE2D_F64 ? 8 : 4;
    const int nf = precision == WAVE2D_F64 ? 2 : 3;
    void* buf = nullptr;
    hipError_t e = hipMalloc(&buf, 2 * nf * align256(n * elt));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(WAVE2D_ENOMEM, "autotune scratch: %s", hipGetErrorString(e));
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    // Scratch and events are released on every return below.
    struct Release {
        void* buf;
        hipEvent_t* e0;
        hipEvent_t* e1;
        ~Release()
        {
            if (*e0) (void)hipEventDestroy(*e0);
            if (*e1) (void)hipEventDestroy(*e1);
            (void)hipFree(buf);
        }
    } release{buf, &e0, &e1};
    W2D_HIP(hipMemsetAsync(buf, 0, 2 * nf * align256(n * elt), s));
    char* c = (char*)buf;
    auto arr = [&](int k) { return (void*)(c + k * align256(n * elt)); };
    const Fork* fk = nullptr;
    if ((r = side_of(s, &fk))) return r;
    // Candidate shapes: every supported depth whose interior kernel keeps
    // its state in registers, with fixed segment heights plus the heights
    // at which the work items fill k/2 rounds of the resident wave slots.
    static const int depths[] = {1, 2, 3, 4, 6, 8};
    static const int rows_fixed[] = {8, 16, 24, 32, 48, 64};
    W2D_HIP(hipEventCreate(&e0));
    W2D_HIP(hipEventCreate(&e1));
    // Time per level of one shape over about `target_ms` (a short probe
    // sizes the run), ping-ponging between the two scratch states.
    auto time_shape = [&](int dep, int rows, float target_ms, float* per_level) -> int {
        const StreamShape sh{dep, rows, fk};
        auto pass = [&](int k) -> hipError_t {
            const int a = (k & 1) ? nf : 0, b2 = (k & 1) ? 0 : nf;
            if (precision == WAVE2D_F64)
                return stream_step_f64(p.g, p.kind, step_w64(p), sh, (const double*)arr(a), (const double*)arr(a + 1),
                                       (double*)arr(b2), (double*)arr(b2 + 1), s);
            return stream_step_f32c(p.g, p.kind, step_w32(p), sh, (const float*)arr(a), (const float*)arr(a + 1),
                                    (const float*)arr(a + 2), (float*)arr(b2), (float*)arr(b2 + 1), (float*)arr(b2 + 2),
                                    s);
        };
        auto timed = [&](int reps, float* ms) -> int {
            W2D_HIP(hipEventRecord(e0, s));
            for (int k = 0; k < reps; ++k) W2D_HIP(pass(k + 1));
            W2D_HIP(hipEventRecord(e1, s));
            W2D_HIP(hipEventSynchronize(e1));
            W2D_HIP(hipEventElapsedTime(ms, e0, e1));
            return WAVE2D_OK;
        };
        W2D_HIP(pass(0));
        float ms = 0.f;
        int rr;
        if ((rr = timed(2, &ms))) return rr;
        const int reps = std::min(256, std::max(2, (int)std::ceil(target_ms / std::max(ms / 2, 1e-3f))));
        if ((rr = timed(reps, &ms))) return rr;
        *per_level = ms / (reps * dep);
        return WAVE2D_OK;
    };
    struct Cand {
        float per_level;
        int depth, rows;
    };
    std::vector<Cand> timed_c;
    for (int dep : depths) {
        const ShapeFit fit = stream_shape_fit(precision, p.kind, dep);
        if (fit.spills || fit.slots < 1 || fit.strip_cols < 1) continue;
        const int64_t nstrips = (nx + fit.strip_cols - 1) / fit.strip_cols;
        std::vector<int> rows_c(std::begin(rows_fixed), std::end(rows_fixed));
        for (int k = 2; k <= 16; ++k) {
            const int64_t segs = (int64_t)k * fit.slots / (2 * nstrips);
            if (segs < 1) continue;
            const int64_t r = (ny + segs - 1) / segs;
            if (r >= 8 && r <= 256) rows_c.push_back((int)r);
        }
        std::sort(rows_c.begin(), rows_c.end());
        rows_c.erase(std::unique(rows_c.begin(), rows_c.end()), rows_c.end());
        for (int rows : rows_c) {
            if (rows > std::max<int64_t>(8, ny)) continue;
            float per_level = 0.f;
            if ((r = time_shape(dep, rows, 2.0f, &per_level))) return r;
            timed_c.push_back(Cand{per_level, dep, rows});
        }
    }
    // The few fastest shapes again, each timed over about 10 ms: single
    // 2 ms timings of shapes within a few percent of each other can rank
    // them wrongly.
    std::sort(timed_c.begin(), timed_c.end(), [](const Cand& a, const Cand& b) { return a.per_level < b.per_level; });
    float best_t = 1e30f;
    wave2d_tuning bt{1, 16};
    for (size_t k = 0; k < timed_c.size() && k < 4; ++k) {
        float per_level = 0.f;
        if ((r = time_shape(timed_c[k].depth, timed_c[k].rows, 10.0f, &per_level))) return r;
        if (per_level < best_t) {
            best_t = per_level;
            bt = wave2d_tuning{timed_c[k].depth, timed_c[k].rows};
        }
    }
    W2D_HIP(hipStreamSynchronize(s));
    set_tuning_entry(precision, scheme, bt);
    set_tuning_size_entry(precision, scheme, nx, ny, bt);
    save_tune_cache(precision, scheme, nx, ny, bt);
    *best = bt;
    return WAVE2D_OK;
}

}  // extern "C"

// Batches of compensated-FP32 solves and the launch-shape autotuner.
//
// A batch is planned once.  Every instance's levels after the first step
// are split into passes of its stencil class's depth plus a remainder; the
// remainder passes run first, in rounds of batched launches (all instances
// of a class taking the same depth share one launch whose work items form
// one index space), and all full-depth passes of all instances then run in
// ONE persistent launch: instances are pinned to the device's XCCs (L2
// domains) by a greedy balance of their work, each XCC works through its own
// queue of (instance, pass) tasks in pass-major order, and a wave waits only
// for the previous pass of its own instance (see k_stream_persist).  First
// steps, and the copies that leave each final state in the caller's
// arrays, are one launch each.  Tables are built on the host and uploaded
// once; with WAVE2D_BATCH_GRAPH the whole sequence is captured into one
// hipGraph.  WAVE2D_BATCH_ROUNDS runs every pass in rounds instead (the
// same passes, bit for bit).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
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

// A wait of the persistent kernels gives up after this long (100 MHz
// real-time clock ticks: 2 s; a healthy wait lasts at most a few item times,
// about a millisecond); a wait that gives up is counted, its item is
// skipped and every later wait of the launch gives up at once, so a launch
// always ends.  WAVE2D_BATCH_WAIT_MS overrides it (tests of that path).
constexpr long long kWaitTicks = 200000000LL;
constexpr int kClasses = kPersistClasses;  // stencil classes KIND5, KIND9, KIND13: one persistent launch each

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
    // One-launch parts of a run (offsets into `tables`).
    size_t first_recs = 0, first_prefix = 0;
    int first_count = 0, first_blocks = 0;
    size_t copy_recs = 0, copy_prefix = 0;
    int copy_count = 0, copy_blocks = 0;
    bool persist = false;
    // Per stencil class: whether it has persistent work, its queue offsets
    // and item counts, and its counter block (n_ctr ints each).
    size_t p_insts = 0, p_tasks = 0, p_qoff[kClasses] = {}, p_qn[kClasses] = {}, p_ctr[kClasses] = {};
    bool p_has[kClasses] = {};
    int n_ctr[kClasses] = {};         // counters per class: heads, stalls, tiles
    std::vector<int> tile_off;        // per instance, within its class's tile counters
    long long wait_ticks = kWaitTicks;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // around the persistent launches
    // The stencil classes' persistent launches run concurrently: the first
    // on the caller's stream, the others on two private streams forked from
    // it and joined back (a class that runs out of work leaves its CUs to
    // the others instead of idling through the tail of its queues).
    hipStream_t p_side[kClasses - 1] = {};
    hipEvent_t p_fork = nullptr, p_join[kClasses - 1] = {};
    bool ran = false;
    // Persistent plan inputs: full passes and the parity of the first one
    // per instance, and the tallest segment of a work item.
    std::vector<int64_t> full;
    std::vector<int> par0;
    int rows_cap = kPersistRowsCap;
    int64_t p_item_rows = 0;
};

namespace {

void release_streams(wave2d_batch* b)
{
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->p_fork) (void)hipEventDestroy(b->p_fork);
    for (int k = 0; k < kClasses - 1; ++k) {
        if (b->p_join[k]) (void)hipEventDestroy(b->p_join[k]);
        if (b->p_side[k]) (void)hipStreamDestroy(b->p_side[k]);
    }
    b->ev0 = b->ev1 = b->p_fork = nullptr;
}

int largest_supported(int d)
{
    static const int sup[] = {8, 6, 4, 3, 2, 1};
    for (int v : sup)
        if (v <= d && stream_depth_supported(v)) return v;
    return 1;
}

int plan_persist(const wave2d_batch* b, int cap, PersistPlan* pl)
{
    const size_t ni = b->inst.size();
    std::vector<PersistInput> in(ni);
    for (size_t i = 0; i < ni; ++i) {
        const InstRec& rc = b->inst[i];
        PersistInput& x = in[i];
        x.g = rc.p.g;
        x.kind = rc.p.kind;
        x.w = step_w32(rc.p);
        x.s0[0] = rc.in.u;
        x.s0[1] = rc.in.lo;
        x.s0[2] = rc.in.d;
        x.s1[0] = rc.bu;
        x.s1[1] = rc.bl;
        x.s1[2] = rc.bd;
        x.tile_off = b->tile_off[i];
        x.passes = b->full[i];
        x.par0 = b->par0[i];
    }
    return persist_plan(in, cap, pl);
}

// timing: record the batch's events around the persistent launches (not
// inside a graph capture: events recorded by graph nodes cannot be timed).
int enqueue(wave2d_batch* b, hipStream_t s, bool timing)
{
    char* base = (char*)b->tables;
    for (int c = 0; c < kClasses; ++c)
        if (b->p_has[c]) W2D_HIP(fill_i32((int*)(base + b->p_ctr[c]), b->n_ctr[c], 0, s));
    // First steps (fused with the state split) of every instance: one launch.
    W2D_HIP(first_step_f32c_batch((const FirstRecF32C*)(base + b->first_recs), (const int*)(base + b->first_prefix),
                                  b->first_count, b->first_blocks, s));
    const Fork* fk = nullptr;
    int rc;
    if (!b->rounds.empty() && (rc = side_of(s, &fk))) return rc;
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
    if (b->persist) {
        if (timing) W2D_HIP(hipEventRecord(b->ev0, s));
        W2D_HIP(hipEventRecord(b->p_fork, s));
        int used = 0;
        for (int c = kClasses - 1; c >= 0; --c) {
            if (!b->p_has[c]) continue;
            hipStream_t sc = s;
            if (used > 0) {
                sc = b->p_side[used - 1];
                W2D_HIP(hipStreamWaitEvent(sc, b->p_fork, 0));
            }
            W2D_HIP(persist_launch(c, base + b->p_insts, (const PersistTask*)(base + b->p_tasks),
                                   (const int*)(base + b->p_qoff[c]), (const int*)(base + b->p_qn[c]),
                                   (int*)(base + b->p_ctr[c]), b->wait_ticks, sc));
            if (used > 0) W2D_HIP(hipEventRecord(b->p_join[used - 1], sc));
            ++used;
        }
        for (int k = 0; k + 1 < used; ++k) W2D_HIP(hipStreamWaitEvent(s, b->p_join[k], 0));
        if (timing) W2D_HIP(hipEventRecord(b->ev1, s));
    }
    W2D_HIP(copy_f32x3_batch((const CopyRec3*)(base + b->copy_recs), (const int*)(base + b->copy_prefix),
                             b->copy_count, b->copy_blocks, s));
    return WAVE2D_OK;
}

// Re-plan the persistent tables for segments of at most `cap` rows and
// upload them in place (the layout does not depend on `cap`).  Queue
// membership follows the work model, which depends on the height, so every
// per-class table is rewritten.
int upload_plan(wave2d_batch* b, int cap, hipStream_t s)
{
    PersistPlan pl;
    int r = plan_persist(b, cap, &pl);
    if (r) return r;
    char* base = (char*)b->tables;
    W2D_HIP(hipStreamSynchronize(s));
    W2D_HIP(hipMemcpy(base + b->p_insts, pl.recs.data(), pl.recs.size(), hipMemcpyHostToDevice));
    W2D_HIP(hipMemcpy(base + b->p_tasks, pl.tasks.data(), pl.tasks.size() * sizeof(PersistTask),
                      hipMemcpyHostToDevice));
    for (int c = 0; c < kClasses; ++c) {
        W2D_HIP(hipMemcpy(base + b->p_qoff[c], pl.qoff[c].data(), pl.qoff[c].size() * sizeof(int),
                          hipMemcpyHostToDevice));
        W2D_HIP(hipMemcpy(base + b->p_qn[c], pl.qn[c].data(), pl.qn[c].size() * sizeof(int), hipMemcpyHostToDevice));
    }
    b->st.items += pl.items - b->st.persistent_items;
    b->st.item_rows += pl.item_rows - b->p_item_rows;
    b->st.persistent_items = pl.items;
    b->p_item_rows = pl.item_rows;
    b->rows_cap = cap;
    return WAVE2D_OK;
}

}  // namespace

extern "C" {

int wave2d_batch_create(const wave2d_instance* inst, int64_t count, uint32_t flags, wave2d_batch** out)
{
    if (!out) return fail(WAVE2D_EINVAL, "out is NULL");
    *out = nullptr;
    if (!inst || count < 1 || count > (1 << 20)) return fail(WAVE2D_EINVAL, "need 1..2^20 instances");
    if (flags & ~(WAVE2D_BATCH_GRAPH | WAVE2D_BATCH_ROUNDS))
        return fail(WAVE2D_EINVAL, "unknown batch flag bits 0x%x", flags);
    wave2d_batch* b = new wave2d_batch();
    b->flags = flags;
    int r;
    if ((r = get_device(&b->device))) {
        delete b;
        return r;
    }
    if (const char* e = std::getenv("WAVE2D_BATCH_WAIT_MS")) b->wait_ticks = std::max(0LL, 100000LL * std::atoll(e));
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
        if (rec.p.kind == KINDW) {
            delete b;
            return fail(WAVE2D_EINVAL,
                        "instance %lld: scheme %d reaches three lines out; batches take the 5-, 9- and 13-point "
                        "classes (run it with wave2d_f32c_run)",
                        (long long)i, in.scheme);
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

    const size_t ni = b->inst.size();
    b->persist = !(flags & WAVE2D_BATCH_ROUNDS) && xcc_layout_ok(b->device);
    // Levels after the first step: full passes of the persistent kernel's
    // depth (none in rounds mode) and a remainder run in rounds first.
    std::vector<int64_t> left(ni), full(ni, 0);
    for (size_t i = 0; i < ni; ++i) {
        const int64_t lv = b->inst[i].in.steps - 1;
        if (b->persist) {
            const int D = persist_depth(b->inst[i].p.kind);
            full[i] = lv / D;
            left[i] = lv - full[i] * D;
        } else {
            left[i] = lv;
        }
    }

    // Rounds classes: (stencil class, tuned depth, rows).
    struct Cls {
        int kind, depth, rows;
        std::vector<size_t> members;
    };
    std::vector<Cls> classes;
    for (size_t i = 0; i < ni; ++i) {
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

    std::vector<bool> in_b(ni, false);
    std::vector<unsigned char> host;
    auto align_host = [&]() { host.resize(align256(host.size())); };
    auto put = [&](const void* p, size_t n) {
        align_host();
        const size_t off = host.size();
        host.insert(host.end(), (const unsigned char*)p, (const unsigned char*)p + n);
        return off;
    };
    int64_t lup = 0, sbytes = 0;
    for (const InstRec& rc : b->inst) {
        lup += (int64_t)(rc.p.g.nx - 2) * (rc.p.g.ny - 2) * rc.in.steps;
        sbytes += 12 * (int64_t)rc.p.g.nx * rc.p.g.ny;
    }

    // First steps: one record per instance.
    {
        std::vector<FirstRecF32C> recs(ni);
        std::vector<int> prefix(1, 0);
        for (size_t i = 0; i < ni; ++i) {
            const InstRec& rc = b->inst[i];
            recs[i] = FirstRecF32C{rc.p.g, rc.p.kind, rc.fw, rc.in.u0, rc.in.v0, rc.in.u, rc.in.lo, rc.in.d};
            prefix.push_back(prefix.back() + node_tiles(rc.p.g));
        }
        b->first_recs = put(recs.data(), recs.size() * sizeof(FirstRecF32C));
        b->first_prefix = put(prefix.data(), prefix.size() * sizeof(int));
        b->first_count = (int)ni;
        b->first_blocks = prefix.back();
    }

    // Rounds of the remainder levels (all levels in rounds mode).
    BatchTables gen, inr;
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
                    L.items_off = put(t.items.data(), t.items.size());
                    L.prefix_off = put(t.prefix.data(), t.prefix.size() * sizeof(int));
                    b->launches.push_back(L);
                }
                active = true;
            }
        }
        rd.last = b->launches.size();
        if (!active) break;
        b->rounds.push_back(rd);
    }

    // The persistent launch: instance records, per-XCC task queues, and the
    // tile counters of each class (every instance of a class gets a block
    // sized for its smallest segments, so that re-planning for another
    // segment height keeps the layout).
    if (b->persist) {
        b->full = full;
        b->tile_off.assign(ni, 0);
        int64_t tiles[kClasses] = {};
        for (size_t i = 0; i < ni; ++i) {
            const int c = b->inst[i].p.kind;
            b->tile_off[i] = (int)tiles[c];
            tiles[c] += persist_max_tiles(b->inst[i].p.g, c);
        }
        for (int c = 0; c < kClasses; ++c) {
            if (kPersistTileBase + tiles[c] >= (int64_t(1) << 30)) {
                (void)hipFree(b->work);
                delete b;
                return fail(WAVE2D_EINVAL, "batch too large for one persistent launch (%lld tiles)", (long long)tiles[c]);
            }
            b->n_ctr[c] = kPersistTileBase + (int)tiles[c];
        }
        b->par0.assign(ni, 0);
        for (size_t i = 0; i < ni; ++i) {
            b->par0[i] = in_b[i] ? 1 : 0;
            if (full[i] & 1) in_b[i] = !in_b[i];
        }
        PersistPlan pl;
        if ((r = plan_persist(b, b->rows_cap, &pl))) {
            (void)hipFree(b->work);
            delete b;
            return r;
        }
        if (pl.tasks.empty()) {
            b->persist = false;
        } else {
            b->p_insts = put(pl.recs.data(), pl.recs.size());
            b->p_tasks = put(pl.tasks.data(), pl.tasks.size() * sizeof(PersistTask));
            for (int c = 0; c < kClasses; ++c) {
                b->p_has[c] = pl.qoff[c][kPersistQueues] > pl.qoff[c][0];
                b->p_qoff[c] = put(pl.qoff[c].data(), pl.qoff[c].size() * sizeof(int));
                b->p_qn[c] = put(pl.qn[c].data(), pl.qn[c].size() * sizeof(int));
                const std::vector<int> zeros((size_t)b->n_ctr[c], 0);
                b->p_ctr[c] = put(zeros.data(), zeros.size() * sizeof(int));
            }
            b->st.items += pl.items;
            b->st.item_rows += pl.item_rows;
            b->st.persistent_items = pl.items;
            b->p_item_rows = pl.item_rows;
            for (size_t i = 0; i < ni; ++i) {
                const Grid& g = b->inst[i].p.g;
                b->st.persistent_lup += full[i] * persist_depth(b->inst[i].p.kind) * (int64_t)(g.nx - 2) * (g.ny - 2);
                b->st.persistent_bytes += full[i] * 24 * (int64_t)g.nx * g.ny;
            }
            bool ok = hipEventCreate(&b->ev0) == hipSuccess && hipEventCreate(&b->ev1) == hipSuccess &&
                      hipEventCreateWithFlags(&b->p_fork, hipEventDisableTiming) == hipSuccess;
            for (int k = 0; ok && k < kClasses - 1; ++k)
                ok = hipStreamCreateWithFlags(&b->p_side[k], hipStreamNonBlocking) == hipSuccess &&
                     hipEventCreateWithFlags(&b->p_join[k], hipEventDisableTiming) == hipSuccess;
            if (!ok) {
                (void)hipGetLastError();
                release_streams(b);
                (void)hipFree(b->work);
                delete b;
                return fail(WAVE2D_EDEVICE, "batch streams and events");
            }
        }
    }

    // Copies of final states that ended in the second state: one launch.
    {
        std::vector<CopyRec3> recs;
        std::vector<int> prefix(1, 0);
        for (size_t i = 0; i < ni; ++i) {
            InstRec& rc = b->inst[i];
            rc.ends_in_b = in_b[i];
            if (!rc.ends_in_b) continue;
            recs.push_back(CopyRec3{rc.p.g, {rc.bu, rc.bl, rc.bd}, {rc.in.u, rc.in.lo, rc.in.d}});
            prefix.push_back(prefix.back() + node_tiles(rc.p.g));
        }
        b->copy_recs = put(recs.data(), recs.size() * sizeof(CopyRec3));
        b->copy_prefix = put(prefix.data(), prefix.size() * sizeof(int));
        b->copy_count = (int)recs.size();
        b->copy_blocks = prefix.back();
    }

    align_host();
    e = hipMalloc(&b->tables, host.size());
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release_streams(b);
        (void)hipFree(b->work);
        delete b;
        return fail(WAVE2D_ENOMEM, "batch tables of %zu bytes: %s", host.size(), hipGetErrorString(e));
    }
    b->tables_bytes = host.size();
    e = hipMemcpy(b->tables, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release_streams(b);
        (void)hipFree(b->tables);
        (void)hipFree(b->work);
        delete b;
        return hip_fail(e, "hipMemcpy(batch tables)");
    }
    b->st.instances = (int64_t)ni;
    b->st.rounds = (int64_t)b->rounds.size();
    b->st.launches = 1 + (int64_t)b->launches.size() + (b->persist ? 2 : 0) + (b->copy_count > 0 ? 1 : 0);
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
        const int r = enqueue(b, s, true);
        b->ran = b->ran || r == WAVE2D_OK;
        return r;
    }
    if (!b->exec) {
        // The caller's stream may be the null stream, which cannot be
        // captured: capture on a private stream and launch on the caller's.
        if (!b->capture) W2D_HIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
        int rs = side_of(b->capture, &fk);  // created outside the capture
        if (rs) return rs;
        W2D_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed));
        int r = enqueue(b, b->capture, false);
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
    st->stalled_waits = 0;
    if (b->persist) {
        // Waits of the last run that gave up (the run's results are then wrong).
        W2D_HIP(hipDeviceSynchronize());
        int v = 0;
        for (int c = 0; c < kClasses; ++c) {
            if (!b->p_has[c]) continue;
            W2D_HIP(hipMemcpy(&v, (const char*)b->tables + b->p_ctr[c] + kPersistStride * kPersistQueues * sizeof(int),
                              sizeof(int), hipMemcpyDeviceToHost));
            st->stalled_waits += v;
        }
        if (b->ran) {
            float ms = 0.f;
            W2D_HIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
            st->last_persistent_ms = ms;
        }
    }
    return WAVE2D_OK;
}

int wave2d_batch_autotune(wave2d_batch* b, void* stream, int32_t* rows_cap)
{
    if (!b) return fail(WAVE2D_EINVAL, "batch is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (!b->persist) {
        if (rows_cap) *rows_cap = 0;
        return WAVE2D_OK;
    }
    // Time whole runs (eager launches) with each candidate height, the
    // current one included, and keep the fastest.  The table layout does
    // not change, so a captured graph stays valid.
    static const int cand[] = {64, 96, 128, 160, 224, 320, 512};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    W2D_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(hipErrorOutOfMemory, "hipEventCreate");
    }
    struct Release {
        hipEvent_t a, b;
        ~Release()
        {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } rel{e0, e1};
    float best_ms = 1e30f;
    int best = b->rows_cap;
    int r;
    for (int cap : cand) {
        if ((r = upload_plan(b, cap, s))) return r;
        if ((r = enqueue(b, s, true))) return r;  // warm-up
        float tot = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
            W2D_HIP(hipEventRecord(e0, s));
            if ((r = enqueue(b, s, true))) return r;
            W2D_HIP(hipEventRecord(e1, s));
            W2D_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            W2D_HIP(hipEventElapsedTime(&ms, e0, e1));
            tot += ms;
        }
        if (tot < best_ms) {
            best_ms = tot;
            best = cap;
        }
    }
    if ((r = upload_plan(b, best, s))) return r;
    b->ran = true;
    if (rows_cap) *rows_cap = best;
    return WAVE2D_OK;
}

int wave2d_batch_set_rows_cap(wave2d_batch* b, int32_t rows_cap, void* stream)
{
    if (!b) return fail(WAVE2D_EINVAL, "batch is NULL");
    if (rows_cap < 8 || rows_cap > 4096) return fail(WAVE2D_EINVAL, "rows_cap %d outside 8..4096", (int)rows_cap);
    if (!b->persist) return WAVE2D_OK;
    return upload_plan(b, rows_cap, (hipStream_t)stream);
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
    release_streams(b);
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
    if (p.kind == KINDW) return fail(WAVE2D_EINVAL, "scheme %d runs one level per launch: no launch shape to tune", scheme);
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
    // Grids too small to fill the slots at 8-row segments also try 2 and 4
    // rows: there a pass lasts as long as one item, and a shorter segment
    // shortens the item (257^2 5-point FP64, 400 levels: 1.22 ms at depth 8
    // and 8 rows, 0.99 ms at 2 rows).
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
        if (nstrips * ((ny + 7) / 8) < fit.slots) {
            rows_c.push_back(2);
            rows_c.push_back(4);
        }
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
    // A pick of fewer than 8 rows only suits grids as small as this one: it
    // is kept for this size alone.
    if (bt.rows >= 8) set_tuning_entry(precision, scheme, bt);
    set_tuning_size_entry(precision, scheme, nx, ny, bt);
    save_tune_cache(precision, scheme, nx, ny, bt);
    *best = bt;
    return WAVE2D_OK;
}

}  // extern "C"

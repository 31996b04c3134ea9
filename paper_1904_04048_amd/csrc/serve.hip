// Serving: solve requests admitted as device memory allows and advanced
// together, one batched pass ("quantum") at a time, by a worker thread.
//
// Memory.  The server owns one device arena and hands out 256-byte aligned
// blocks first-fit from a free list kept on the host.  A request holds
// 32 bytes per node while active: its compensated state (12 B), the second
// state the passes ping-pong into (12 B) and the FP64 result (8 B).  Sine
// series initial data are sampled into the result block (u0) and the second
// state's block (v0), which the first step consumes before either is
// needed again.  When a request finishes, its two states return to the
// arena; the result block stays until the client releases it.
//
// Scheduling.  Requests are admitted in arrival order; one that does not fit
// waits while later ones that fit go ahead.  Every quantum advances each
// active request by one pass of up to its class's tuned depth; requests join
// and leave at quantum boundaries.  The pass tables of a quantum go through
// a small ring of pinned staging buffers to device slots; at most
// kRing quanta are in flight, so the host never runs far ahead of the GPU
// and newly arrived requests join promptly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "host.h"

using namespace w2d;
using namespace w2d_host;

namespace {

constexpr int kMaxModes = 64;
constexpr int kRing = 3;

struct ModeSet {
    int n;
    double m[kMaxModes][4];
};

__global__ __launch_bounds__(256) void k_sine_series(Grid g, ModeSet ms, double* __restrict__ u0,
                                                     double* __restrict__ v0)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63), j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= g.nx || j >= g.ny) return;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < ms.n; ++k) {
        const double e = sin(ms.m[k][0] * M_PI * i / (g.nx - 1)) * sin(ms.m[k][1] * M_PI * j / (g.ny - 1));
        a += ms.m[k][2] * e;
        b += ms.m[k][3] * e;
    }
    u0[(size_t)j * g.ld + i] = a;
    v0[(size_t)j * g.ld + i] = b;
}

hipError_t sine_series(const Grid& g, const ModeSet& ms, double* u0, double* v0, hipStream_t s)
{
    dim3 grid((g.nx + 63) / 64, (g.ny + 3) / 4);
    k_sine_series<<<grid, 256, 0, s>>>(g, ms, u0, v0);
    return hipGetLastError();
}

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) with coalescing free list.
class Arena {
public:
    void init(size_t size) { free_ = {{0, size}}; size_ = size; }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                it->first += bytes;
                it->second -= bytes;
                if (it->second == 0) free_.erase(it);
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align256(bytes);
        used_ -= bytes;
        auto it = free_.begin();
        while (it != free_.end() && it->first < off) ++it;
        it = free_.insert(it, {off, bytes});
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
                it = pv;
            }
        }
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

private:
    std::list<std::pair<size_t, size_t>> free_;
    size_t size_ = 0, used_ = 0;
};

enum ReqState { QUEUED, ACTIVE, FINISHING, DONE, FAILED };

struct Req {
    uint64_t id;
    wave2d_request rq;
    ModeSet modes;
    Params p;
    FirstW fw;
    std::atomic<int> st{QUEUED};  // read by poll() under the lock, written by the worker
    int status = WAVE2D_OK;
    size_t off_state = 0, bytes_state = 0, off_res = 0, bytes_res = 0;
    bool has_state = false, has_res = false;
    float *u = nullptr, *lo = nullptr, *d = nullptr, *bu = nullptr, *bl = nullptr, *bd = nullptr;
    double* res = nullptr;
    int64_t left = 0;
    bool in_b = false;
    hipEvent_t done_ev = nullptr;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct wave2d_server {
    int device = 0;
    char* base = nullptr;
    Arena arena;
    hipStream_t s = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stopping = false;
    uint64_t next_id = 1;
    std::map<uint64_t, Req*> reqs;
    std::deque<uint64_t> queue;
    std::vector<Req*> active;  // worker-owned
    wave2d_server_stats st{};
    // quantum table ring
    void* host_stage[kRing] = {};
    void* dev_tables[kRing] = {};
    size_t cap[kRing] = {};
    hipEvent_t ring_ev[kRing] = {};
    bool ring_used[kRing] = {};
    int ring_next = 0;
};

namespace {

size_t state_bytes(const Grid& g) { return 6 * align256((size_t)g.ld * g.ny * sizeof(float)); }
size_t result_bytes(const Grid& g) { return align256((size_t)g.ld * g.ny * sizeof(double)); }

// Worker-side: allocate and start newly admitted requests (lock held for the
// arena and queue only).
void admit(wave2d_server* sv, std::vector<Req*>& fresh)
{
    for (auto it = sv->queue.begin(); it != sv->queue.end();) {
        Req* r = sv->reqs[*it];
        const size_t sb = state_bytes(r->p.g), rb = result_bytes(r->p.g);
        size_t o1, o2;
        if (!sv->arena.alloc(sb, &o1)) {
            ++it;
            continue;
        }
        if (!sv->arena.alloc(rb, &o2)) {
            sv->arena.release(o1, sb);
            ++it;
            continue;
        }
        r->off_state = o1;
        r->bytes_state = sb;
        r->off_res = o2;
        r->bytes_res = rb;
        r->has_state = r->has_res = true;
        const size_t a = align256((size_t)r->p.g.ld * r->p.g.ny * sizeof(float));
        char* p0 = sv->base + o1;
        r->u = (float*)p0;
        r->lo = (float*)(p0 + a);
        r->d = (float*)(p0 + 2 * a);
        r->bu = (float*)(p0 + 3 * a);
        r->bl = (float*)(p0 + 4 * a);
        r->bd = (float*)(p0 + 5 * a);
        r->res = (double*)(sv->base + o2);
        r->st = ACTIVE;
        r->t_admit = now_s();
        sv->st.admitted++;
        fresh.push_back(r);
        it = sv->queue.erase(it);
    }
}

int start_request(wave2d_server* sv, Req* r)
{
    const double* u0 = r->rq.u0;
    const double* v0 = r->rq.v0;
    if (r->modes.n > 0) {
        double* su0 = r->res;        // result block, FP64, free until the export
        double* sv0 = (double*)r->bu; // second state block (>= 8 B per node), free until the first pass
        W2D_HIP(sine_series(r->p.g, r->modes, su0, sv0, sv->s));
        u0 = su0;
        v0 = sv0;
    }
    W2D_HIP(simple_first_step_f32c(r->p.g, r->p.kind, r->fw, u0, v0, r->u, r->lo, r->d, sv->s));
    r->left = r->rq.steps - 1;
    r->in_b = false;
    W2D_HIP(hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming));
    return WAVE2D_OK;
}

int finish_request(wave2d_server* sv, Req* r)
{
    const float* u = r->in_b ? r->bu : r->u;
    const float* lo = r->in_b ? r->bl : r->lo;
    W2D_HIP(f32c_export(r->p.g, u, lo, r->res, sv->s));
    W2D_HIP(hipEventRecord(r->done_ev, sv->s));
    r->st = FINISHING;
    return WAVE2D_OK;
}

int largest_supported(int d)
{
    static const int sup[] = {8, 6, 4, 3, 2, 1};
    for (int v : sup)
        if (v <= d && stream_depth_supported(v)) return v;
    return 1;
}

// One quantum: every active request with levels left advances one pass.
int run_quantum(wave2d_server* sv)
{
    struct Key {
        int kind, depth, rows;
        bool operator<(const Key& o) const
        {
            return kind != o.kind ? kind < o.kind : depth != o.depth ? depth < o.depth : rows < o.rows;
        }
    };
    std::map<Key, std::vector<Req*>> groups;
    for (Req* r : sv->active) {
        if (r->st != ACTIVE || r->left <= 0) continue;
        const wave2d_tuning tn = tuning_for(WAVE2D_F32C, r->p.scheme, 0, 0);
        const int dep = largest_supported((int)std::min<int64_t>(tn.depth, r->left));
        groups[Key{r->p.kind, dep, tn.rows}].push_back(r);
    }
    if (groups.empty()) return WAVE2D_OK;
    struct L {
        Key k;
        bool interior;
        size_t items_off, prefix_off;
        int count, total;
    };
    std::vector<L> ls;
    std::vector<unsigned char> host;
    BatchTables gen, inr;
    for (auto& kv : groups) {
        std::vector<BatchInst> bi;
        for (Req* r : kv.second) {
            BatchInst x{};
            x.g = r->p.g;
            x.kind = r->p.kind;
            x.in_w0 = r->in_b ? r->bu : r->u;
            x.in_w1 = r->in_b ? r->bl : r->lo;
            x.in_p = r->in_b ? r->bd : r->d;
            x.out_w0 = r->in_b ? r->u : r->bu;
            x.out_w1 = r->in_b ? r->lo : r->bl;
            x.out_p = r->in_b ? r->d : r->bd;
            x.w32 = step_w32(r->p);
            bi.push_back(x);
            r->left -= kv.first.depth;
            r->in_b = !r->in_b;
        }
        batch_tables(WAVE2D_F32C, kv.first.kind, kv.first.depth, kv.first.rows, bi, gen, inr);
        for (int pass = 0; pass < 2; ++pass) {
            const BatchTables& t = pass ? inr : gen;
            if (t.count == 0) continue;
            host.resize(align256(host.size()));
            L l{kv.first, pass == 1, host.size(), 0, t.count, t.prefix.back()};
            host.insert(host.end(), t.items.begin(), t.items.end());
            host.resize(align256(host.size()));
            l.prefix_off = host.size();
            const unsigned char* pp = (const unsigned char*)t.prefix.data();
            host.insert(host.end(), pp, pp + t.prefix.size() * sizeof(int));
            ls.push_back(l);
        }
    }
    // Table slot of the ring: wait until the quantum that used it is done.
    const int k = sv->ring_next;
    sv->ring_next = (k + 1) % kRing;
    if (sv->ring_used[k]) W2D_HIP(hipEventSynchronize(sv->ring_ev[k]));
    if (sv->cap[k] < host.size()) {
        if (sv->host_stage[k]) W2D_HIP(hipHostFree(sv->host_stage[k]));
        if (sv->dev_tables[k]) W2D_HIP(hipFree(sv->dev_tables[k]));
        sv->host_stage[k] = sv->dev_tables[k] = nullptr;
        const size_t c = std::max<size_t>(host.size() * 2, 1 << 16);
        W2D_HIP(hipHostMalloc(&sv->host_stage[k], c, hipHostMallocDefault));
        W2D_HIP(hipMalloc(&sv->dev_tables[k], c));
        sv->cap[k] = c;
    }
    memcpy(sv->host_stage[k], host.data(), host.size());
    W2D_HIP(hipMemcpyAsync(sv->dev_tables[k], sv->host_stage[k], host.size(), hipMemcpyHostToDevice, sv->s));
    const Fork* fk = nullptr;
    int rc;
    if ((rc = side_of(sv->s, &fk))) return rc;
    bool any_gen = false;
    for (const L& l : ls) any_gen |= !l.interior;
    if (any_gen) {
        W2D_HIP(hipEventRecord(fk->ev_fork, sv->s));
        W2D_HIP(hipStreamWaitEvent(fk->side, fk->ev_fork, 0));
    }
    const char* base = (const char*)sv->dev_tables[k];
    for (const L& l : ls)
        W2D_HIP(batch_launch(WAVE2D_F32C, l.k.kind, l.k.depth, l.interior, base + l.items_off,
                             (const int*)(base + l.prefix_off), l.count, l.total, l.interior ? sv->s : fk->side));
    if (any_gen) {
        W2D_HIP(hipEventRecord(fk->ev_join, fk->side));
        W2D_HIP(hipStreamWaitEvent(sv->s, fk->ev_join, 0));
    }
    W2D_HIP(hipEventRecord(sv->ring_ev[k], sv->s));
    sv->ring_used[k] = true;
    sv->st.quanta++;
    return WAVE2D_OK;
}

void fail_active(wave2d_server* sv, int status)
{
    std::lock_guard<std::mutex> lk(sv->mu);
    for (Req* r : sv->active) {
        r->st = FAILED;
        r->status = status;
        sv->st.failed++;
    }
    sv->active.clear();
}

void worker_main(wave2d_server* sv)
{
    (void)hipSetDevice(sv->device);
    for (;;) {
        std::vector<Req*> fresh;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->active.empty() && sv->queue.empty()) {
                if (sv->stopping) break;
                sv->cv.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
            if (!sv->stopping) admit(sv, fresh);
        }
        int rc = WAVE2D_OK;
        for (Req* r : fresh) {
            if (!rc) rc = start_request(sv, r);
            sv->active.push_back(r);
        }
        // Requests with no pass left (steps == 1) finish right away.
        for (Req* r : sv->active)
            if (!rc && r->st == ACTIVE && r->left <= 0) rc = finish_request(sv, r);
        if (!rc) rc = run_quantum(sv);
        for (Req* r : sv->active)
            if (!rc && r->st == ACTIVE && r->left <= 0) rc = finish_request(sv, r);
        if (rc) {
            fail_active(sv, rc);
            continue;
        }
        // Retire finished requests whose export has completed.
        std::vector<Req*> keep;
        for (Req* r : sv->active) {
            if (r->st == FINISHING && hipEventQuery(r->done_ev) == hipSuccess) {
                std::lock_guard<std::mutex> lk(sv->mu);
                r->t_done = now_s();
                r->st = DONE;
                (void)hipEventDestroy(r->done_ev);
                r->done_ev = nullptr;
                sv->arena.release(r->off_state, r->bytes_state);
                r->has_state = false;
                sv->st.completed++;
                sv->st.lup_done += (int64_t)(r->p.g.nx - 2) * (r->p.g.ny - 2) * r->rq.steps;
            } else {
                keep.push_back(r);
            }
        }
        sv->active.swap(keep);
        // When only exports are pending, wait for the stream instead of spinning.
        bool running = false;
        for (Req* r : sv->active) running |= (r->st == ACTIVE);
        if (!running && !sv->active.empty()) {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->queue.empty()) {
                lk.unlock();
                (void)hipStreamSynchronize(sv->s);
            }
        }
    }
    (void)hipStreamSynchronize(sv->s);
}

}  // namespace

extern "C" {

int wave2d_sine_series(int64_t nx, int64_t ny, int64_t ld, int32_t nmodes, const double* modes, double* u0,
                       double* v0, void* stream)
{
    if (nx < 2 || ny < 2 || ld < nx || ld * ny >= (int64_t(1) << 31) || nx > (1 << 18) || ny > (1 << 18))
        return fail(WAVE2D_EINVAL, "bad grid");
    if (nmodes < 0 || nmodes > kMaxModes || (nmodes > 0 && !modes)) return fail(WAVE2D_EINVAL, "bad modes");
    if (!u0 || !v0) return fail(WAVE2D_EINVAL, "NULL output");
    ModeSet ms{};
    ms.n = nmodes;
    for (int k = 0; k < nmodes; ++k)
        for (int c = 0; c < 4; ++c) ms.m[k][c] = modes[4 * k + c];
    W2D_HIP(sine_series(Grid{(int)nx, (int)ny, (int)ld}, ms, u0, v0, (hipStream_t)stream));
    return WAVE2D_OK;
}

int wave2d_server_create(size_t mem_budget, uint32_t flags, wave2d_server** out)
{
    if (!out) return fail(WAVE2D_EINVAL, "out is NULL");
    *out = nullptr;
    if (flags) return fail(WAVE2D_EINVAL, "unknown server flags 0x%x", flags);
    wave2d_server* sv = new wave2d_server();
    int r;
    if ((r = get_device(&sv->device))) {
        delete sv;
        return r;
    }
    if (mem_budget == 0) {
        size_t fr = 0, tot = 0;
        hipError_t e = hipMemGetInfo(&fr, &tot);
        if (e != hipSuccess) {
            delete sv;
            return hip_fail(e, "hipMemGetInfo");
        }
        mem_budget = fr / 10 * 8;
    }
    mem_budget = align256(mem_budget);
    hipError_t e = hipMalloc((void**)&sv->base, mem_budget);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete sv;
        return fail(WAVE2D_ENOMEM, "server arena of %zu bytes: %s", mem_budget, hipGetErrorString(e));
    }
    sv->arena.init(mem_budget);
    sv->st.bytes_budget = (int64_t)mem_budget;
    e = hipStreamCreateWithFlags(&sv->s, hipStreamNonBlocking);
    for (int k = 0; e == hipSuccess && k < kRing; ++k) e = hipEventCreateWithFlags(&sv->ring_ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipFree(sv->base);
        delete sv;
        return hip_fail(e, "server stream/events");
    }
    sv->worker = std::thread(worker_main, sv);
    *out = sv;
    return WAVE2D_OK;
}

int wave2d_server_submit(wave2d_server* sv, const wave2d_request* rq, uint64_t* id)
{
    if (!sv || !rq || !id) return fail(WAVE2D_EINVAL, "NULL argument");
    Req* r = new Req();
    r->rq = *rq;
    r->rq.modes = nullptr;
    int rc = validate(rq->nx, rq->ny, rq->nx, rq->h, rq->tau, rq->c, rq->scheme,
                      rq->flags & ~(uint32_t)WAVE2D_KERNEL_SIMPLE, &r->p);
    if (!rc && rq->steps < 1) rc = fail(WAVE2D_EINVAL, "steps must be >= 1");
    if (!rc && r->p.kind == KINDW)
        rc = fail(WAVE2D_EINVAL, "scheme %d reaches three lines out; the server takes the 5-, 9- and 13-point classes",
                  rq->scheme);
    if (!rc && !stream_ok(r->p.g, sizeof(float)))
        rc = fail(WAVE2D_EINVAL, "periodic requests need an even nx and nx*ny*4 < 2^31");
    if (!rc && (rq->nmodes < 0 || rq->nmodes > kMaxModes || (rq->nmodes > 0 && !rq->modes)))
        rc = fail(WAVE2D_EINVAL, "nmodes must be in 0..%d with a modes array", kMaxModes);
    if (!rc && rq->nmodes == 0 && (!rq->u0 || !rq->v0))
        rc = fail(WAVE2D_EINVAL, "initial data: give modes or device grids u0, v0");
    if (!rc && state_bytes(r->p.g) + result_bytes(r->p.g) > sv->arena.size())
        rc = fail(WAVE2D_ENOMEM, "request needs %zu bytes, the arena has %zu",
                  state_bytes(r->p.g) + result_bytes(r->p.g), sv->arena.size());
    if (rc) {
        delete r;
        return rc;
    }
    r->modes.n = rq->nmodes;
    for (int k = 0; k < rq->nmodes; ++k)
        for (int c = 0; c < 4; ++c) r->modes.m[k][c] = rq->modes[4 * k + c];
    r->fw = first_w(r->p, rq->flags, rq->tau);
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stopping) {
            delete r;
            return fail(WAVE2D_EBUSY, "server is stopping");
        }
        r->id = sv->next_id++;
        sv->reqs[r->id] = r;
        sv->queue.push_back(r->id);
        sv->st.submitted++;
        *id = r->id;
    }
    sv->cv.notify_one();
    return WAVE2D_OK;
}

int wave2d_server_poll(wave2d_server* sv, uint64_t id, wave2d_result* out)
{
    if (!sv || !out) return fail(WAVE2D_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return fail(WAVE2D_ENOTFOUND, "unknown request %llu", (unsigned long long)id);
    Req* r = it->second;
    if (r->st != DONE && r->st != FAILED) return WAVE2D_EBUSY;
    out->status = r->status;
    out->u = (r->st == DONE) ? r->res : nullptr;
    out->nx = r->p.g.nx;
    out->ny = r->p.g.ny;
    out->ld = r->p.g.ld;
    out->t_submit = r->t_submit;
    out->t_admit = r->t_admit;
    out->t_done = r->t_done;
    return WAVE2D_OK;
}

int wave2d_server_release(wave2d_server* sv, uint64_t id)
{
    if (!sv) return fail(WAVE2D_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return fail(WAVE2D_ENOTFOUND, "unknown request %llu", (unsigned long long)id);
    Req* r = it->second;
    if (r->st != DONE && r->st != FAILED) return fail(WAVE2D_EBUSY, "request %llu still running", (unsigned long long)id);
    if (r->has_res) sv->arena.release(r->off_res, r->bytes_res);
    if (r->has_state) sv->arena.release(r->off_state, r->bytes_state);
    delete r;
    sv->reqs.erase(it);
    return WAVE2D_OK;
}

int wave2d_server_stats_get(wave2d_server* sv, wave2d_server_stats* st)
{
    if (!sv || !st) return fail(WAVE2D_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    *st = sv->st;
    st->queued = (int64_t)sv->queue.size();
    st->active = st->admitted - st->completed - st->failed;
    st->bytes_in_use = (int64_t)sv->arena.used();
    return WAVE2D_OK;
}

int wave2d_server_destroy(wave2d_server* sv)
{
    if (!sv) return WAVE2D_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
        for (uint64_t id : sv->queue) {
            Req* r = sv->reqs[id];
            r->st = FAILED;
            r->status = WAVE2D_EBUSY;
            sv->st.failed++;
        }
        sv->queue.clear();
    }
    sv->cv.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    (void)hipStreamSynchronize(sv->s);
    for (auto& kv : sv->reqs) {
        if (kv.second->done_ev) (void)hipEventDestroy(kv.second->done_ev);
        delete kv.second;
    }
    for (int k = 0; k < kRing; ++k) {
        if (sv->host_stage[k]) (void)hipHostFree(sv->host_stage[k]);
        if (sv->dev_tables[k]) (void)hipFree(sv->dev_tables[k]);
        if (sv->ring_ev[k]) (void)hipEventDestroy(sv->ring_ev[k]);
    }
    (void)hipStreamDestroy(sv->s);
    (void)hipFree(sv->base);
    delete sv;
    return WAVE2D_OK;
}

}  // extern "C"

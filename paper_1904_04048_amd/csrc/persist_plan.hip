// Planning of persistent launches (host code): the work items of every
// instance, their pinning to the per-XCC queues and the order of the passes
// in each queue, shared by batches and the server.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "host.h"

namespace w2d_host {

using namespace w2d;

bool xcc_layout_ok(int dev)
{
    static std::mutex mu;
    static std::map<int, bool> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    bool ok = false;
    const int n = 64 * kPersistQueues;
    int* d = nullptr;
    if (hipMalloc(&d, n * sizeof(int)) == hipSuccess) {
        std::vector<int> h(n, -1);
        if (xcc_probe(d, n, nullptr) == hipSuccess &&
            hipMemcpy(h.data(), d, n * sizeof(int), hipMemcpyDeviceToHost) == hipSuccess) {
            std::vector<int> cnt(kPersistQueues, 0);
            ok = true;
            for (int v : h) {
                if (v < 0 || v >= kPersistQueues) ok = false;
                else ++cnt[v];
            }
            for (int c : cnt) ok = ok && c > 0;
        }
        (void)hipFree(d);
    }
    (void)hipGetLastError();
    cache[dev] = ok;
    return ok;
}

int persist_rows(int ny, int cap)
{
    if (ny <= cap) return ny;
    const int nseg = (ny + cap - 1) / cap;
    return (ny + nseg - 1) / nseg;
}

namespace {

// The invariants the persistent kernel relies on: per class and queue, the
// tasks [qoff[q], qoff[q+1]) cover items 0 .. qn[q]-1 in order (each task's
// first item is the previous task's end), every task's instance belongs to
// the class, and each instance's passes appear in order 0, 1, ..., once
// each (a pass waits only for passes queued before it).
int check_plan(const std::vector<PersistInput>& in, const PersistPlan& pl, const std::vector<int>& items)
{
    std::vector<int64_t> seen(in.size(), 0);
    for (int c = 0; c < kPersistClasses; ++c)
        for (int q = 0; q < kPersistQueues; ++q) {
            int64_t next = 0;
            for (int t = pl.qoff[c][q]; t < pl.qoff[c][q + 1]; ++t) {
                const PersistTask& k = pl.tasks[(size_t)t];
                if (k.inst < 0 || (size_t)k.inst >= in.size() || in[(size_t)k.inst].kind != c || k.first != next ||
                    items[(size_t)k.inst] < 1 || k.pass != seen[(size_t)k.inst])
                    return fail(WAVE2D_EDEVICE, "persistent plan inconsistent at class %d queue %d task %d", c, q, t);
                ++seen[(size_t)k.inst];
                next += items[(size_t)k.inst];
            }
            if (next != pl.qn[c][q]) return fail(WAVE2D_EDEVICE, "persistent plan: queue %d item count", q);
        }
    for (size_t i = 0; i < in.size(); ++i)
        if (seen[i] != in[i].passes)
            return fail(WAVE2D_EDEVICE, "persistent plan: instance %zu has %lld of %lld passes", i, (long long)seen[i],
                        (long long)in[i].passes);
    return WAVE2D_OK;
}

}  // namespace

int persist_plan(const std::vector<PersistInput>& in, int cap, PersistPlan* pl)
{
    const size_t ni = in.size();
    const size_t isz = persist_inst_size();
    pl->recs.assign(ni * isz, 0);
    pl->tasks.clear();
    pl->items = pl->item_rows = 0;
    std::vector<int> items(ni, 0);
    std::vector<double> cost(ni, 0.0);
    for (size_t i = 0; i < ni; ++i) {
        const PersistInput& x = in[i];
        int nb = 0, rows_used = 0;
        const int D = persist_depth(x.kind);
        const int R = x.kind == KIND13 ? 2 : 1;
        float* s0[3] = {x.s0[0], x.s0[1], x.s0[2]};
        float* s1[3] = {x.s1[0], x.s1[1], x.s1[2]};
        items[i] = persist_inst(x.g, x.kind, x.w, persist_rows(x.g.ny, cap), x.tile_off, s0, s1,
                                pl->recs.data() + i * isz, &nb, &rows_used);
        if (items[i] < 1)
            return fail(WAVE2D_EINVAL, "instance %zu: segments of %d rows leave too many tiles", i,
                        persist_rows(x.g.ny, cap));
        // Work model: an item streams rows + R (D - 1) + 2R + 1 rows of D
        // levels, each about 2R + 1 times the 5-point work.
        cost[i] = (double)x.passes * items[i] * (rows_used + R * (D - 1) + 2 * R + 1) * D * (2 * R + 1);
        pl->items += x.passes * items[i];
        pl->item_rows += x.passes * items[i] * (int64_t)rows_used;
    }
    // Per class, pin instances to queues: largest work first onto the
    // least-loaded queue.
    std::vector<size_t> order(ni);
    for (size_t i = 0; i < ni; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    for (int c = 0; c < kPersistClasses; ++c) {
        std::vector<double> load(kPersistQueues, 0.0);
        std::vector<std::vector<size_t>> members(kPersistQueues);
        for (size_t i : order) {
            if (in[i].passes == 0 || in[i].kind != c) continue;
            const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[q] += cost[i];
            members[q].push_back(i);
        }
        pl->qoff[c].assign(kPersistQueues + 1, 0);
        pl->qn[c].assign(kPersistQueues, 0);
        for (int q = 0; q < kPersistQueues; ++q) {
            pl->qoff[c][q] = (int)pl->tasks.size();
            // Passes in order of the progress they complete, (p + 1) /
            // passes: every instance advances at the same relative pace, so
            // instances with many passes are not left alone at the end of
            // the queue as chains of small passes that cannot fill the XCC.
            struct Key {
                double prog;
                size_t i;
                int64_t p;
            };
            std::vector<Key> keys;
            for (size_t i : members[q])
                for (int64_t p = 0; p < in[i].passes; ++p)
                    keys.push_back(Key{(double)(p + 1) / (double)in[i].passes, i, p});
            std::stable_sort(keys.begin(), keys.end(), [](const Key& x, const Key& y) { return x.prog < y.prog; });
            int64_t first = 0;
            for (const Key& k : keys) {
                pl->tasks.push_back(PersistTask{(int)k.i, (int)((in[k.i].par0 + k.p) & 1), (int)k.p, (int)first});
                first += items[k.i];
            }
            if (first >= (int64_t(1) << 31))
                return fail(WAVE2D_EINVAL, "batch too large for one persistent launch (%lld items on one XCC)",
                            (long long)first);
            pl->qn[c][q] = (int)first;
        }
        pl->qoff[c][kPersistQueues] = (int)pl->tasks.size();
    }
    return check_plan(in, *pl, items);
}

}  // namespace w2d_host

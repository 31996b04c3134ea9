// Host-side helpers shared by the C-ABI translation units (validation,
// weights, tuning, library-owned buffers, error reporting).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <initializer_list>
#include <utility>
#include <vector>

#include "w2d.h"
#include "wave2d.h"
#include "wide.h"

namespace w2d_host {

using w2d::FirstW;
using w2d::Fork;
using w2d::Grid;
using w2d::StepW32;
using w2d::StepW64;

// Node weights per class (q1, q2) in the order (1,0), (1,1), (2,0), (2,1),
// (2,2), (3,0), (3,1), (3,2), (3,3); the schemes of Sec. 6 use the first
// three.
struct Params {
    Grid g;
    int scheme;
    int kind;
    double lam;
    double wa[w2d::kWideClasses], wb[w2d::kWideClasses];
    bool has_b;
};

// A scheme built by wave2d_scheme_create: per node class (the order of
// Params) the node weights of A and of B / tau as polynomials in lambda
// (coefficient k of lambda^k), the stencil class the kernels run it as,
// and its stability limit.
struct CustomScheme {
    static constexpr int kDeg = 12;
    double a[w2d::kWideClasses][kDeg + 1];
    double b[w2d::kWideClasses][kDeg + 1];
    int kind;
    double lambda_max;
};
constexpr int kCustomBase = 1000;
int custom_scheme_create(int m, const int32_t* nodes, const int32_t* exps, int* id);
bool custom_scheme(int id, CustomScheme* out);

int fail(int status, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int kind_of(int scheme);
int validate(int64_t nx, int64_t ny, int64_t ld, double h, double tau, double c, int scheme, uint32_t flags,
             Params* p);
StepW64 step_w64(const Params& p);
StepW32 step_w32(const Params& p);
FirstW first_w(const Params& p, uint32_t flags, double tau);
w2d::WideW64 wide_w64(const Params& p);
w2d::WideW32 wide_w32(const Params& p);
w2d::WideFirstW wide_first_w(const Params& p, uint32_t flags, double tau);
// Stencil radius of a kind (KIND5/9: 1, KIND13: 2, KINDW: 3).
int radius_of_kind(int kind);
bool overlap(const void* a, size_t na, const void* b, size_t nb);
size_t grid_bytes(const Grid& g, size_t elt);
int check_ptrs(const Grid& g, std::initializer_list<std::pair<const void*, size_t>> arrs);
wave2d_tuning tuning_for(int precision, int scheme, int64_t nx, int64_t ny);
bool stream_ok(const Grid& g, size_t elt);
void set_tuning_entry(int precision, int scheme, const wave2d_tuning& t);
void set_tuning_size_entry(int precision, int scheme, int64_t nx, int64_t ny, const wave2d_tuning& t);
void save_tune_cache(int precision, int scheme, int64_t nx, int64_t ny, const wave2d_tuning& t);
int get_device(int* dev);
size_t align256(size_t v);
int side_of(hipStream_t s, const Fork** out);
// Second-state workspace bytes of a multi-step call (FP64: two grids, f32c:
// three), each grid aligned to 256 bytes.
size_t work_bytes_of(int precision, const Grid& g);
// Compensated state (u, lo, d) advanced `steps` levels in place; `work`
// (work_bytes) is the second state, or NULL for the library's own buffer.
int run_steps_f32c(const Params& p, uint32_t flags, int64_t steps, float* u, float* lo, float* d, void* work,
                   size_t work_bytes, hipStream_t s);

// ---- persistent launches (persist_plan.hip) -----------------------------------
// Stencil classes with a persistent kernel (KIND5, KIND9, KIND13).
constexpr int kPersistClasses = 3;
// Tallest segment of a persistent work item by default (taller grids are
// cut into equal segments of at most this many rows).
constexpr int kPersistRowsCap = 160;
// Whether the workgroups of a launch land on exactly the kPersistQueues
// XCCs 0..kPersistQueues-1 (one probe per device): the persistent kernel
// keys its queues on them.
bool xcc_layout_ok(int dev);
// Segment height of an instance's persistent items: the whole grid up to
// `cap` rows, else the grid cut into equal segments of at most `cap` rows.
int persist_rows(int ny, int cap);
// One instance of a persistent launch: its grid, class, weights, the state
// it starts from (s0) and the other state (s1), its tile counters' offset
// within its class, its passes and the parity of the first (1: the first
// pass reads s1).
struct PersistInput {
    w2d::Grid g;
    int kind;
    w2d::StepW32 w;
    float* s0[3];
    float* s1[3];
    int tile_off;
    int64_t passes;
    int par0;
};
// Tables of one persistent launch per class: instance records, tasks in
// per-queue order, queue offsets and item counts.
struct PersistPlan {
    std::vector<unsigned char> recs;
    std::vector<w2d::PersistTask> tasks;     // all classes, class by class
    std::vector<int> qoff[kPersistClasses];  // per class: task index ranges of the queues (absolute)
    std::vector<int> qn[kPersistClasses];    // per class: items per queue
    int64_t items = 0, item_rows = 0;
};
// Plan with segments of at most `cap` rows: pin each instance to the
// least-loaded queue of its class (largest work first) and list each
// queue's passes in order of the progress they complete.  Checks the
// plan's invariants before returning.
int persist_plan(const std::vector<PersistInput>& in, int cap, PersistPlan* pl);

}  // namespace w2d_host

#define W2D_HIP(call)                                                 \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) return w2d_host::hip_fail(e_, #call);   \
    } while (0)

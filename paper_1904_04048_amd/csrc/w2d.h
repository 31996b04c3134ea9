// Internal declarations of the wave2d library (kernels and launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "point.h"

namespace w2d {

struct Grid {
    int nx, ny, ld;
    int periodic = 0;  // boundary rule: 0 Dirichlet (odd reflection), 1 periodic with period nx, ny
};

// Two-step weights (2 x the A-operator node weights).
struct StepW64 {
    double w10, w11, w20, wx;  // wx = w10 + 2 w11 + 4 w20
};
// wc = -4 (w10 + w11 + w20) (centre weight), wx = w10 + 2 w11 + 4 w20 (the
// weight of Dx + Dy in the regrouped increments; equal to w10 for the
// 5-point class).  wx is carried as an unevaluated sum wx + wxl of two
// floats (wxl = the rounding error of wx): a weight rounded to single
// precision changes the scheme's frequencies by up to 3e-8 relative, a phase
// error that grows with the step count (about 1.4e-5 of max|u| after 5000
// steps on a 64^2 grid).  The other weights multiply higher differences,
// whose share of the increment is smaller by lambda^2 theta^2 / 6 or less.
struct StepW32 {
    float w10, w11, w20, wc, wx, wxl;
};
// First-step weights: A node weights and B node weights divided by tau.
struct FirstW {
    double a10, a11, a20, b10, b11, b20, tau;
    int poisson;  // 0: conventional first step (no v0 stencil term)
};

// ---- one-node-per-thread kernels (simple.hip) -----------------------------
hipError_t simple_first_step(const Grid& g, int kind, const FirstW& w, const double* u0, const double* v0,
                             double* u1, hipStream_t s);
hipError_t simple_first_step_f32c(const Grid& g, int kind, const FirstW& w, const double* u0,
                                  const double* v0, float* u, float* lo, float* d, hipStream_t s);
// u_next may equal u_prev (in place).
hipError_t simple_step_f64(const Grid& g, int kind, const StepW64& w, const double* u_prev,
                           const double* u_cur, double* u_next, hipStream_t s);
hipError_t simple_step_f32c(const Grid& g, int kind, const StepW32& w, const float* u, const float* lo,
                            const float* d, float* u2, float* lo2, float* d2, hipStream_t s);
hipError_t f32c_init(const Grid& g, const double* u_prev, const double* u_cur, float* u, float* lo, float* d,
                     hipStream_t s);
hipError_t f32c_export(const Grid& g, const float* u, const float* lo, double* out, hipStream_t s);
// Element-wise copies of 1..3 grids (unused pointers NULL).
hipError_t copy_f32x3(const Grid& g, const float* a, const float* b, const float* c, float* a2, float* b2,
                      float* c2, hipStream_t s);
hipError_t copy_f64x2(const Grid& g, const double* a, const double* b, double* a2, double* b2, hipStream_t s);
hipError_t swap_f64(const Grid& g, double* a, double* b, hipStream_t s);
// Batched one-node-per-thread launches over many grids: record r owns the
// blocks [prefix[r], prefix[r+1]) of one launch of `blocks` blocks
// (node_tiles(g) blocks per grid).
struct FirstRecF32C {
    Grid g;
    int kind;
    FirstW w;
    const double* u0;
    const double* v0;
    float *u, *lo, *d;
};
struct CopyRec3 {
    Grid g;
    const float* src[3];
    float* dst[3];
};
int node_tiles(const Grid& g);
hipError_t first_step_f32c_batch(const FirstRecF32C* recs, const int* prefix, int count, int blocks, hipStream_t s);
hipError_t copy_f32x3_batch(const CopyRec3* recs, const int* prefix, int count, int blocks, hipStream_t s);
// p[0..n) = v (a kernel, so that it can be captured in a graph).
hipError_t fill_i32(int* p, int n, int v, hipStream_t s);
// b <- a on interior nodes, 0 on the boundary.
hipError_t copy_interior_f64(const Grid& g, const double* a, double* b, hipStream_t s);

// ---- temporally blocked streaming kernels (stream.hip) ----------------------
// Optional side stream: the boundary-strip kernel of a pass runs there,
// concurrently with the interior kernel, fenced by two events.
struct Fork {
    hipStream_t side;
    hipEvent_t ev_fork, ev_join;
};
struct StreamShape {
    int depth;                 // time levels per pass
    int rows;                  // output rows per wavefront work item
    const Fork* fork = nullptr;
};
// FP64: levels (p_in, c_in) = (k-1, k) -> (p_out, c_out) = (k+depth-1, k+depth).
// With depth == 1 and p_out == p_in (in place), c_out must be NULL and only
// level k+1 is written (into p_in).
hipError_t stream_step_f64(const Grid& g, int kind, const StepW64& w, const StreamShape& sh,
                           const double* p_in, const double* c_in, double* p_out, double* c_out,
                           hipStream_t s);
hipError_t stream_step_f32c(const Grid& g, int kind, const StepW32& w, const StreamShape& sh, const float* u,
                            const float* lo, const float* d, float* u2, float* lo2, float* d2, hipStream_t s);
bool stream_depth_supported(int depth);

// ---- batched passes (stream.hip) ----------------------------------------------
// One instance's part of a batched pass: its grid, stencil class, input and
// output state (FP64: window field u^k, point field u^{k-1}; compensated:
// u, lo and d) and weights.
struct BatchInst {
    Grid g;
    int kind;
    const void* in_w0;
    const void* in_w1;
    const void* in_p;
    void* out_w0;
    void* out_w1;
    void* out_p;
    StepW32 w32;
    StepW64 w64;
};
// Host staging of the device tables of one batched launch.
struct BatchTables {
    std::vector<unsigned char> items;
    std::vector<int> prefix;  // prefix[k] = first work id of item k; back() = total
    int count = 0;
    int rows = 0;  // segment rows the launch uses
};
size_t batch_item_size(int precision);
// Tables of one pass at `depth` for the instances (all of stencil class
// `kind`): boundary items into gen, interior items into inr.  `rows` is the
// least segment height; taller segments are taken where the launch still
// has enough work items to fill the GPU (see batch_rows in stream.hip).
void batch_tables(int precision, int kind, int depth, int rows, const std::vector<BatchInst>& insts, BatchTables& gen,
                  BatchTables& inr);
hipError_t batch_launch(int precision, int kind, int depth, bool interior, const void* d_items, const int* d_prefix,
                        int count, int total, hipStream_t s);
// How a launch shape fits the current device: output columns per strip,
// waves of the interior step kernel resident on the whole device, and
// whether that kernel spills registers to scratch memory.
struct ShapeFit {
    int strip_cols;  // output columns of one work item
    int slots;       // resident waves of the interior kernel on the device
    bool spills;     // the kernel uses scratch memory
    int simd_waves;  // resident waves per SIMD
    int halo_rows;   // rows a pass reaches beyond its outputs (R x depth)
};
ShapeFit stream_shape_fit(int precision, int kind, int depth);

// ---- persistent batched passes (stream.hip) --------------------------------
// One launch runs all passes of many compensated instances: one work queue
// per XCC (instances pinned to one XCC), tasks of one item per wave.
constexpr int kPersistQueues = 8;
// Counters of a persistent launch: queue heads 0..7 and the count of waits
// that gave up, one per 128-byte line (kPersistStride ints apart), then one
// counter per tile (strip x segment) of every instance of the launch, the
// passes that tile has finished.  All zero before the launch.
constexpr int kPersistStride = 32;
constexpr int kPersistTileBase = kPersistStride * (kPersistQueues + 1);
// Segments of a persistent item have at least this many rows (fewer only
// when the grid has fewer), which bounds an instance's tiles.
constexpr int kPersistMinRows = 8;
// Items [first, first + items) of a queue: pass number `pass` (parity
// `par` of the state it reads) of instance `inst`.  An item runs once every
// tile whose output it reads has finished `pass` passes.
struct PersistTask {
    int inst, par, pass, first;
};
size_t persist_inst_size();
// Pass depth of the persistent kernel for a stencil class.
int persist_depth(int kind);
// Most tiles an instance of the class can have (segments of
// kPersistMinRows rows): the size of its block of tile counters.
int persist_max_tiles(const Grid& g, int kind);
// Write the device record of one instance into rec (persist_inst_size()
// bytes): grid, class, weights, states s0 (u, lo, d) and s1 (the second
// state), segment height `rows` (clamped like single-grid passes), and the
// offset of its tile counters.  Returns its work items per pass (-1 when
// the clamped height leaves more tiles than persist_max_tiles); *nb = how
// many of them are boundary items, *rows_used = the height applied.
int persist_inst(const Grid& g, int kind, const StepW32& w, int rows, int tile_off, float* const s0[3],
                 float* const s1[3], unsigned char* rec, int* nb, int* rows_used);
// Workgroups of one persistent launch of a class (the kernel's resident
// capacity).
int persist_blocks(int kind);
// All queued passes of one stencil class's instances; a wait gives up after
// wait_ticks of the 100 MHz real-time clock.
hipError_t persist_launch(int kind, const void* insts, const PersistTask* tasks, const int* qt_off, const int* qn,
                          int* ctr, long long wait_ticks, hipStream_t s);
// XCC id of each of n workgroups (out[k], device).
hipError_t xcc_probe(int* out, int n, hipStream_t s);

// ---- reductions (norms.hip) -------------------------------------------------
// Partial sums into `part` (nblk x 4 doubles), then a single-block final
// reduction into part[nblk*4 .. +4].
int norms_blocks();
hipError_t norms_f64(const Grid& g, const double* a, const double* b, double* part, hipStream_t s);
hipError_t norms_f32c(const Grid& g, const float* u, const float* lo, const double* b, double* part,
                      hipStream_t s);

}  // namespace w2d

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
// weight of Dx + Dy in the regrouped 9- and 13-point increments).
struct StepW32 {
    float w10, w11, w20, wc, wx;
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

// ---- reductions (norms.hip) -------------------------------------------------
// Partial sums into `part` (nblk x 4 doubles), then a single-block final
// reduction into part[nblk*4 .. +4].
int norms_blocks();
hipError_t norms_f64(const Grid& g, const double* a, const double* b, double* part, hipStream_t s);
hipError_t norms_f32c(const Grid& g, const float* u, const float* lo, const double* b, double* part,
                      hipStream_t s);

}  // namespace w2d

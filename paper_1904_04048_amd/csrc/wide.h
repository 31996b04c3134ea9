// Schemes with nodes up to three lines from the centre (built by the
// construction of Sec. 4-5 from larger monomial sets): their stencil class,
// weights and kernels.  The temporally blocked, batched and served kernels
// take only the 5-, 9- and 13-point classes.
#pragma once

#include "w2d.h"

namespace w2d {

// Stencil class of these schemes, beside KIND5, KIND9 and KIND13.
constexpr int KINDW = 3;

// Weights per node class (q1, q2) in the order (1,0), (1,1), (2,0), (2,1),
// (2,2), (3,0), (3,1), (3,2), (3,3): two-step weights (2 x the A node
// weights), in FP32 as a two-float pair each; first-step A node weights and
// B node weights divided by tau.
constexpr int kWideClasses = 9;
struct WideW64 {
    double w[kWideClasses];
};
struct WideW32 {
    float w[kWideClasses], wl[kWideClasses];
};
struct WideFirstW {
    double a[kWideClasses], b[kWideClasses], tau;
    int poisson;  // 0: conventional first step (no v0 stencil term)
};

// One level per launch (wide.hip): LDS-staged tiles for the first step and
// FP64, waves streaming down column strips for the compensated update.
hipError_t wide_first_step(const Grid& g, const WideFirstW& w, const double* u0, const double* v0, double* u1,
                           hipStream_t s);
hipError_t wide_first_step_f32c(const Grid& g, const WideFirstW& w, const double* u0, const double* v0, float* u,
                                float* lo, float* d, hipStream_t s);
// u_next may equal u_prev (in place).
hipError_t wide_step_f64(const Grid& g, const WideW64& w, const double* u_prev, const double* u_cur,
                         double* u_next, hipStream_t s);
hipError_t wide_step_f32c(const Grid& g, const WideW32& w, const float* u, const float* lo, const float* d,
                          float* u2, float* lo2, float* d2, hipStream_t s);

}  // namespace w2d

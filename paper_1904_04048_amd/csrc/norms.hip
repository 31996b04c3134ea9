// Deterministic FP64 error norms: { max|a-b|, max|b|, sum (a-b)^2, sum b^2 }.
//
// Pass 1: a fixed number of blocks; block k takes rows k, k + nblk, ...,
// its threads stride along the row, and a fixed-shape tree in LDS combines
// the threads.  Pass 2: one block combines the per-block partials in index
// order.  The result therefore does not depend on timing.  A NaN anywhere
// propagates into the maxima.
#include "w2d.h"

namespace w2d {
namespace {

constexpr int kBlocks = 1024;
constexpr int kThreads = 256;

__device__ __forceinline__ double nanmax(double m, double x) { return (x > m || x != x) ? x : m; }

struct Acc {
    double m, mb, s, sb;
};

__device__ __forceinline__ void acc_add(Acc& a, double x, double b)
{
    const double d = x - b;
    a.m = nanmax(a.m, fabs(d));
    a.mb = nanmax(a.mb, fabs(b));
    a.s += d * d;
    a.sb += b * b;
}

__device__ void block_reduce_store(Acc a, double* out)
{
    __shared__ double sh[4][kThreads];
    const int t = threadIdx.x;
    sh[0][t] = a.m;
    sh[1][t] = a.mb;
    sh[2][t] = a.s;
    sh[3][t] = a.sb;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            sh[0][t] = nanmax(sh[0][t], sh[0][t + w]);
            sh[1][t] = nanmax(sh[1][t], sh[1][t + w]);
            sh[2][t] = sh[2][t] + sh[2][t + w];
            sh[3][t] = sh[3][t] + sh[3][t + w];
        }
        __syncthreads();
    }
    if (t < 4) out[t] = sh[t][0];
}

__global__ __launch_bounds__(kThreads) void k_part_f64(Grid g, const double* __restrict__ a,
                                                      const double* __restrict__ b, double* __restrict__ part)
{
    Acc acc{0.0, 0.0, 0.0, 0.0};
    for (int j = blockIdx.x; j < g.ny; j += gridDim.x) {
        const size_t r = (size_t)j * g.ld;
        for (int i = threadIdx.x; i < g.nx; i += kThreads) acc_add(acc, a[r + i], b[r + i]);
    }
    block_reduce_store(acc, part + 4 * blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_part_f32c(Grid g, const float* __restrict__ u,
                                                       const float* __restrict__ lo, const double* __restrict__ b,
                                                       double* __restrict__ part)
{
    Acc acc{0.0, 0.0, 0.0, 0.0};
    for (int j = blockIdx.x; j < g.ny; j += gridDim.x) {
        const size_t r = (size_t)j * g.ld;
        for (int i = threadIdx.x; i < g.nx; i += kThreads) acc_add(acc, f32c_join(u[r + i], lo[r + i]), b[r + i]);
    }
    block_reduce_store(acc, part + 4 * blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_final(int nblk, double* part)
{
    Acc acc{0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < nblk; k += kThreads) {
        acc.m = nanmax(acc.m, part[4 * k + 0]);
        acc.mb = nanmax(acc.mb, part[4 * k + 1]);
        acc.s += part[4 * k + 2];
        acc.sb += part[4 * k + 3];
    }
    block_reduce_store(acc, part + 4 * nblk);
}

}  // namespace

int norms_blocks() { return kBlocks; }

hipError_t norms_f64(const Grid& g, const double* a, const double* b, double* part, hipStream_t s)
{
    k_part_f64<<<kBlocks, kThreads, 0, s>>>(g, a, b, part);
    k_final<<<1, kThreads, 0, s>>>(kBlocks, part);
    return hipGetLastError();
}

hipError_t norms_f32c(const Grid& g, const float* u, const float* lo, const double* b, double* part, hipStream_t s)
{
    k_part_f32c<<<kBlocks, kThreads, 0, s>>>(g, u, lo, b, part);
    k_final<<<1, kThreads, 0, s>>>(kBlocks, part);
    return hipGetLastError();
}

}  // namespace w2d

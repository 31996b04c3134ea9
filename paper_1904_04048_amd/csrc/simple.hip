// One-node-per-thread kernels: the first step (run once per solve), state
// conversions, copies, and a plain two-step sweep used for small grids and
// as an in-library cross-check of the temporally blocked kernels.
//
// Every grid read goes through bc_load, which applies the boundary rule:
// boundary nodes read as 0, a node one line outside reads as minus its
// mirror image (only the 13-point stencil reaches there); on periodic grids
// indices wrap around and every node is updated.
#include "w2d.h"

namespace w2d {
namespace {

constexpr int BX = 64, BY = 4;

template <typename T>
__device__ __forceinline__ T bc_load(const T* __restrict__ p, const Grid& g, int i, int j)
{
    const int nx = g.nx, ny = g.ny, ld = g.ld;
    if (g.periodic) {
        i = (i < 0) ? i + nx : (i >= nx ? i - nx : i);
        j = (j < 0) ? j + ny : (j >= ny ? j - ny : j);
        return p[(size_t)j * ld + i];
    }
    bool neg = false;
    if (i < 0) { i = -i; neg = !neg; }
    else if (i > nx - 1) { i = 2 * (nx - 1) - i; neg = !neg; }
    if (j < 0) { j = -j; neg = !neg; }
    else if (j > ny - 1) { j = 2 * (ny - 1) - j; neg = !neg; }
    if (i <= 0 || i >= nx - 1 || j <= 0 || j >= ny - 1) return T(0);
    const T v = p[(size_t)j * ld + i];
    return neg ? -v : v;
}

// Plain load of a node that the boundary rule leaves as stored.
template <typename T>
__device__ __forceinline__ T plain_load(const T* __restrict__ p, const Grid& g, int i, int j)
{
    return p[(size_t)j * g.ld + i];
}

// Whether every node within `r` of the BX x BY tile at (i0, j0) reads as
// stored (inside the grid, off its boundary under the Dirichlet rule), so
// that the tile can gather without the boundary rule.
__device__ __forceinline__ bool plain_tile(const Grid& g, int i0, int j0, int r)
{
    const int lo = g.periodic ? 0 : 1;
    return i0 - r >= lo && j0 - r >= lo && i0 + BX - 1 + r <= g.nx - 1 - lo && j0 + BY - 1 + r <= g.ny - 1 - lo;
}

template <int K, typename T, bool PLAIN = false>
__device__ __forceinline__ Nbh<T> gather(const T* __restrict__ p, const Grid& g, int i, int j)
{
    auto bc_load = [&](const T* __restrict__ q, const Grid& gg, int ii, int jj) {
        if constexpr (PLAIN) return plain_load(q, gg, ii, jj);
        else return w2d::bc_load(q, gg, ii, jj);
    };
    Nbh<T> v;
    v.C = bc_load(p, g, i, j);
    v.E = bc_load(p, g, i + 1, j);
    v.W = bc_load(p, g, i - 1, j);
    v.N = bc_load(p, g, i, j + 1);
    v.S = bc_load(p, g, i, j - 1);
    if constexpr (KT<K>::DIAG) {
        v.NE = bc_load(p, g, i + 1, j + 1);
        v.NW = bc_load(p, g, i - 1, j + 1);
        v.SE = bc_load(p, g, i + 1, j - 1);
        v.SW = bc_load(p, g, i - 1, j - 1);
    } else {
        v.NE = v.NW = v.SE = v.SW = T(0);
    }
    if constexpr (KT<K>::AX2) {
        v.EE = bc_load(p, g, i + 2, j);
        v.WW = bc_load(p, g, i - 2, j);
        v.NN = bc_load(p, g, i, j + 2);
        v.SS = bc_load(p, g, i, j - 2);
    } else {
        v.EE = v.WW = v.NN = v.SS = T(0);
    }
    return v;
}

// Nodes the update writes: every node on a periodic grid, else the
// non-boundary nodes.
__device__ __forceinline__ bool interior(const Grid& g, int i, int j)
{
    return g.periodic || (i > 0 && i < g.nx - 1 && j > 0 && j < g.ny - 1);
}

template <int K>
__global__ __launch_bounds__(BX* BY) void k_first_step(Grid g, FirstW w, const double* __restrict__ u0,
                                                       const double* __restrict__ v0, double* __restrict__ u1)
{
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    double r = 0.0;
    if (interior(g, i, j)) {
        const Nbh<double> a = gather<K>(u0, g, i, j);
        const Nbh<double> b = gather<K>(v0, g, i, j);
        const double sa = lap_diff<K>(a, w.a10, w.a11, w.a20);
        const double sb = w.poisson ? lap_diff<K>(b, w.b10, w.b11, w.b20) : 0.0;
        r = first_update(a.C, sa, b.C, sb, w.tau);
    }
    u1[(size_t)j * g.ld + i] = r;
}

// First step and split at node (i, j) (inside the grid); PLAIN: the
// node's whole stencil reads as stored (see plain_tile).
template <int K, bool PLAIN = false>
__device__ __forceinline__ void first_node_f32c(const Grid& g, const FirstW& w, const double* __restrict__ u0,
                                                const double* __restrict__ v0, float* __restrict__ u,
                                                float* __restrict__ lo, float* __restrict__ d, int i, int j)
{
    float ru = 0.f, rl = 0.f, rd = 0.f;
    if (PLAIN || interior(g, i, j)) {
        const Nbh<double> a = gather<K, double, PLAIN>(u0, g, i, j);
        const Nbh<double> b = gather<K, double, PLAIN>(v0, g, i, j);
        const double sa = lap_diff<K>(a, w.a10, w.a11, w.a20);
        const double sb = w.poisson ? lap_diff<K>(b, w.b10, w.b11, w.b20) : 0.0;
        f32c_split(first_update(a.C, sa, b.C, sb, w.tau), a.C, ru, rl, rd);
    }
    const size_t o = (size_t)j * g.ld + i;
    u[o] = ru;
    lo[o] = rl;
    d[o] = rd;
}

template <int K>
__global__ __launch_bounds__(BX* BY) void k_first_step_f32c(Grid g, FirstW w, const double* __restrict__ u0,
                                                            const double* __restrict__ v0, float* __restrict__ u,
                                                            float* __restrict__ lo, float* __restrict__ d)
{
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    first_node_f32c<K>(g, w, u0, v0, u, lo, d, i, j);
}

// Batched launches over many grids: record r owns the blocks
// [prefix[r], prefix[r+1]) of a 1-D launch, one BX x BY tile of its grid
// each (tiles numbered row by row), so every node is computed by the same
// code as in the single-grid kernels.
__device__ __forceinline__ int find_record(const int* __restrict__ prefix, int count, int b)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(BX* BY) void k_first_step_f32c_batch(const FirstRecF32C* __restrict__ recs,
                                                                  const int* __restrict__ prefix, int count)
{
    const int b = (int)blockIdx.x;
    const int r = find_record(prefix, count, b);
    const FirstRecF32C rc = recs[r];
    const int t = b - prefix[r];
    const int tx = (rc.g.nx + BX - 1) / BX;
    const int i0 = (t % tx) * BX, j0 = (t / tx) * BY;
    const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
    if (i >= rc.g.nx || j >= rc.g.ny) return;
    const bool plain = plain_tile(rc.g, i0, j0, rc.kind == KIND13 ? 2 : 1);
    switch (rc.kind) {
    case KIND5:
        if (plain) first_node_f32c<KIND5, true>(rc.g, rc.w, rc.u0, rc.v0, rc.u, rc.lo, rc.d, i, j);
        else first_node_f32c<KIND5>(rc.g, rc.w, rc.u0, rc.v0, rc.u, rc.lo, rc.d, i, j);
        break;
    case KIND9:
        if (plain) first_node_f32c<KIND9, true>(rc.g, rc.w, rc.u0, rc.v0, rc.u, rc.lo, rc.d, i, j);
        else first_node_f32c<KIND9>(rc.g, rc.w, rc.u0, rc.v0, rc.u, rc.lo, rc.d, i, j);
        break;
    default:
        if (plain) first_node_f32c<KIND13, true>(rc.g, rc.w, rc.u0, rc.v0, rc.u, rc.lo, rc.d, i, j);
        else first_node_f32c<KIND13>(rc.g, rc.w, rc.u0, rc.v0, rc.u, rc.lo, rc.d, i, j);
        break;
    }
}

__global__ __launch_bounds__(BX* BY) void k_copy3_batch(const CopyRec3* __restrict__ recs,
                                                        const int* __restrict__ prefix, int count)
{
    const int b = (int)blockIdx.x;
    const int r = find_record(prefix, count, b);
    const CopyRec3 rc = recs[r];
    const int t = b - prefix[r];
    const int tx = (rc.g.nx + BX - 1) / BX;
    const int i = (t % tx) * BX + threadIdx.x, j = (t / tx) * BY + threadIdx.y;
    if (i >= rc.g.nx || j >= rc.g.ny) return;
    const size_t o = (size_t)j * rc.g.ld + i;
#pragma unroll
    for (int f = 0; f < 3; ++f) rc.dst[f][o] = rc.src[f][o];
}

__global__ void k_fill_i32(int* p, int n, int v)
{
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k < n) p[k] = v;
}

template <int K>
__global__ __launch_bounds__(BX* BY) void k_step_f64(Grid g, StepW64 w, const double* u_prev,
                                                     const double* __restrict__ u_cur, double* u_next)
{
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    double r = 0.0;
    if (interior(g, i, j)) {
        const Nbh<double> v = gather<K>(u_cur, g, i, j);
        r = f64_update(v.C, u_prev[(size_t)j * g.ld + i], f64_incr<K>(v, w.w10, w.w11, w.w20, w.wx));
    }
    u_next[(size_t)j * g.ld + i] = r;
}

template <int K>
__global__ __launch_bounds__(BX* BY) void k_step_f32c(Grid g, StepW32 w, const float* __restrict__ u,
                                                      const float* __restrict__ lo, const float* __restrict__ d,
                                                      float* __restrict__ u2, float* __restrict__ lo2,
                                                      float* __restrict__ d2)
{
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    float ru = 0.f, rl = 0.f, rd = 0.f;
    const size_t o = (size_t)j * g.ld + i;
    if (interior(g, i, j)) {
        const Nbh<float> a = gather<K>(u, g, i, j);
        const Nbh<float> b = gather<K>(lo, g, i, j);
        const float s = f32c_incr<K>(a, b, w.wc, w.w10, w.w11, w.w20, w.wx, w.wxl);
        f32c_update(s, a.C, b.C, d[o], ru, rl, rd);
    }
    u2[o] = ru;
    lo2[o] = rl;
    d2[o] = rd;
}

__global__ __launch_bounds__(BX* BY) void k_init(Grid g, const double* __restrict__ p, const double* __restrict__ c,
                                                 float* __restrict__ u, float* __restrict__ lo,
                                                 float* __restrict__ d)
{
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const size_t o = (size_t)j * g.ld + i;
    float ru, rl, rd;
    f32c_split(c[o], p[o], ru, rl, rd);
    u[o] = ru;
    lo[o] = rl;
    d[o] = rd;
}

__global__ __launch_bounds__(BX* BY) void k_export(Grid g, const float* __restrict__ u, const float* __restrict__ lo,
                                                   double* __restrict__ out)
{
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const size_t o = (size_t)j * g.ld + i;
    out[o] = f32c_join(u[o], lo[o]);
}

__global__ __launch_bounds__(BX* BY) void k_copy3(Grid g, const float* a, const float* b, const float* c, float* a2,
                                                  float* b2, float* c2)
{
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const size_t o = (size_t)j * g.ld + i;
    if (a) a2[o] = a[o];
    if (b) b2[o] = b[o];
    if (c) c2[o] = c[o];
}

__global__ __launch_bounds__(BX* BY) void k_copy2d(Grid g, const double* a, const double* b, double* a2, double* b2)
{
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const size_t o = (size_t)j * g.ld + i;
    if (a) a2[o] = a[o];
    if (b) b2[o] = b[o];
}

__global__ __launch_bounds__(BX* BY) void k_copy_interior(Grid g, const double* __restrict__ a,
                                                          double* __restrict__ b)
{
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const size_t o = (size_t)j * g.ld + i;
    b[o] = interior(g, i, j) ? a[o] : 0.0;
}

__global__ __launch_bounds__(BX* BY) void k_swap(Grid g, double* a, double* b)
{
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const size_t o = (size_t)j * g.ld + i;
    const double t = a[o];
    a[o] = b[o];
    b[o] = t;
}

dim3 grid_of(const Grid& g) { return dim3((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY); }
const dim3 kBlock(BX, BY);

}  // namespace

#define W2D_DISPATCH_KIND(kind, KERNEL, ...)                                          \
    switch (kind) {                                                                   \
    case KIND5: KERNEL<KIND5><<<grid_of(g), kBlock, 0, s>>>(__VA_ARGS__); break;    \
    case KIND9: KERNEL<KIND9><<<grid_of(g), kBlock, 0, s>>>(__VA_ARGS__); break;    \
    case KIND13: KERNEL<KIND13><<<grid_of(g), kBlock, 0, s>>>(__VA_ARGS__); break;  \
    default: return hipErrorInvalidValue;                                             \
    }                                                                                 \
    return hipGetLastError();

hipError_t simple_first_step(const Grid& g, int kind, const FirstW& w, const double* u0, const double* v0,
                             double* u1, hipStream_t s)
{
    W2D_DISPATCH_KIND(kind, k_first_step, g, w, u0, v0, u1)
}

hipError_t simple_first_step_f32c(const Grid& g, int kind, const FirstW& w, const double* u0, const double* v0,
                                  float* u, float* lo, float* d, hipStream_t s)
{
    W2D_DISPATCH_KIND(kind, k_first_step_f32c, g, w, u0, v0, u, lo, d)
}

hipError_t simple_step_f64(const Grid& g, int kind, const StepW64& w, const double* u_prev, const double* u_cur,
                           double* u_next, hipStream_t s)
{
    W2D_DISPATCH_KIND(kind, k_step_f64, g, w, u_prev, u_cur, u_next)
}

hipError_t simple_step_f32c(const Grid& g, int kind, const StepW32& w, const float* u, const float* lo,
                            const float* d, float* u2, float* lo2, float* d2, hipStream_t s)
{
    W2D_DISPATCH_KIND(kind, k_step_f32c, g, w, u, lo, d, u2, lo2, d2)
}

hipError_t f32c_init(const Grid& g, const double* u_prev, const double* u_cur, float* u, float* lo, float* d,
                     hipStream_t s)
{
    k_init<<<grid_of(g), kBlock, 0, s>>>(g, u_prev, u_cur, u, lo, d);
    return hipGetLastError();
}

hipError_t f32c_export(const Grid& g, const float* u, const float* lo, double* out, hipStream_t s)
{
    k_export<<<grid_of(g), kBlock, 0, s>>>(g, u, lo, out);
    return hipGetLastError();
}

hipError_t copy_f32x3(const Grid& g, const float* a, const float* b, const float* c, float* a2, float* b2,
                      float* c2, hipStream_t s)
{
    k_copy3<<<grid_of(g), kBlock, 0, s>>>(g, a, b, c, a2, b2, c2);
    return hipGetLastError();
}

int node_tiles(const Grid& g) { return ((g.nx + BX - 1) / BX) * ((g.ny + BY - 1) / BY); }

hipError_t first_step_f32c_batch(const FirstRecF32C* recs, const int* prefix, int count, int blocks, hipStream_t s)
{
    if (count <= 0 || blocks <= 0) return hipSuccess;
    k_first_step_f32c_batch<<<blocks, kBlock, 0, s>>>(recs, prefix, count);
    return hipGetLastError();
}

hipError_t copy_f32x3_batch(const CopyRec3* recs, const int* prefix, int count, int blocks, hipStream_t s)
{
    if (count <= 0 || blocks <= 0) return hipSuccess;
    k_copy3_batch<<<blocks, kBlock, 0, s>>>(recs, prefix, count);
    return hipGetLastError();
}

hipError_t fill_i32(int* p, int n, int v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<(n + 255) / 256, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t copy_f64x2(const Grid& g, const double* a, const double* b, double* a2, double* b2, hipStream_t s)
{
    k_copy2d<<<grid_of(g), kBlock, 0, s>>>(g, a, b, a2, b2);
    return hipGetLastError();
}

hipError_t copy_interior_f64(const Grid& g, const double* a, double* b, hipStream_t s)
{
    k_copy_interior<<<grid_of(g), kBlock, 0, s>>>(g, a, b);
    return hipGetLastError();
}

hipError_t swap_f64(const Grid& g, double* a, double* b, hipStream_t s)
{
    k_swap<<<grid_of(g), kBlock, 0, s>>>(g, a, b);
    return hipGetLastError();
}

}  // namespace w2d

// Kernels for schemes whose stencil reaches up to three lines from the
// centre: the schemes that the construction of Sec. 4-5 builds from larger
// monomial sets (the complete set of degree 6 weights the classes (2,1) and
// (3,0) besides the 13-point ones).  One level per launch: a block of 64 x 8
// threads stages its 64 x 32 tile of the level, with a halo of three nodes
// on every side, in LDS (the boundary rule applied while loading, plain
// loads for tiles inside the grid), and each thread then forms the class
// sums of four nodes of one column from LDS.
//
// Node classes (q1, q2), q1 >= q2 >= 0, in this order: (1,0), (1,1), (2,0),
// (2,1), (2,2), (3,0), (3,1), (3,2), (3,3).  A class holds the rotations of
// (q1, q2) and, when q1 != q2 and q2 != 0, those of (q2, q1) as well; its
// sum is taken over (node - centre), opposite nodes paired first, the same
// way the 5/9/13-point kernels form their rotation sums.
#include "wide.h"

namespace w2d {
namespace {

constexpr int WX = 64, WY = 8, RPT = 4, HALO = 3;  // threads x, y; rows per thread
constexpr int BH = WY * RPT;                        // rows per block
constexpr int TX = WX + 2 * HALO, TY = BH + 2 * HALO;
constexpr int kQ[kWideClasses][2] = {{1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}, {3, 0}, {3, 1}, {3, 2}, {3, 3}};

// Value of node (i, j) under the boundary rule, for (i, j) up to three
// lines outside the grid.  Dirichlet: boundary nodes read as 0, a node
// outside reads as minus its mirror image (a mirror that lands on the
// boundary or beyond the far side reads as 0: no updated node reads those);
// periodic: indices wrap around.
template <typename T>
__device__ __forceinline__ T wide_load(const T* __restrict__ p, const Grid& g, int i, int j)
{
    const int nx = g.nx, ny = g.ny;
    if (g.periodic) {
        i %= nx;
        j %= ny;
        i += (i < 0) ? nx : 0;
        j += (j < 0) ? ny : 0;
        return p[(size_t)j * g.ld + i];
    }
    bool neg = false;
    if (i < 0) { i = -i; neg = !neg; }
    else if (i > nx - 1) { i = 2 * (nx - 1) - i; neg = !neg; }
    if (j < 0) { j = -j; neg = !neg; }
    else if (j > ny - 1) { j = 2 * (ny - 1) - j; neg = !neg; }
    if (i <= 0 || i >= nx - 1 || j <= 0 || j >= ny - 1) return T(0);
    const T v = p[(size_t)j * g.ld + i];
    return neg ? -v : v;
}

// Stage the block's tile (block origin x0, y0; tile origin three nodes
// above and to the left) of one field in LDS.  A tile whose nodes are all
// read as stored (inside the grid, off its boundary under the Dirichlet
// rule) is loaded without the boundary rule; the choice is the same for
// every thread of the block.
template <typename T>
__device__ __forceinline__ void load_tile(T (*t)[TX], const T* __restrict__ p, const Grid& g, int x0, int y0)
{
    const int xa = x0 - HALO, ya = y0 - HALO;
    const int lo = g.periodic ? 0 : 1;
    const bool plain = xa >= lo && ya >= lo && xa + TX - 1 <= g.nx - 1 - lo && ya + TY - 1 <= g.ny - 1 - lo;
    const int tx0 = threadIdx.x, tx1 = threadIdx.x + WX;
    if (plain) {
        const T* q = p + (size_t)ya * g.ld + xa;
        for (int ty = threadIdx.y; ty < TY; ty += WY) {
            t[ty][tx0] = q[(size_t)ty * g.ld + tx0];
            if (tx1 < TX) t[ty][tx1] = q[(size_t)ty * g.ld + tx1];
        }
    } else {
        for (int ty = threadIdx.y; ty < TY; ty += WY) {
            t[ty][tx0] = wide_load(p, g, xa + tx0, ya + ty);
            if (tx1 < TX) t[ty][tx1] = wide_load(p, g, xa + tx1, ya + ty);
        }
    }
}

// Sum over class c of (node - centre) at tile position (ly, lx).
template <typename T, int C>
__device__ __forceinline__ T class_sum(const T (*t)[TX], int ly, int lx)
{
    constexpr int q1 = kQ[C][0], q2 = kQ[C][1];
    const T c = t[ly][lx];
    // (q1, q2), (-q1, -q2), (-q2, q1), (q2, -q1): offsets (dx, dy) at t[ly + dy][lx + dx].
    T s = ((t[ly + q2][lx + q1] - c) + (t[ly - q2][lx - q1] - c)) +
          ((t[ly + q1][lx - q2] - c) + (t[ly - q1][lx + q2] - c));
    if constexpr (q2 != 0 && q2 != q1) {
        // (q2, q1), (-q2, -q1), (-q1, q2), (q1, -q2)
        s = s + (((t[ly + q1][lx + q2] - c) + (t[ly - q1][lx - q2] - c)) +
                 ((t[ly + q2][lx - q1] - c) + (t[ly - q2][lx + q1] - c)));
    }
    return s;
}

// sum_c w[c] S_c in class order, skipping classes without weight.
template <int C = 0>
__device__ __forceinline__ double wide_sum(const double (*t)[TX], int ly, int lx, const double* w, double s)
{
    if constexpr (C < kWideClasses) {
        if (w[C] != 0.0) s = fmaT(w[C], class_sum<double, C>(t, ly, lx), s);
        return wide_sum<C + 1>(t, ly, lx, w, s);
    } else {
        return s;
    }
}

// Increment of the compensated level u + lo: sum_c (w[c] + wl[c]) (S_c(u) +
// S_c(lo)), each class sum formed from differences before the two fields
// are added, each weight applied as its two-float pair.
template <int C = 0>
__device__ __forceinline__ float wide_sum_f32c(const float (*tu)[TX], const float (*tl)[TX], int ly, int lx,
                                               const float* w, const float* wl, float s)
{
    if constexpr (C < kWideClasses) {
        if (w[C] != 0.f) s = s + mul_w2(w[C], wl[C], class_sum<float, C>(tu, ly, lx) + class_sum<float, C>(tl, ly, lx));
        return wide_sum_f32c<C + 1>(tu, tl, ly, lx, w, wl, s);
    } else {
        return s;
    }
}

__device__ __forceinline__ bool wide_interior(const Grid& g, int i, int j)
{
    return g.periodic || (i > 0 && i < g.nx - 1 && j > 0 && j < g.ny - 1);
}

// First step (eq. A1) for FP64 output or split into the compensated state.
template <bool F32C>
__global__ __launch_bounds__(WX* WY) void k_wide_first(Grid g, WideFirstW w, const double* __restrict__ u0,
                                                       const double* __restrict__ v0, double* __restrict__ u1,
                                                       float* __restrict__ u, float* __restrict__ lo,
                                                       float* __restrict__ d)
{
    __shared__ double ta[TY][TX], tb[TY][TX];
    const int x0 = blockIdx.x * WX, y0 = blockIdx.y * BH;
    load_tile(ta, u0, g, x0, y0);
    if (w.poisson) load_tile(tb, v0, g, x0, y0);
    __syncthreads();
    const int i = x0 + threadIdx.x;
    if (i >= g.nx) return;
    const int lx = threadIdx.x + HALO;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ry = threadIdx.y * RPT + k, j = y0 + ry;
        if (j >= g.ny) break;
        const int ly = ry + HALO;
        double r = 0.0, prev = 0.0;
        const bool in = wide_interior(g, i, j);
        if (in) {
            const double c = ta[ly][lx];
            const double sa = wide_sum(ta, ly, lx, w.a, 0.0);
            const double sb = w.poisson ? wide_sum(tb, ly, lx, w.b, 0.0) : 0.0;
            r = first_update(c, sa, v0[(size_t)j * g.ld + i], sb, w.tau);
            prev = c;
        }
        const size_t o = (size_t)j * g.ld + i;
        if constexpr (F32C) {
            float ru = 0.f, rl = 0.f, rd = 0.f;
            if (in) f32c_split(r, prev, ru, rl, rd);
            u[o] = ru;
            lo[o] = rl;
            d[o] = rd;
        } else {
            u1[o] = r;
        }
    }
}

// FP64 two-step update (eq. A2).  u_next may equal u_prev: each thread reads
// its own nodes of u_prev before writing them, and never reads other nodes
// of it.
__global__ __launch_bounds__(WX* WY) void k_wide_step_f64(Grid g, WideW64 w, const double* u_prev,
                                                          const double* __restrict__ u_cur, double* u_next)
{
    __shared__ double t[TY][TX];
    const int x0 = blockIdx.x * WX, y0 = blockIdx.y * BH;
    load_tile(t, u_cur, g, x0, y0);
    __syncthreads();
    const int i = x0 + threadIdx.x;
    if (i >= g.nx) return;
    const int lx = threadIdx.x + HALO;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ry = threadIdx.y * RPT + k, j = y0 + ry;
        if (j >= g.ny) break;
        const size_t o = (size_t)j * g.ld + i;
        double r = 0.0;
        if (wide_interior(g, i, j)) {
            const int ly = ry + HALO;
            r = f64_update(t[ly][lx], u_prev[o], wide_sum(t, ly, lx, w.w, 0.0));
        }
        u_next[o] = r;
    }
}

// Compensated FP32 two-step update: (u, lo, d) -> (u2, lo2, d2).
__global__ __launch_bounds__(WX* WY) void k_wide_step_f32c(Grid g, WideW32 w, const float* __restrict__ u,
                                                           const float* __restrict__ lo,
                                                           const float* __restrict__ d, float* __restrict__ u2,
                                                           float* __restrict__ lo2, float* __restrict__ d2)
{
    __shared__ float tu[TY][TX], tl[TY][TX];
    const int x0 = blockIdx.x * WX, y0 = blockIdx.y * BH;
    load_tile(tu, u, g, x0, y0);
    load_tile(tl, lo, g, x0, y0);
    __syncthreads();
    const int i = x0 + threadIdx.x;
    if (i >= g.nx) return;
    const int lx = threadIdx.x + HALO;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ry = threadIdx.y * RPT + k, j = y0 + ry;
        if (j >= g.ny) break;
        const size_t o = (size_t)j * g.ld + i;
        float ru = 0.f, rl = 0.f, rd = 0.f;
        if (wide_interior(g, i, j)) {
            const int ly = ry + HALO;
            const float s = wide_sum_f32c(tu, tl, ly, lx, w.w, w.wl, 0.f);
            f32c_update(s, tu[ly][lx], tl[ly][lx], d[o], ru, rl, rd);
        }
        u2[o] = ru;
        lo2[o] = rl;
        d2[o] = rd;
    }
}

dim3 wide_grid(const Grid& g) { return dim3((g.nx + WX - 1) / WX, (g.ny + BH - 1) / BH); }

}  // namespace

hipError_t wide_first_step(const Grid& g, const WideFirstW& w, const double* u0, const double* v0, double* u1,
                           hipStream_t s)
{
    k_wide_first<false><<<wide_grid(g), dim3(WX, WY), 0, s>>>(g, w, u0, v0, u1, nullptr, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t wide_first_step_f32c(const Grid& g, const WideFirstW& w, const double* u0, const double* v0, float* u,
                                float* lo, float* d, hipStream_t s)
{
    k_wide_first<true><<<wide_grid(g), dim3(WX, WY), 0, s>>>(g, w, u0, v0, nullptr, u, lo, d);
    return hipGetLastError();
}

hipError_t wide_step_f64(const Grid& g, const WideW64& w, const double* u_prev, const double* u_cur,
                         double* u_next, hipStream_t s)
{
    k_wide_step_f64<<<wide_grid(g), dim3(WX, WY), 0, s>>>(g, w, u_prev, u_cur, u_next);
    return hipGetLastError();
}

hipError_t wide_step_f32c(const Grid& g, const WideW32& w, const float* u, const float* lo, const float* d,
                          float* u2, float* lo2, float* d2, hipStream_t s)
{
    k_wide_step_f32c<<<wide_grid(g), dim3(WX, WY), 0, s>>>(g, w, u, lo, d, u2, lo2, d2);
    return hipGetLastError();
}

}  // namespace w2d

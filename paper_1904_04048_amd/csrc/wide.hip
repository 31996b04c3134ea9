// Kernels for schemes whose stencil reaches up to three lines from the
// centre: the schemes that the construction of Sec. 4-5 builds from larger
// monomial sets (the complete set of degree 6 weights the classes (2,1) and
// (3,0) besides the 13-point ones).  One level per launch: a block of 64 x 8
// threads stages its tile of the level, with a halo of three nodes on every
// side, in LDS (the boundary rule applied while loading, plain loads for
// tiles inside the grid), and each thread forms the class sums of four
// nodes of one column from LDS.  The FP64 update so moves about as many
// bytes per second as a device copy.  The compensated update, which does
// about twice the arithmetic per node, streams instead: each wave walks
// down a strip of 64 columns, loading rows three ahead of their use, and
// keeps the 7 x 7 neighbourhood of both fields of its node in registers (a
// ring of rows; each new row passes through a wave-private LDS row so that
// every lane picks up its seven columns).  No block barrier, no tile
// reloads.
//
// Node classes (q1, q2), q1 >= q2 >= 0, in this order: (1,0), (1,1), (2,0),
// (2,1), (2,2), (3,0), (3,1), (3,2), (3,3).  A class holds the rotations of
// (q1, q2) and, when q1 != q2 and q2 != 0, those of (q2, q1) as well; its
// sum is taken over (node - centre), opposite nodes paired first, the same
// way the 5/9/13-point kernels form their rotation sums.
#include <algorithm>
#include <map>
#include <mutex>

#include "wide.h"

namespace w2d {
namespace {

constexpr int WX = 64, WY = 8, RPT = 4, HALO = 3;  // threads x, y; rows per thread
constexpr int BH = WY * RPT;                        // rows per block
constexpr int TX = WX + 2 * HALO, TY = BH + 2 * HALO;
constexpr int NR = 2 * HALO + 1;                    // rows and columns of a node's neighbourhood
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

// The same sum from a thread's register neighbourhood: w[(cs + dy) mod NR]
// [HALO + dx] holds the node at offset (dx, dy) from the centre, cs being
// the centre row's slot (a compile-time constant once the row loop is
// unrolled).  Same operands in the same order as class_sum.
template <typename T, int C>
__device__ __forceinline__ T class_sum_w(const T (&w)[NR][NR], int cs)
{
    constexpr int q1 = kQ[C][0], q2 = kQ[C][1];
    auto at = [&](int dy, int dx) { return w[(cs + dy + NR) % NR][HALO + dx]; };
    const T c = at(0, 0);
    T s = ((at(q2, q1) - c) + (at(-q2, -q1) - c)) + ((at(q1, -q2) - c) + (at(-q1, q2) - c));
    if constexpr (q2 != 0 && q2 != q1) s = s + (((at(q1, q2) - c) + (at(-q1, -q2) - c)) + ((at(q2, -q1) - c) + (at(-q2, q1) - c)));
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

template <int C = 0>
__device__ __forceinline__ float wide_sum_f32c_w(const float (&wu)[NR][NR], const float (&wl)[NR][NR], int cs,
                                                 const float* w, const float* wlo, float s)
{
    if constexpr (C < kWideClasses) {
        if (w[C] != 0.f) s = s + mul_w2(w[C], wlo[C], class_sum_w<float, C>(wu, cs) + class_sum_w<float, C>(wl, cs));
        return wide_sum_f32c_w<C + 1>(wu, wl, cs, w, wlo, s);
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

// Compensated FP32 two-step update: (u, lo, d) -> (u2, lo2, d2), by waves
// streaming down strips (see the top of the file).
constexpr int SWW = 64;            // output columns per wave, one per lane
constexpr int PFW = 2;             // rows loaded ahead of their first use
constexpr int kWideWaves = 4;      // waves per block (independent: no barrier)
constexpr int kWideRounds = 4;     // work items per resident wave the segment height aims at

// Grid node that node x of the extended line stands for (idx) and the
// factor its value is read with: the rule of wide_load, 1 or -1 (mirror
// image), or 0 (a boundary line, or a mirror beyond it; idx is then 0).
__device__ __forceinline__ int wide_map(int x, int n, bool periodic, int& idx)
{
    if (periodic) {
        int m = x % n;
        m += (m < 0) ? n : 0;
        idx = m;
        return 1;
    }
    int sg = 1;
    if (x < 0) {
        x = -x;
        sg = -sg;
    } else if (x > n - 1) {
        x = 2 * (n - 1) - x;
        sg = -sg;
    }
    if (x <= 0 || x >= n - 1) {
        idx = 0;
        return 0;
    }
    idx = x;
    return sg;
}

// Ordering of a wave's LDS accesses across its lanes: the wave's LDS
// operations execute in program order, so only the compiler must keep
// them in order (a lane's read of another lane's write is invisible to
// its per-thread analysis).
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(SWW* kWideWaves) void k_wide_step_f32c(Grid g, WideW32 w, const float* __restrict__ u,
                                                                     const float* __restrict__ lo,
                                                                     const float* __restrict__ d,
                                                                     float* __restrict__ u2, float* __restrict__ lo2,
                                                                     float* __restrict__ d2, int segw)
{
    __shared__ float rowbuf[kWideWaves][2][SWW + 2 * HALO];
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int nx = g.nx, ny = g.ny;
    const int nstrips = (nx + SWW - 1) / SWW, nseg = (ny + segw - 1) / segw;
    const int item = __builtin_amdgcn_readfirstlane((int)blockIdx.x * kWideWaves + wave);
    if (item >= nstrips * nseg) return;  // whole waves; no barrier follows
    const int x0 = (item % nstrips) * SWW, y0 = (item / nstrips) * segw, y1 = min(y0 + segw, ny);
    const bool per = g.periodic != 0;
    // The lane's output column xm; lanes 0..5 also load one halo column
    // (three on each side).  LDS slot s of a row holds column x0 - 3 + s.
    const int xm = x0 + lane;
    const bool has_h = lane < 2 * HALO;
    const int xh = (lane < HALO) ? x0 - HALO + lane : x0 + SWW + lane - HALO;
    int im = 0, ih = 0;
    const int sm = wide_map(xm, nx, per, im);
    const int sh = has_h ? wide_map(xh, nx, per, ih) : 0;
    const int slot_m = HALO + lane, slot_h = (lane < HALO) ? lane : SWW + lane;
    // Columns read as stored for every lane (no sign or zero to apply).
    const int lb = per ? 0 : 1;
    const bool plain_cols = x0 - HALO >= lb && x0 + SWW - 1 + HALO <= nx - 1 - lb;
    float* const bu = rowbuf[wave][0];
    float* const bl = rowbuf[wave][1];

    // Row r of the extended grid, both fields, main and halo column.
    auto load_row = [&](int r, float (&v)[2][2]) {
        int jr;
        const int sr = wide_map(r, ny, per, jr);
        const size_t ro = (size_t)jr * g.ld;
        const float a0 = u[ro + im], a1 = lo[ro + im];
        float b0 = 0.f, b1 = 0.f;
        if (has_h) {
            b0 = u[ro + ih];
            b1 = lo[ro + ih];
        }
        if (plain_cols && sr == 1) {
            v[0][0] = a0;
            v[1][0] = a1;
            v[0][1] = b0;
            v[1][1] = b1;
        } else {
            const float fm = (float)(sr * sm), fh = (float)(sr * sh);
            v[0][0] = (fm != 0.f) ? a0 * fm : 0.f;
            v[1][0] = (fm != 0.f) ? a1 * fm : 0.f;
            v[0][1] = (fh != 0.f) ? b0 * fh : 0.f;
            v[1][1] = (fh != 0.f) ? b1 * fh : 0.f;
        }
    };
    // d at output row j (clamped into the grid: rows and columns without an
    // output are loaded but never used).
    const int xd = min(xm, nx - 1);
    auto load_d = [&](int j) { return d[(size_t)min(j, ny - 1) * g.ld + xd]; };

    float W[2][NR][NR];   // [field][row slot][column]: row y0 + k sits in slot k mod 7
    float st[NR][2][2];   // loaded rows on their way to the window, by the same slot
    float dr[NR];         // d of output rows, by slot
    auto enter = [&](const float (&v)[2][2], int slot) {
        wave_lds_order();
        bu[slot_m] = v[0][0];
        bl[slot_m] = v[1][0];
        if (has_h) {
            bu[slot_h] = v[0][1];
            bl[slot_h] = v[1][1];
        }
        wave_lds_order();
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            W[0][slot][c] = bu[lane + c];
            W[1][slot][c] = bl[lane + c];
        }
    };
#pragma unroll
    for (int r = -HALO; r < HALO; ++r) {
        float v[2][2];
        load_row(y0 + r, v);
        enter(v, (r + NR) % NR);
    }
#pragma unroll
    for (int r = 0; r < PFW; ++r) {
        load_row(y0 + HALO + r, st[(HALO + r) % NR]);
        dr[r % NR] = load_d(y0 + r);
    }
    for (int k0 = 0; y0 + k0 < y1; k0 += NR) {
#pragma unroll
        for (int kk = 0; kk < NR; ++kk) {
            const int j = y0 + k0 + kk;
            enter(st[(kk + HALO) % NR], (kk + HALO) % NR);
            load_row(j + HALO + PFW, st[(kk + HALO + PFW) % NR]);
            dr[(kk + PFW) % NR] = load_d(j + PFW);
            if (j < y1 && xm < nx) {
                const size_t o = (size_t)j * g.ld + xm;
                float ru = 0.f, rl = 0.f, rd = 0.f;
                if (wide_interior(g, xm, j)) {
                    const float s = wide_sum_f32c_w(W[0], W[1], kk, w.w, w.wl, 0.f);
                    f32c_update(s, W[0][kk][HALO], W[1][kk][HALO], dr[kk], ru, rl, rd);
                }
                u2[o] = ru;
                lo2[o] = rl;
                d2[o] = rd;
            }
        }
    }
}

dim3 wide_grid(const Grid& g) { return dim3((g.nx + WX - 1) / WX, (g.ny + BH - 1) / BH); }

// Output rows per wave of the compensated update: a multiple of 7 (whole
// turns of the register ring), the largest that still gives about
// kWideRounds work items per resident wave (shorter segments reload more
// rows above and below, taller ones leave waves idle on small grids).
int wide_stream_rows(const Grid& g)
{
    static std::mutex mu;
    static std::map<int, int> slots;  // resident waves per device
    int dev = 0;
    (void)hipGetDevice(&dev);
    int res;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = slots.find(dev);
        if (it == slots.end()) {
            int nb = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_wide_step_f32c),
                                                             SWW * kWideWaves, 0) != hipSuccess || nb < 1)
                nb = 1;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
                cus = 256;
            (void)hipGetLastError();
            it = slots.emplace(dev, nb * kWideWaves * cus).first;
        }
        res = it->second;
    }
    const long long groups = (long long)((g.nx + SWW - 1) / SWW) * ((g.ny + NR - 1) / NR);
    const long long m = groups / ((long long)kWideRounds * res);
    return NR * (int)std::max(1LL, std::min(16LL, m));
}

int wide_stream_blocks(const Grid& g, int segw)
{
    const int items = ((g.nx + SWW - 1) / SWW) * ((g.ny + segw - 1) / segw);
    return (items + kWideWaves - 1) / kWideWaves;
}

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
    const int segw = wide_stream_rows(g);
    k_wide_step_f32c<<<wide_stream_blocks(g, segw), SWW * kWideWaves, 0, s>>>(g, w, u, lo, d, u2, lo2, d2, segw);
    return hipGetLastError();
}

}  // namespace w2d

// Temporally blocked two-step kernels for gfx950.
//
// Each wavefront owns a work item: a strip of 64*CW consecutive columns
// (CW contiguous columns per lane) and a segment of output rows.  It streams
// down the rows once, keeping for every time level t < DEPTH a window of the
// last 2R+1 rows in registers, and computes level t at row j - t*R as soon
// as level t-1 has row j - (t-1)*R.  One pass over memory therefore advances
// DEPTH time levels: level 0 is read once and level DEPTH written once.
//
// Neighbours along x come from the adjacent lanes through DPP whole-wave
// shifts (no LDS, no barriers, no inter-wave communication); the strip
// carries R*DEPTH halo columns on each side, whose values go stale one
// stencil radius per level and are never stored.  Segments overlap by
// R*DEPTH rows for the same reason.  Rows and columns at and beyond the grid
// boundary follow the boundary rule after every level: boundary nodes are 0,
// the line one outside is the odd reflection of the line one inside
// (13-point stencil only).
//
// Per-node arithmetic is the same inline code as in the one-node-per-thread
// kernels (point.h), so results are bit-identical to them for every DEPTH,
// segment length and strip width.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>

#include "w2d.h"

namespace w2d {
namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;

__device__ __forceinline__ int dpp_from_left(int x)  // lane l receives lane l-1
{
    return __builtin_amdgcn_update_dpp(0, x, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_from_right(int x)  // lane l receives lane l+1
{
    return __builtin_amdgcn_update_dpp(0, x, 0x130 /* wave_shl:1 */, 0xf, 0xf, false);
}
__device__ __forceinline__ float from_left(float x) { return __int_as_float(dpp_from_left(__float_as_int(x))); }
__device__ __forceinline__ float from_right(float x) { return __int_as_float(dpp_from_right(__float_as_int(x))); }
__device__ __forceinline__ double from_left(double x)
{
    const long long v = __double_as_longlong(x);
    const int lo = dpp_from_left((int)v), hi = dpp_from_left((int)(v >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_right(double x)
{
    const long long v = __double_as_longlong(x);
    const int lo = dpp_from_right((int)v), hi = dpp_from_right((int)(v >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Precision policies.  NW "window" fields need stencil neighbours; the one
// "point" field is read only at the node itself.
struct PF64 {
    using T = double;
    static constexpr int NW = 1;  // u^k
    using W = StepW64;           // point field: u^{k-1}
};
struct PF32C {
    using T = float;
    static constexpr int NW = 2;  // u, lo
    using W = StepW32;           // point field: d
};

template <typename T>
struct SArgs {
    Grid g;
    int nstrips, nwork, rows;
    const T* in_w0;
    const T* in_w1;
    const T* in_p;
    T* out_w0;
    T* out_w1;
    T* out_p;  // may be NULL (FP64 in place)
};

constexpr int floor_div(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }
constexpr int mod_c(int a, int b) { return ((a % b) + b) % b; }

// Halo columns per strip side, rounded up to even so that every lane's
// column pair starts at an even column (8- or 16-byte aligned vectors).
template <int R, int DEPTH>
constexpr int halo_cols() { return (R * DEPTH + 1) & ~1; }

// Raw buffer resources give loads and stores a scalar row offset and a
// per-lane column offset that never changes along the stream, so the
// address arithmetic stays off the vector ALU.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename T, int CW>
struct Vec {
    T v[CW];
};

template <typename T, int CW>
__device__ __forceinline__ Vec<T, CW> buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    static_assert(sizeof(T) * CW == 8 || sizeof(T) * CW == 16, "vector width");
    if constexpr (sizeof(T) * CW == 8)
        return __builtin_bit_cast(Vec<T, CW>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
        return __builtin_bit_cast(Vec<T, CW>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

template <typename T, int CW>
__device__ __forceinline__ void buf_store(const Vec<T, CW>& x, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                          uint32_t soff)
{
    if constexpr (sizeof(T) * CW == 8) {
        using V = unsigned __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, x), r, voff, soff, 0);
    } else {
        using V = unsigned __attribute__((ext_vector_type(4)));
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V, x), r, voff, soff, 0);
    }
}

template <typename T>
__device__ __forceinline__ void buf_store1(T x, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, voff, soff, 0);
    } else {
        using V = unsigned __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, x), r, voff, soff, 0);
    }
}

// Compensated single precision with differences carried from row to row:
// going down the rows of one level, what row y-1 computed for its northern
// neighbours serves row y as its southern ones.  Every operation and its
// operands are those of f32c_incr (a + (-b) rounds exactly as a - b), so
// the result is bit-identical to the one-node-per-thread kernels; only
// repeated subtractions are saved.
//   5-point: N - C of u (its negation is the next row's S - C) and the lo
//            row sums lo(i+1) + lo(i-1) of rows y-1 and y.
//   9-point: N - C of u and of lo (the next row's C - S).
//   13-point: the same one row further north, the summed second difference
//            q = Dy u + Dy lo of row y and q(y) - q(y-1).
// Column neighbours beyond the lane's own CW columns come from the adjacent
// lanes (DPP shifts folded into the consuming subtraction or addition).
template <typename T, int CW>
struct Carry {
    T dv[CW];  // N - C of u
    T dl[CW];  // N - C of lo (9-, 13-point)
    T hs0[CW]; // lo(i+1) + lo(i-1) of row y-1 (5-point)
    T hs1[CW]; // lo(i+1) + lo(i-1) of row y (5-point)
    T q[CW];   // q of row y (13-point)
    T eq[CW];  // q(y) - q(y-1) (13-point)
};

template <typename T, int CW>
__device__ __forceinline__ void carry_zero(Carry<T, CW>& c)
{
#pragma unroll
    for (int m = 0; m < CW; ++m) c.dv[m] = c.dl[m] = c.hs0[m] = c.hs1[m] = c.q[m] = c.eq[m] = T(0);
}

// column m + o of a lane's row, o in [-1, 1]
template <typename T, int CW>
__device__ __forceinline__ T lane_col(const T (&r)[CW], int m, int o)
{
    const int c = m + o;
    if (c >= 0 && c < CW) return r[c];
    if (c >= CW) return from_right(r[c - CW]);
    return from_left(r[c + CW]);
}

// Second difference along x of a lane's row: out[m] = d2(r(m+1), r(m), r(m-1)),
// from the first differences e[k] = r(k) - r(k-1), k = 0..CW.
template <typename T, int CW>
__device__ __forceinline__ void row_d2x(const T (&r)[CW], T (&out)[CW])
{
    T e[CW + 1];
    e[0] = r[0] - from_left(r[CW - 1]);
#pragma unroll
    for (int k = 1; k < CW; ++k) e[k] = r[k] - r[k - 1];
    e[CW] = from_right(r[0]) - r[CW - 1];
#pragma unroll
    for (int m = 0; m < CW; ++m) out[m] = e[m + 1] - e[m];
}

template <int K, int CW>
__device__ __forceinline__ void row_update_carry(const float (&Wc)[2][CW], const float (&Wn)[2][CW],
                                                 const float (&Ws)[2][CW], const float (&Wnn)[2][CW],
                                                 const float (&Wss)[2][CW], const float (&Pin)[CW],
                                                 Carry<float, CW>& cr, const StepW32& w, bool update,
                                                 float (&nv)[2][CW], float (&np)[CW])
{
    const float(&U)[CW] = Wc[0];
    const float(&L)[CW] = Wc[1];
    if constexpr (K == KIND5) {
        float dv[CW], hsn[CW];
#pragma unroll
        for (int m = 0; m < CW; ++m) {
            dv[m] = Wn[0][m] - U[m];
            hsn[m] = lane_col(Wn[1], m, 1) + lane_col(Wn[1], m, -1);
        }
        if (update) {
            float eh[CW + 1];
            eh[0] = U[0] - from_left(U[CW - 1]);
#pragma unroll
            for (int k = 1; k < CW; ++k) eh[k] = U[k] - U[k - 1];
            eh[CW] = from_right(U[0]) - U[CW - 1];
#pragma unroll
            for (int m = 0; m < CW; ++m) {
                const float su = mul_w2(w.wx, w.wxl, (eh[m + 1] - eh[m]) + (dv[m] - cr.dv[m]));
                const float sl = fmaT(w.w10, cr.hs1[m] + (Wn[1][m] + Ws[1][m]), w.wc * L[m]);
                f32c_update(su + sl, U[m], L[m], Pin[m], nv[0][m], nv[1][m], np[m]);
            }
        }
#pragma unroll
        for (int m = 0; m < CW; ++m) {
            cr.dv[m] = dv[m];
            cr.hs0[m] = cr.hs1[m];
            cr.hs1[m] = hsn[m];
        }
    } else if constexpr (K == KIND9) {
        float dv[CW], dl[CW];
#pragma unroll
        for (int m = 0; m < CW; ++m) {
            dv[m] = Wn[0][m] - U[m];
            dl[m] = Wn[1][m] - L[m];
        }
        if (update) {
            float q[CW], xu[CW], xl[CW], xq[CW];
#pragma unroll
            for (int m = 0; m < CW; ++m) q[m] = (dv[m] - cr.dv[m]) + (dl[m] - cr.dl[m]);
            row_d2x(U, xu);
            row_d2x(L, xl);
            row_d2x(q, xq);
#pragma unroll
            for (int m = 0; m < CW; ++m) {
                const float s = fmaT(w.w11, xq[m], mul_w2(w.wx, w.wxl, (xu[m] + xl[m]) + q[m]));
                f32c_update(s, U[m], L[m], Pin[m], nv[0][m], nv[1][m], np[m]);
            }
        }
#pragma unroll
        for (int m = 0; m < CW; ++m) {
            cr.dv[m] = dv[m];
            cr.dl[m] = dl[m];
        }
    } else {
        // q of row y+1 from rows y .. y+2; q of row y and q(y) - q(y-1) carried.
        float dv[CW], dl[CW], qn[CW];
#pragma unroll
        for (int m = 0; m < CW; ++m) {
            dv[m] = Wnn[0][m] - Wn[0][m];
            dl[m] = Wnn[1][m] - Wn[1][m];
            qn[m] = (dv[m] - cr.dv[m]) + (dl[m] - cr.dl[m]);
        }
        if (update) {
            float p[CW], xu[CW], xl[CW], xq[CW], xp[CW];
            row_d2x(U, xu);
            row_d2x(L, xl);
#pragma unroll
            for (int m = 0; m < CW; ++m) p[m] = xu[m] + xl[m];
            row_d2x(cr.q, xq);
            row_d2x(p, xp);
#pragma unroll
            for (int m = 0; m < CW; ++m) {
                const float q = cr.q[m];
                float s = fmaT(w.w11, xq[m], mul_w2(w.wx, w.wxl, p[m] + q));
                s = fmaT(w.w20, xp[m] + ((qn[m] - q) - cr.eq[m]), s);
                f32c_update(s, U[m], L[m], Pin[m], nv[0][m], nv[1][m], np[m]);
            }
        }
#pragma unroll
        for (int m = 0; m < CW; ++m) {
            cr.dv[m] = dv[m];
            cr.dl[m] = dl[m];
            cr.eq[m] = qn[m] - cr.q[m];
            cr.q[m] = qn[m];
        }
    }
}

// The double-precision two-step update (one field u; the point field holds
// the previous level) with the same carried differences: f64_incr row by
// row, bit-identical to the one-node-per-thread kernel.  Neighbour columns
// beyond the lane's pair come from the adjacent lanes (two 32-bit DPP moves
// per value).
template <int K, int CW>
__device__ __forceinline__ void row_update_carry(const double (&Wc)[1][CW], const double (&Wn)[1][CW],
                                                 const double (&Ws)[1][CW], const double (&Wnn)[1][CW],
                                                 const double (&Wss)[1][CW], const double (&Pin)[CW],
                                                 double (&cdv)[CW], double (&cq)[CW], double (&ceq)[CW],
                                                 const StepW64& w, bool update, double (&nv)[1][CW],
                                                 double (&np)[CW])
{
    const double(&U)[CW] = Wc[0];
    if constexpr (K == KIND5) {
        double dv[CW];
#pragma unroll
        for (int m = 0; m < CW; ++m) dv[m] = Wn[0][m] - U[m];
        if (update) {
            double eh[CW + 1];
            eh[0] = U[0] - from_left(U[CW - 1]);
#pragma unroll
            for (int k = 1; k < CW; ++k) eh[k] = U[k] - U[k - 1];
            eh[CW] = from_right(U[0]) - U[CW - 1];
#pragma unroll
            for (int m = 0; m < CW; ++m) {
                const double s = w.w10 * ((eh[m + 1] - eh[m]) + (dv[m] - cdv[m]));
                nv[0][m] = f64_update(U[m], Pin[m], s);
                np[m] = U[m];
            }
        }
#pragma unroll
        for (int m = 0; m < CW; ++m) cdv[m] = dv[m];
    } else if constexpr (K == KIND9) {
        double dv[CW];
#pragma unroll
        for (int m = 0; m < CW; ++m) dv[m] = Wn[0][m] - U[m];
        if (update) {
            double q[CW], xu[CW], xq[CW];
#pragma unroll
            for (int m = 0; m < CW; ++m) q[m] = dv[m] - cdv[m];
            row_d2x(U, xu);
            row_d2x(q, xq);
#pragma unroll
            for (int m = 0; m < CW; ++m) {
                const double s = fmaT(w.w11, xq[m], w.wx * (xu[m] + q[m]));
                nv[0][m] = f64_update(U[m], Pin[m], s);
                np[m] = U[m];
            }
        }
#pragma unroll
        for (int m = 0; m < CW; ++m) cdv[m] = dv[m];
    } else {
        double dv[CW], qn[CW];
#pragma unroll
        for (int m = 0; m < CW; ++m) {
            dv[m] = Wnn[0][m] - Wn[0][m];
            qn[m] = dv[m] - cdv[m];
        }
        if (update) {
            double p[CW], xq[CW], xp[CW];
            row_d2x(U, p);
            row_d2x(cq, xq);
            row_d2x(p, xp);
#pragma unroll
            for (int m = 0; m < CW; ++m) {
                const double q = cq[m];
                double s = fmaT(w.w11, xq[m], w.wx * (p[m] + q));
                s = fmaT(w.w20, xp[m] + ((qn[m] - q) - ceq[m]), s);
                nv[0][m] = f64_update(U[m], Pin[m], s);
                np[m] = U[m];
            }
        }
#pragma unroll
        for (int m = 0; m < CW; ++m) {
            cdv[m] = dv[m];
            ceq[m] = qn[m] - cq[m];
            cq[m] = qn[m];
        }
    }
}

// Work decomposition shared by the host and both kernels: strips of SW
// output columns, segments of `rows` output rows, and the rectangle of
// (strip, segment) pairs whose whole stream stays inside the grid interior
// (strips [s_lo, s_lo + ns), segments [g_lo, g_lo + ng)).  The edge strips
// (outside [s_lo, s_lo + ns)), whose items reflect columns on every row and
// run longer, may be cut into shorter segments of their own: nseg_e
// segments of rows_e rows (rows_e = rows in batched and persistent
// launches).
struct Decomp {
    int nstrips, nseg, s_lo, ns, g_lo, ng, nseg_e, rows_e;
};

// Map a boundary work id (the complement of the interior rectangle) to
// (strip, segment) and the item's segment height.  One segmentation: first
// every strip of the segments outside the interior range, then the edge
// strips of the interior segments (a persistent launch then finishes the
// rows above the interior first, which the next pass's items there wait
// for).  Edge strips in segments of their own: first every segment of the
// edge strips, then the interior strips' segments outside the interior
// range.
__device__ __forceinline__ void boundary_item(const Decomp& d, int rows, int wid, int& strip, int& seg, int& h)
{
    const int ne = d.nstrips - d.ns;
    h = rows;
    if (d.rows_e == rows) {
        const int outer = (d.nseg - d.ng) * d.nstrips;
        if (wid < outer) {
            const int k = wid / d.nstrips;
            strip = wid % d.nstrips;
            seg = (k < d.g_lo) ? k : k + d.ng;
        } else {
            const int w2 = wid - outer;
            seg = d.g_lo + w2 / ne;
            const int k = w2 % ne;
            strip = (k < d.s_lo) ? k : k + d.ns;
        }
        return;
    }
    const int first = ne * d.nseg_e;
    if (wid < first) {
        const int k = wid % ne;
        strip = (k < d.s_lo) ? k : k + d.ns;
        seg = wid / ne;
        h = d.rows_e;
    } else {
        const int w2 = wid - first;
        strip = d.s_lo + w2 % d.ns;
        const int k = w2 / d.ns;
        seg = (k < d.g_lo) ? k : k + d.ng;
        h = rows;
    }
}

// Renumber blocks so that each XCD (blocks are dealt round-robin to the 8
// XCDs) gets a contiguous run of work items: neighbouring strips and
// segments, whose halos overlap, then share one L2.
__device__ __forceinline__ int xcd_block()
{
    const int nblk = gridDim.x;
    const int xcd = blockIdx.x % 8, kb = blockIdx.x / 8;
    const int q8 = nblk / 8, r8 = nblk % 8;
    return xcd * q8 + min(xcd, r8) + kb;
}

// General body: any work item, boundary rule applied everywhere.  `wid`
// is a wave-uniform boundary work id in [0, nwork).
// Odd reflection about the boundary lines, continued with period 2(n-1):
// node x of the extended line maps to the grid node idx it mirrors, and the
// result is the sign of the image: 1 inside, -1 on a mirror image, 0 on a
// boundary node.  The boundary rule (boundary nodes 0; the line one outside
// equal to minus the line one inside) is exactly this extension, and every
// operation of the update is sign-symmetric (opposite neighbours are paired
// by commutative additions; rounding to nearest is symmetric), so a level
// computed from an odd-reflected level is odd-reflected again, with exact
// zeros on the boundary lines.
__device__ __forceinline__ int reflect(int x, int n, int& idx)
{
    if (x >= 1 && x <= n - 2) {
        idx = x;
        return 1;
    }
    const int P = 2 * (n - 1);
    int m = x % P;
    if (m < 0) m += P;
    if (m == 0 || m == n - 1) {
        idx = m;
        return 0;
    }
    if (m < n - 1) {
        idx = m;
        return 1;
    }
    idx = P - m;
    return -1;
}

// Grid node that node x of the extended line stands for, and its sign: the
// odd reflection above, or on periodic grids plain wrapping (sign 1).
__device__ __forceinline__ int map_node(int x, int n, bool periodic, int& idx)
{
    if (!periodic) return reflect(x, n, idx);
    int m = x % n;
    if (m < 0) m += n;
    idx = m;
    return 1;
}

// One body for every work item.  Interior items (BND false) have a strip
// inside columns [1, nx-2] and a whole stream (rows y0 - H - NS ..
// y1 + H + 2 NS) inside rows [2, ny-3]: no boundary rule applies and every
// access is in bounds without checks.  Boundary items (BND true) run the
// same loop on the odd reflection of the grid: rows and columns beyond the
// boundary are loaded as the negated mirror rows and columns, boundary rows
// and columns as 0, and from then on the stencil itself keeps the boundary
// rule at every level (see reflect()).  On periodic grids they load the
// wrapped rows and columns instead (the host runs this path only for even
// nx, so a lane's column pair never straddles the wrap).  Interior items
// never reach the grid's edges and serve both rules.  Loads and stores are one vector per
// field through buffer resources with a scalar row offset.  `wid` is a
// wave-uniform work id of the item's class.
template <class Prec, int K, int DEPTH, int CW, bool BND>
__device__ __forceinline__ void stream_body(const SArgs<typename Prec::T>& a, const Decomp& dc, int wid,
                                            const typename Prec::W& w)
{
    using T = typename Prec::T;
    constexpr int R = KT<K>::R;
    constexpr int NS = 2 * R + 1;  // rows in a level's window
    constexpr int NW = Prec::NW;
    constexpr int H = R * DEPTH;   // rows / columns a pass reaches beyond its outputs
    constexpr int HP = halo_cols<R, DEPTH>();
    constexpr int SW = kWave * CW - 2 * HP;
    // Rows hold only the lane's own columns; neighbours beyond them are
    // fetched from the adjacent lanes where they are used.
    constexpr int E = CW;
    static_assert(CW == 2, "reflected loads assume column pairs");

    const int lane = threadIdx.x & (kWave - 1);
    int strip, seg, rows = a.rows;
    if constexpr (BND) {
        boundary_item(dc, a.rows, wid, strip, seg, rows);
    } else {
        strip = dc.s_lo + wid % dc.ns;
        seg = dc.g_lo + wid / dc.ns;
    }
    const int nx = a.g.nx, ny = a.g.ny, ld = a.g.ld;
    const int x0 = strip * SW - HP;
    const int xl = x0 + lane * CW;
    const int y0 = seg * rows;
    const int y1 = min(y0 + rows, ny);
    const bool st_lane = (xl >= x0 + HP) && (xl < x0 + HP + SW) && (!BND || xl < nx);
    // The last lane of an odd-width grid stores its first column only.
    const bool st_full = !BND || (xl + CW <= nx);

    // Columns of this lane on the reflected grid.  Adjacent columns mirror
    // adjacent grid columns, so one vector load at lc covers both (swapped
    // when the image runs backwards).  Only strips that reach column 0 or
    // nx-1 have lanes that are not plain.
    const bool per = a.g.periodic != 0;
    const bool edge = BND && !per && (x0 <= 0 || x0 + kWave * CW - 1 >= nx - 1);
    int lc = xl;
    bool swp = false, z0 = false, z1 = false, n0 = false, n1 = false;
    if constexpr (BND) {
        int i0, i1;
        const int s0 = map_node(xl, nx, per, i0), s1 = map_node(xl + 1, nx, per, i1);
        swp = i0 > i1;
        lc = swp ? i1 : i0;
        z0 = (s0 == 0);
        z1 = (s1 == 0);
        n0 = (s0 < 0);
        n1 = (s1 < 0);
    }
    // Loaded values of one row (two columns) as the reflected grid holds
    // them; sy is the row's sign.  Applied where the row is first used, not
    // right after its load, so the load keeps its latency hidden.
    auto reflect_vals = [&](T& v0, T& v1, int sy) {
        if (sy == 0) {
            v0 = v1 = T(0);
            return;
        }
        if (edge) {
            const T e0 = swp ? v1 : v0, e1 = swp ? v0 : v1;
            v0 = z0 ? T(0) : (n0 ? -e0 : e0);
            v1 = z1 ? T(0) : (n1 ? -e1 : e1);
        }
        if (sy < 0) {
            v0 = -v0;
            v1 = -v1;
        }
    };

    // Rows are fetched PF rows ahead of the phase that first uses them: with
    // DEPTH > 1 a row's loads land in a staging ring (indexed like the
    // window, by row mod NS) and are moved into the window one phase before
    // use, so each load has about two phases of work to hide behind.
    constexpr int PF = (DEPTH > 1) ? 3 : 1;
    const int jA = floor_div(y0 - H, NS) * NS;
    const int jhi = y1 - 1 + H;
    // Rows this wave touches: loads from jA - R up to PF rows past the last
    // iteration (< jhi + NS + PF), stores in [y0, y1).  Boundary items read
    // the mirror images of rows outside the grid.  The host bounds the byte
    // size.
    int base_row = jA - NS, top_row = jhi + 2 * NS + 1;
    if constexpr (BND) {
        const int ra = jA - R, rb = jhi + NS + PF - 1;
        const int P = 2 * (ny - 1);
        if (per) {
            // Wrapped rows may come from either end of the grid (the host
            // runs this only where the whole grid fits a buffer range).
            base_row = 0;
            top_row = ny;
        } else if (ra >= 0 && rb <= ny - 1) {
            base_row = ra;
            top_row = rb + 1;
        } else if (rb - ra + 1 < P && ra < 0 && rb <= ny - 1 && -ra <= ny - 1) {
            base_row = 0;
            top_row = max(rb, -ra) + 1;
        } else if (rb - ra + 1 < P && ra >= 0 && rb > ny - 1 && P - rb >= 0) {
            base_row = min(ra, P - rb);
            top_row = ny;
        } else {
            base_row = 0;
            top_row = ny;
        }
    }
    const uint32_t rbytes = (uint32_t)(top_row - base_row) * (uint32_t)ld * (uint32_t)sizeof(T);
    __amdgpu_buffer_rsrc_t rs_in[2], rs_out[2];
    rs_in[0] = make_rsrc(a.in_w0 + (size_t)base_row * ld, rbytes);
    rs_in[1] = make_rsrc((NW > 1 ? a.in_w1 : a.in_w0) + (size_t)base_row * ld, rbytes);
    rs_out[0] = make_rsrc(a.out_w0 + (size_t)base_row * ld, rbytes);
    rs_out[1] = make_rsrc((NW > 1 ? a.out_w1 : a.out_w0) + (size_t)base_row * ld, rbytes);
    const __amdgpu_buffer_rsrc_t rs_pin = make_rsrc(a.in_p + (size_t)base_row * ld, rbytes);
    const __amdgpu_buffer_rsrc_t rs_pout = make_rsrc((a.out_p ? a.out_p : a.out_w0) + (size_t)base_row * ld, rbytes);
    const uint32_t voff = (uint32_t)(lc * (int)sizeof(T));
    const uint32_t voff_st = (uint32_t)(xl * (int)sizeof(T));
    const int row_bytes = ld * (int)sizeof(T);

    T win[DEPTH][NS][NW][E];
    T pf[DEPTH][NS][CW];
#pragma unroll
    for (int t = 0; t < DEPTH; ++t)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
#pragma unroll
            for (int f = 0; f < NW; ++f)
#pragma unroll
                for (int e = 0; e < E; ++e) win[t][s][f][e] = T(0);
#pragma unroll
            for (int m = 0; m < CW; ++m) pf[t][s][m] = T(0);
        }

    // Point-field row read with window row jj.  With DEPTH 1 it is read only
    // on this segment's rows and output columns (it may be the array being
    // written in place).
    auto point_row = [&](int jj) {
        int jp = jj - R;
        if constexpr (DEPTH == 1) jp = min(max(jp, y0), y1 - 1);
        return jp;
    };
    T stg[PF > 1 ? NS : 1][NW][CW];
    T stp[PF > 1 ? NS : 1][CW];
    // Level-0 row jj (window fields) and the point field at point_row(jj).
    auto issue_loads = [&](int jj, auto& v, auto& p) {
        int jr = jj;
        if constexpr (BND) (void)map_node(jj, ny, per, jr);
        const uint32_t so = (uint32_t)((jr - base_row) * row_bytes);
#pragma unroll
        for (int f = 0; f < NW; ++f) {
            const Vec<T, CW> x = buf_load<T, CW>(rs_in[f], voff, so);
#pragma unroll
            for (int m = 0; m < CW; ++m) v[f][m] = x.v[m];
        }
        int jp = point_row(jj);
        if constexpr (DEPTH == 1) {
            if (!st_lane) return;
        }
        if constexpr (BND) (void)map_node(jp, ny, per, jp);
        const Vec<T, CW> x = buf_load<T, CW>(rs_pin, voff, (uint32_t)((jp - base_row) * row_bytes));
#pragma unroll
        for (int m = 0; m < CW; ++m) p[m] = x.v[m];
    };

    // Differences carried down the rows of each level.  They are refreshed
    // at every row of every level, also where a level's update is skipped
    // during the warm-up, so the first updated row of a level finds the
    // previous row's values.
    // Single precision: Carry structs.  Double precision: plain arrays (the
    // compiler keeps a struct of double arrays in scratch memory).
    Carry<float, CW> carry[NW > 1 ? DEPTH : 1];
    T cdv[DEPTH][CW], cq[DEPTH][CW], ceq[DEPTH][CW];
#pragma unroll
    for (int t = 0; t < DEPTH; ++t) {
        if constexpr (NW > 1) carry_zero(carry[t]);
#pragma unroll
        for (int m = 0; m < CW; ++m) cdv[t][m] = cq[t][m] = ceq[t][m] = T(0);
    }

    auto phase = [&](int ph, int j, bool warm) {
        // Finish level-0 row j and its point-field row (loaded one row ago).
        if constexpr (BND) {
            if (!per) {
                int jr;
                const int sy = reflect(j, ny, jr);
#pragma unroll
                for (int f = 0; f < NW; ++f) reflect_vals(win[0][ph][f][0], win[0][ph][f][1], sy);
                const int sp = reflect(point_row(j), ny, jr);
                T(&p)[CW] = pf[0][mod_c(ph - R, NS)];
                reflect_vals(p[0], p[1], sp);
            }
        }
        // Levels 1..DEPTH at rows j - t*R; the next row enters the window
        // right after level 1, whose inputs it overwrites.
#pragma unroll
        for (int t = 1; t <= DEPTH; ++t) {
            if (t == 2) {
                if constexpr (PF > 1) {
                    T(&dv)[NW][E] = win[0][mod_c(ph + 1, NS)];
                    T(&dp)[CW] = pf[0][mod_c(ph + 1 - R, NS)];
#pragma unroll
                    for (int f = 0; f < NW; ++f)
#pragma unroll
                        for (int m = 0; m < CW; ++m) dv[f][m] = stg[mod_c(ph + 1, NS)][f][m];
#pragma unroll
                    for (int m = 0; m < CW; ++m) dp[m] = stp[mod_c(ph + 1, NS)][m];
                    issue_loads(j + PF, stg[mod_c(ph + PF, NS)], stp[mod_c(ph + PF, NS)]);
                } else {
                    issue_loads(j + 1, win[0][mod_c(ph + 1, NS)], pf[0][mod_c(ph + 1 - R, NS)]);
                }
            }
            const int y = j - t * R;
            // Warm-up rows below a level's first needed row are skipped in
            // single precision.  Double precision computes them (they lie
            // outside the outputs' dependency cone): the branch lets the
            // compiler merge stores to different private arrays, which then
            // stay in scratch memory.
            const bool skip = (NW > 1) && warm && y < y0 - (DEPTH - t) * R;
            const int sy = mod_c(ph - t * R, NS);
            T nv[NW][E];
            T np[CW];
            if constexpr (NW > 1)
                row_update_carry<K, CW>(win[t - 1][sy], win[t - 1][mod_c(ph - t * R + 1, NS)],
                                        win[t - 1][mod_c(ph - t * R - 1, NS)], win[t - 1][mod_c(ph - t * R + 2, NS)],
                                        win[t - 1][mod_c(ph - t * R - 2, NS)], pf[t - 1][sy], carry[t - 1], w, !skip,
                                        nv, np);
            else
                row_update_carry<K, CW>(win[t - 1][sy], win[t - 1][mod_c(ph - t * R + 1, NS)],
                                        win[t - 1][mod_c(ph - t * R - 1, NS)], win[t - 1][mod_c(ph - t * R + 2, NS)],
                                        win[t - 1][mod_c(ph - t * R - 2, NS)], pf[t - 1][sy], cdv[t - 1], cq[t - 1],
                                        ceq[t - 1], w, !skip, nv, np);
            if (skip) continue;
            if (t < DEPTH) {
                T(&dst)[NW][E] = win[t][sy];
#pragma unroll
                for (int f = 0; f < NW; ++f)
#pragma unroll
                    for (int e = 0; e < E; ++e) dst[f][e] = nv[f][e];
#pragma unroll
                for (int m = 0; m < CW; ++m) pf[t][sy][m] = np[m];
            } else if (y >= y0 && y < y1 && st_lane) {
                const uint32_t so = (uint32_t)((y - base_row) * row_bytes);
                if (st_full) {
#pragma unroll
                    for (int f = 0; f < NW; ++f) {
                        Vec<T, CW> x;
#pragma unroll
                        for (int m = 0; m < CW; ++m) x.v[m] = nv[f][m];
                        buf_store<T, CW>(x, rs_out[f], voff_st, so);
                    }
                    if (a.out_p) {
                        Vec<T, CW> x;
#pragma unroll
                        for (int m = 0; m < CW; ++m) x.v[m] = np[m];
                        buf_store<T, CW>(x, rs_pout, voff_st, so);
                    }
                } else {
                    // Last lane of the grid: its first column only (xl = nx - 1).
#pragma unroll
                    for (int f = 0; f < NW; ++f) buf_store1<T>(nv[f][0], rs_out[f], voff_st, so);
                    if (a.out_p) buf_store1<T>(np[0], rs_pout, voff_st, so);
                }
            }
        }
        if constexpr (DEPTH == 1) issue_loads(j + 1, win[0][mod_c(ph + 1, NS)], pf[0][mod_c(ph + 1 - R, NS)]);
    };

    issue_loads(jA, win[0][0], pf[0][mod_c(-R, NS)]);
    if constexpr (PF > 1) {
#pragma unroll
        for (int k = 1; k < PF; ++k) issue_loads(jA + k, stg[mod_c(k, NS)], stp[mod_c(k, NS)]);
    }
    int jb = jA;
    // Warm-up: levels whose rows are not yet needed are skipped.
    for (; jb <= jhi && jb < y0 + H; jb += NS) {
#pragma unroll
        for (int ph = 0; ph < NS; ++ph) phase(ph, jb + ph, true);
    }
    for (; jb <= jhi; jb += NS) {
#pragma unroll
        for (int ph = 0; ph < NS; ++ph) phase(ph, jb + ph, false);
    }
}

// Wave-uniform global wave id (kept in scalar registers, so the work item
// and the buffer resources derived from it are scalar too).
__device__ __forceinline__ int wave_id()
{
    return __builtin_amdgcn_readfirstlane(xcd_block() * kWavesPerBlock + (int)(threadIdx.x >> 6));
}

template <class Prec, int K, int DEPTH, int CW>
__global__ __launch_bounds__(kWave* kWavesPerBlock, 2) void k_stream_general(SArgs<typename Prec::T> a, Decomp dc,
                                                                              int nwork, typename Prec::W w)
{
    const int wid = wave_id();
    if (wid >= nwork) return;  // whole wavefronts only
    stream_body<Prec, K, DEPTH, CW, true>(a, dc, wid, w);
}

template <class Prec, int K, int DEPTH, int CW>
__global__ __launch_bounds__(kWave* kWavesPerBlock, 2) void k_stream_interior(SArgs<typename Prec::T> a, Decomp dc,
                                                                               typename Prec::W w)
{
    const int wid = wave_id();
    if (wid >= dc.ns * dc.ng) return;
    stream_body<Prec, K, DEPTH, CW, false>(a, dc, wid, w);
}

// Both kinds of work items in one launch: boundary items take the first
// wave ids, so the slower reflected passes start first and the interior
// items fill the device around them; no second stream or event is needed.
template <class Prec, int K, int DEPTH, int CW>
__global__ __launch_bounds__(kWave* kWavesPerBlock, 2) void k_stream_fused(SArgs<typename Prec::T> a, Decomp dc,
                                                                            int nb, typename Prec::W w)
{
    const int wid = wave_id();
    if (wid < nb) stream_body<Prec, K, DEPTH, CW, true>(a, dc, wid, w);
    else if (wid - nb < dc.ns * dc.ng) stream_body<Prec, K, DEPTH, CW, false>(a, dc, wid - nb, w);
}

// Batched kernels: one launch advances many instances (different grids,
// weights and buffers) by one pass.  The work items of all instances form
// one index space; prefix[k] is the first global work id of item k and
// prefix[count] the total.  Each wave finds its item by binary search and
// runs the same body as the single-instance kernels.
template <class Prec>
struct BatchItem {
    SArgs<typename Prec::T> a;
    Decomp dc;
    typename Prec::W w;
};

template <class Prec, int K, int DEPTH, int CW, bool INTERIOR>
__global__ __launch_bounds__(kWave* kWavesPerBlock, 2) void k_stream_batch(const BatchItem<Prec>* __restrict__ items,
                                                                            const int* __restrict__ prefix, int count)
{
    const int gw = wave_id();
    if (gw >= prefix[count]) return;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= gw) lo = mid;
        else hi = mid - 1;
    }
    // A copy in registers: read through the table, the fields would be
    // re-read from memory after every store of the pass (the compiler cannot
    // tell the stores from the table).
    const BatchItem<Prec> it = items[lo];
    const int wid = gw - prefix[lo];
    stream_body<Prec, K, DEPTH, CW, !INTERIOR>(it.a, it.dc, wid, it.w);
}

// ---- persistent batched passes ----------------------------------------------
//
// One launch per stencil class advances many compensated-FP32 instances by
// all their full passes.  The host pins every instance to one accelerator
// complex die (XCC, an L2 domain) and lists, per XCC, the instances' passes
// in pass-major order as tasks of one work item per wave.  A wave reads the
// id of the XCC it runs on, takes the next item of that XCC's queue (an
// atomic counter) and, before running it, waits until the tiles whose
// output it reads have finished the previous pass: the item's own tile
// (strip x segment) and its neighbours, `ks` strips to each side and `kr`
// segments up and down (the host finds the reach from the rows and
// columns each item loads, reflected or wrapped by the boundary rule; on
// a periodic grid a short last strip or segment can put the wrapped halo
// two tiles away).  Each tile keeps a counter
// of its finished passes.  The same wait orders the writes of the next pass
// after the reads of the previous one: a tile's pass p+1 overwrites the
// state that the neighbours' pass p read.  Items are taken in queue order,
// so every item a wave waits for was taken earlier by a running wave, and
// the earliest unfinished item never waits: the queue always drains.
//
// Every item of an instance runs on the one XCC its queue belongs to, so
// all of an instance's traffic inside the launch goes through one L2, the
// coherence point of that XCC's CUs; only the CUs' L1 caches (write-through)
// can hold stale lines.  A finished item therefore waits until its stores
// have reached L2 (s_waitcnt on all counters) before it counts itself done,
// and an item that depends on the previous pass invalidates its CU's L1
// (buffer_inv sc1, the device-scope acquire fence) after its wait.  No L2
// write-back is needed inside the launch (kernel boundaries write L2 back
// and invalidate it, which covers the launches before and after).  Two
// alternatives were measured on one MI355X over the 512-instance batch,
// bitwise against the batch run as rounds of ordinary launches: the
// device-scope release fence (buffer_wbl2 sc1, a write-back of the XCC's
// dirty L2 lines per item) was exact but 1.46x slower in total; a
// workgroup-scope invalidation (buffer_inv sc0) instead of sc1 leaves the
// L1 stale and got about 20 instances wrong per run, as did dropping the
// invalidation.
// Two passes apart an instance writes the state it read one pass earlier;
// the neighbour wait orders that too (see above).
//
// Every wave-level decision is made by all 64 lanes on identical values
// (atomics are issued by every lane with the increment carried by the first
// active lane, loads of a counter by every lane), so no lane ever takes a
// different path: a value read from one lane only (for example under
// `lane == 0`) would let the compiler run the other lanes on into the next
// iteration without it, where that value no longer exists.
struct PInst {
    SArgs<float> a[2];  // pass parity 0: state 0 -> state 1; parity 1: back
    Decomp dc;
    StepW32 w;
    int kind, nb, items;
    int tile_off;  // first tile counter of the instance (after kPersistTileBase)
    int ks, kr;    // neighbour strips / segments to wait for on each side
};

// Strip and segment of work item `wid` of a pass (boundary items first).
__device__ __forceinline__ void item_tile(const Decomp& dc, int nb, int wid, int& strip, int& seg)
{
    if (wid < nb) {
        int h;
        boundary_item(dc, dc.rows_e, wid, strip, seg, h);  // one segmentation
    } else {
        const int k = wid - nb;
        strip = dc.s_lo + k % dc.ns;
        seg = dc.g_lo + k / dc.ns;
    }
}

// The XCC the calling wave runs on (hardware register XCC_ID, low 4 bits).
__device__ __forceinline__ int xcc_id()
{
    return __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((16 - 1) << 11)) & 0xf;
}

// One increment per wave: every lane executes the atomic, the first active
// lane adds 1, the others 0; returns the counter's value before the
// increment (wave-uniform).
__device__ __forceinline__ int wave_fetch_inc(int* p)
{
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int first = __builtin_amdgcn_readfirstlane(lane);
    const int old = __hip_atomic_fetch_add(p, lane == first ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_amdgcn_readfirstlane(old);
}

__device__ __forceinline__ int wave_load(const int* p)
{
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

template <int K, int DEPTH>
__global__ __launch_bounds__(kWave* kWavesPerBlock, 2) void k_stream_persist(const PInst* __restrict__ insts,
                                                                              const PersistTask* __restrict__ tasks,
                                                                              const int* __restrict__ qt_off,
                                                                              const int* __restrict__ qn, int* ctr,
                                                                              int nq, long long wait_ticks)
{
    const int q = __builtin_amdgcn_readfirstlane(xcc_id() % nq);
    const int t0 = qt_off[q], t1 = qt_off[q + 1];
    const int total = qn[q];
    int* head = ctr + kPersistStride * q;
    int* stalls = ctr + kPersistStride * kPersistQueues;
    for (;;) {
        const int k = wave_fetch_inc(head);
        if (k >= total) break;
        int lo = t0, hi = t1 - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tasks[mid].first <= k) lo = mid;
            else hi = mid - 1;
        }
        const PersistTask t = tasks[lo];
        const PInst& pi = insts[t.inst];
        const Decomp dc = pi.dc;
        const int wid = k - t.first;
        // A work id outside the task (tables out of step with the queue)
        // is skipped and reported instead of being run.
        bool ok = k >= t.first && wid < pi.items;
        int strip = 0, seg = 0;
        if (ok) item_tile(dc, pi.nb, wid, strip, seg);
        int* tiles = ctr + kPersistTileBase + pi.tile_off;
        if (t.pass > 0) {
            // Neighbour n = (strip + n % (2 ks + 1) - ks, seg + n / (2 ks + 1)
            // - kr), 64 at a time, one per lane; lanes past the last
            // neighbour, and neighbours off a Dirichlet grid, watch the
            // item's own tile.
            const int lane = (int)(threadIdx.x & (kWave - 1));
            const int ks = pi.ks, kr = pi.kr, nst = dc.nstrips, nsg = dc.nseg;
            const int wsx = 2 * ks + 1, nn = wsx * (2 * kr + 1);
            const bool per = pi.a[0].g.periodic != 0;
            auto ready = [&]() {
                bool all = true;
                for (int n0 = 0; n0 < nn; n0 += kWave) {
                    const int n = n0 + lane;
                    int sn = strip + n % wsx - ks, gn = seg + n / wsx - kr;
                    bool use = n < nn;
                    if (per) {
                        sn = ((sn % nst) + nst) % nst;
                        gn = ((gn % nsg) + nsg) % nsg;
                    } else {
                        use = use && sn >= 0 && sn < nst && gn >= 0 && gn < nsg;
                    }
                    const int* watch = tiles + (use ? gn * nst + sn : seg * nst + strip);
                    all = __all(__hip_atomic_load(watch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= t.pass) && all;
                }
                return all;
            };
            if (!ready()) {
                // Poll with a growing pause (up to 64 x 512 cycles); give up
                // after wait_ticks of the 100 MHz real-time clock, or at once
                // when another wait of this launch has given up.
                const long long t_start = (long long)__builtin_amdgcn_s_memrealtime();
                int pause = 1;
                for (int polls = 1;; ++polls) {
                    for (int z = 0; z < pause; ++z) __builtin_amdgcn_s_sleep(8);
                    pause = min(2 * pause, 64);
                    if (ready()) break;
                    if ((polls & 7) == 0 && wave_load(stalls) > 0) {
                        ok = false;
                        break;
                    }
                    if ((long long)__builtin_amdgcn_s_memrealtime() - t_start > wait_ticks) {
                        ok = false;
                        break;
                    }
                }
            }
            // Whether or not it had to wait: this CU's L1 may still hold
            // lines of the state the previous pass rewrote.
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if (ok) {
            const SArgs<float> a = pi.a[t.par];
            const StepW32 w = pi.w;
            const int nb = pi.nb;
            if (wid < nb) stream_body<PF32C, K, DEPTH, 2, true>(a, dc, wid, w);
            else stream_body<PF32C, K, DEPTH, 2, false>(a, dc, wid - nb, w);
        } else {
            (void)wave_fetch_inc(stalls);
        }
        // The item's loads are done and its stores are in this XCC's L2
        // before its tile is counted (the memory clobber keeps the compiler
        // from moving memory operations across the wait).  A skipped item
        // counts too, so that the items waiting for it end.
        asm volatile("s_waitcnt vmcnt(0) expcnt(0) lgkmcnt(0)" ::: "memory");
        (void)wave_fetch_inc(tiles + seg * dc.nstrips + strip);
    }
}

// One write of the XCC id per workgroup (the host counts the XCCs that
// workgroups land on before it plans per-XCC queues).
__global__ void k_xcc_probe(int* out, int n)
{
    if (threadIdx.x == 0 && (int)blockIdx.x < n) out[blockIdx.x] = xcc_id();
}

template <int R, int DEPTH, int CW>
Decomp make_decomp(const Grid& g, int rows, int rows_e = 0)
{
    constexpr int NS = 2 * R + 1;
    constexpr int H = R * DEPTH;
    constexpr int HP = halo_cols<R, DEPTH>();
    constexpr int SW = kWave * CW - 2 * HP;
    Decomp d;
    d.nstrips = (g.nx + SW - 1) / SW;
    d.nseg = (g.ny + rows - 1) / rows;
    d.s_lo = d.nstrips;
    int s_hi = -1;
    for (int s = 0; s < d.nstrips; ++s) {
        const int x0 = s * SW - HP;
        if (x0 >= 1 && x0 + kWave * CW - 1 <= g.nx - 2) {
            d.s_lo = min(d.s_lo, s);
            s_hi = max(s_hi, s);
        }
    }
    d.ns = (s_hi >= d.s_lo) ? s_hi - d.s_lo + 1 : 0;
    d.g_lo = d.nseg;
    int g_hi = -1;
    for (int k = 0; k < d.nseg; ++k) {
        const int y0 = k * rows, y1 = min(y0 + rows, g.ny);
        if (y0 - H - NS >= 2 && y1 + H + 2 * NS <= g.ny - 3) {
            d.g_lo = min(d.g_lo, k);
            g_hi = max(g_hi, k);
        }
    }
    d.ng = (g_hi >= d.g_lo) ? g_hi - d.g_lo + 1 : 0;
    if (d.ns == 0 || d.ng == 0) {
        d.ns = d.ng = 0;
        d.s_lo = d.g_lo = 0;
        rows_e = 0;  // every item is a boundary item of one segmentation
    }
    d.rows_e = (rows_e > 0) ? rows_e : rows;
    d.nseg_e = (g.ny + d.rows_e - 1) / d.rows_e;
    return d;
}

// Rows per segment for a grid: a wave's buffer resources span at most
// rows + 2H + 4NS rows of ld elements, which must stay below 2^31 bytes
// (row strides are bounded by the grid validation, so the cap is >= 8).
template <int R, int DEPTH>
int fit_rows(const Grid& g, int rows, size_t elt)
{
    constexpr int NS = 2 * R + 1, H = R * DEPTH;
    const long long cap = ((1LL << 31) - 1) / ((long long)g.ld * (long long)elt) - (2 * H + 4 * NS);
    return (int)std::max<long long>(1, std::min<long long>(rows, cap));
}

// Segment heights of a single-grid pass with `rows` the tuned height: the
// edge strips' items reflect columns on every row and take longer per row
// (edge_cost: measured best ratios on MI355X, 1.16 for the 5- and 9-point
// kernels, 1.36 for the 13-point ones), so their segments are cut shorter,
// such that rows_e + c0 = (rows + c0) / edge_cost with c0 = 2H + NS the
// rows an item streams beyond its outputs; the interior strips' segments then grow
// until the pass has no more work items than with `rows` throughout, so
// that the tuned filling of the device's wave slots holds.  Where no
// height up to twice `rows` achieves that, or the grid has no interior
// strips, both stay `rows`.  Heights beyond what fit_rows allows are
// never taken.
template <int R>
constexpr double edge_cost() { return R == 1 ? 1.16 : 1.36; }

template <int R, int DEPTH>
void edge_rows(const Grid& g, size_t elt, int& rows, int& rows_e)
{
    constexpr int c0 = 2 * R * DEPTH + 2 * R + 1;
    const Decomp d0 = make_decomp<R, DEPTH, 2>(g, rows);
    rows_e = rows;
    const int ne = d0.nstrips - d0.ns;
    if (d0.ns == 0 || ne == 0) return;
    const int re = (int)((rows + c0) / edge_cost<R>()) - c0;
    if (re < kPersistMinRows || re >= rows) return;
    const long long budget = (long long)d0.nstrips * d0.nseg;
    const long long edge_items = (long long)ne * ((g.ny + re - 1) / re);
    for (int ri = rows; ri <= 2 * rows; ++ri) {
        if (fit_rows<R, DEPTH>(g, ri, elt) != ri) return;
        if (edge_items + (long long)d0.ns * ((g.ny + ri - 1) / ri) <= budget) {
            const Decomp d1 = make_decomp<R, DEPTH, 2>(g, ri, re);
            if (d1.ns != d0.ns) return;
            rows = ri;
            rows_e = re;
            return;
        }
    }
}

template <class Prec, int K, int DEPTH>
hipError_t launch_depth(const Grid& g, const typename Prec::W& w, int rows, const Fork* fork,
                        SArgs<typename Prec::T> a, hipStream_t s)
{
    constexpr int CW = 2;
    constexpr int R = KT<K>::R;
    constexpr int SW = kWave * CW - 2 * halo_cols<R, DEPTH>();
    static_assert(SW > 0, "strip too narrow");
    rows = fit_rows<R, DEPTH>(g, rows, sizeof(typename Prec::T));
    int rows_e = rows;
    edge_rows<R, DEPTH>(g, sizeof(typename Prec::T), rows, rows_e);
    a.g = g;
    a.rows = rows;
    const Decomp dc = make_decomp<R, DEPTH, CW>(g, rows, rows_e);
    a.nstrips = dc.nstrips;
    const int ni = dc.ns * dc.ng;
    const int nb = (dc.nstrips - dc.ns) * dc.nseg_e + dc.ns * (dc.nseg - dc.ng);
    a.nwork = nb + ni;
    // One launch per pass (measured on 4097^2 9-point compensated: 786 ->
    // 826 GLUP/s against a boundary kernel on a side stream beside the
    // interior kernel; 2049^2: 442 -> 579).
    (void)fork;
    const int blocks = (a.nwork + kWavesPerBlock - 1) / kWavesPerBlock;
    if (nb > 0 && ni > 0)
        k_stream_fused<Prec, K, DEPTH, CW><<<blocks, kWave * kWavesPerBlock, 0, s>>>(a, dc, nb, w);
    else if (nb > 0)
        k_stream_general<Prec, K, DEPTH, CW><<<blocks, kWave * kWavesPerBlock, 0, s>>>(a, dc, nb, w);
    else
        k_stream_interior<Prec, K, DEPTH, CW><<<blocks, kWave * kWavesPerBlock, 0, s>>>(a, dc, w);
    return hipGetLastError();
}

template <class Prec, int K>
hipError_t launch_kind(const Grid& g, const typename Prec::W& w, const StreamShape& sh, SArgs<typename Prec::T> a,
                       hipStream_t s)
{
    switch (sh.depth) {
    case 1: return launch_depth<Prec, K, 1>(g, w, sh.rows, sh.fork, a, s);
    case 2: return launch_depth<Prec, K, 2>(g, w, sh.rows, sh.fork, a, s);
    case 3: return launch_depth<Prec, K, 3>(g, w, sh.rows, sh.fork, a, s);
    case 4: return launch_depth<Prec, K, 4>(g, w, sh.rows, sh.fork, a, s);
    case 6: return launch_depth<Prec, K, 6>(g, w, sh.rows, sh.fork, a, s);
    case 8: return launch_depth<Prec, K, 8>(g, w, sh.rows, sh.fork, a, s);
    default: return hipErrorInvalidValue;
    }
}

template <class Prec>
hipError_t launch(int kind, const Grid& g, const typename Prec::W& w, const StreamShape& sh,
                  SArgs<typename Prec::T> a, hipStream_t s)
{
    if (sh.rows < 1) return hipErrorInvalidValue;
    switch (kind) {
    case KIND5: return launch_kind<Prec, KIND5>(g, w, sh, a, s);
    case KIND9: return launch_kind<Prec, KIND9>(g, w, sh, a, s);
    case KIND13: return launch_kind<Prec, KIND13>(g, w, sh, a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool stream_depth_supported(int depth)
{
    return depth == 1 || depth == 2 || depth == 3 || depth == 4 || depth == 6 || depth == 8;
}

namespace {

// Resident waves of a kernel on the current device (all CUs), and whether
// its state does not fit the registers (more than 128 bytes of scratch per
// lane: such depths spill hundreds of bytes, while a few spilled scalars,
// tens of bytes, cost nothing measurable); cached per (kernel, device).
std::pair<int, bool> kernel_fit(const void* fn)
{
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, std::pair<int, bool>> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({fn, dev});
    if (it != cache.end()) return it->second;
    hipFuncAttributes at{};
    bool spills = false;
    if (hipFuncGetAttributes(&at, fn) == hipSuccess) spills = at.localSizeBytes > 128;
    int nb = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kWave * kWavesPerBlock, 0) != hipSuccess || nb < 1)
        nb = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    (void)hipGetLastError();
    const std::pair<int, bool> r{nb * kWavesPerBlock * cus, spills};
    cache[{fn, dev}] = r;
    return r;
}

template <class Prec, int K, int DEPTH>
ShapeFit fit_depth()
{
    // The kernel a pass over a grid with both kinds of items launches.
    const auto f = kernel_fit(reinterpret_cast<const void*>(&k_stream_fused<Prec, K, DEPTH, 2>));
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    (void)hipGetLastError();
    return ShapeFit{kWave * 2 - 2 * halo_cols<KT<K>::R, DEPTH>(), f.first, f.second, f.first / (4 * cus),
                    KT<K>::R * DEPTH};
}

template <class Prec, int K>
ShapeFit fit_kind(int depth)
{
    switch (depth) {
    case 1: return fit_depth<Prec, K, 1>();
    case 2: return fit_depth<Prec, K, 2>();
    case 3: return fit_depth<Prec, K, 3>();
    case 4: return fit_depth<Prec, K, 4>();
    case 6: return fit_depth<Prec, K, 6>();
    default: return fit_depth<Prec, K, 8>();
    }
}

template <class Prec>
ShapeFit fit_prec(int kind, int depth)
{
    switch (kind) {
    case KIND5: return fit_kind<Prec, KIND5>(depth);
    case KIND9: return fit_kind<Prec, KIND9>(depth);
    default: return fit_kind<Prec, KIND13>(depth);
    }
}

}  // namespace

ShapeFit stream_shape_fit(int precision, int kind, int depth)
{
    if (!stream_depth_supported(depth)) return ShapeFit{0, 0, true, 0, 0};
    return precision == 0 ? fit_prec<PF64>(kind, depth) : fit_prec<PF32C>(kind, depth);
}

namespace {

// Segment rows for one batched launch.  A work item recomputes about
// R*(DEPTH-1) rows of its neighbours per level and streams 2R+1 rows of
// warm-up, so its cost grows like rows + R*(DEPTH-1) + 2R+1 while it
// produces `rows` rows; all items of a launch cost the same, so the launch
// takes ceil(items / slots) item times.  The candidate (not below the
// tuned floor) with the least modelled time wins: tall segments when many
// instances share the launch, the floor when they are few.
template <int R, int DEPTH>
int batch_rows(int rows_min, const std::vector<BatchInst>& insts, int slots_i)
{
    constexpr int HP = halo_cols<R, DEPTH>();
    constexpr int SW = kWave * 2 - 2 * HP;
    static const int cand[] = {12, 16, 24, 32, 48, 64, 80, 96, 128, 160, 192};
    const double slots = slots_i;
    auto cost = [&](int r) {
        double items = 0;
        for (const BatchInst& in : insts)
            items += (double)((in.g.nx + SW - 1) / SW) * (double)((in.g.ny + r - 1) / r);
        return std::ceil(items / slots) * (r + R * (DEPTH - 1) + 2 * R + 1);
    };
    int best = rows_min;
    double bc = cost(rows_min);
    for (int r : cand) {
        if (r <= rows_min) continue;
        const double c = cost(r);
        if (c < bc) {
            bc = c;
            best = r;
        }
    }
    return best;
}

template <class Prec, int K, int DEPTH>
void tables_depth(int rows, const std::vector<BatchInst>& insts, BatchTables& gen, BatchTables& inr)
{
    using T = typename Prec::T;
    constexpr int CW = 2;
    constexpr int R = KT<K>::R;
    const int slots = kernel_fit(reinterpret_cast<const void*>(&k_stream_batch<Prec, K, DEPTH, CW, true>)).first;
    rows = batch_rows<R, DEPTH>(rows, insts, slots);
    gen.rows = inr.rows = rows;
    gen.prefix.assign(1, 0);
    inr.prefix.assign(1, 0);
    gen.items.clear();
    inr.items.clear();
    gen.count = inr.count = 0;
    for (const BatchInst& in : insts) {
        BatchItem<Prec> it{};
        it.a.g = in.g;
        it.a.rows = fit_rows<R, DEPTH>(in.g, rows, sizeof(T));
        it.a.in_w0 = (const T*)in.in_w0;
        it.a.in_w1 = (const T*)in.in_w1;
        it.a.in_p = (const T*)in.in_p;
        it.a.out_w0 = (T*)in.out_w0;
        it.a.out_w1 = (T*)in.out_w1;
        it.a.out_p = (T*)in.out_p;
        it.dc = make_decomp<R, DEPTH, CW>(in.g, it.a.rows);
        it.a.nstrips = it.dc.nstrips;
        it.a.nwork = it.dc.nstrips * it.dc.nseg;
        if constexpr (Prec::NW == 1) it.w = in.w64;
        else it.w = in.w32;
        const int ni = it.dc.ns * it.dc.ng;
        const int nb = it.a.nwork - ni;
        const unsigned char* raw = reinterpret_cast<const unsigned char*>(&it);
        if (nb > 0) {
            gen.items.insert(gen.items.end(), raw, raw + sizeof(it));
            gen.prefix.push_back(gen.prefix.back() + nb);
            ++gen.count;
        }
        if (ni > 0) {
            inr.items.insert(inr.items.end(), raw, raw + sizeof(it));
            inr.prefix.push_back(inr.prefix.back() + ni);
            ++inr.count;
        }
    }
}

template <class Prec, int K>
void tables_kind(int depth, int rows, const std::vector<BatchInst>& insts, BatchTables& gen, BatchTables& inr)
{
    switch (depth) {
    case 1: tables_depth<Prec, K, 1>(rows, insts, gen, inr); break;
    case 2: tables_depth<Prec, K, 2>(rows, insts, gen, inr); break;
    case 3: tables_depth<Prec, K, 3>(rows, insts, gen, inr); break;
    case 4: tables_depth<Prec, K, 4>(rows, insts, gen, inr); break;
    case 6: tables_depth<Prec, K, 6>(rows, insts, gen, inr); break;
    case 8: tables_depth<Prec, K, 8>(rows, insts, gen, inr); break;
    default: break;
    }
}

template <class Prec>
void tables_prec(int kind, int depth, int rows, const std::vector<BatchInst>& insts, BatchTables& gen,
                 BatchTables& inr)
{
    switch (kind) {
    case KIND5: tables_kind<Prec, KIND5>(depth, rows, insts, gen, inr); break;
    case KIND9: tables_kind<Prec, KIND9>(depth, rows, insts, gen, inr); break;
    case KIND13: tables_kind<Prec, KIND13>(depth, rows, insts, gen, inr); break;
    default: break;
    }
}

template <class Prec, int K, int DEPTH>
hipError_t blaunch(bool interior, const void* items, const int* prefix, int count, int total, hipStream_t s)
{
    const int blocks = (total + kWavesPerBlock - 1) / kWavesPerBlock;
    const BatchItem<Prec>* it = (const BatchItem<Prec>*)items;
    if (interior) k_stream_batch<Prec, K, DEPTH, 2, true><<<blocks, kWave * kWavesPerBlock, 0, s>>>(it, prefix, count);
    else k_stream_batch<Prec, K, DEPTH, 2, false><<<blocks, kWave * kWavesPerBlock, 0, s>>>(it, prefix, count);
    return hipGetLastError();
}

template <class Prec, int K>
hipError_t blaunch_kind(int depth, bool interior, const void* items, const int* prefix, int count, int total,
                        hipStream_t s)
{
    switch (depth) {
    case 1: return blaunch<Prec, K, 1>(interior, items, prefix, count, total, s);
    case 2: return blaunch<Prec, K, 2>(interior, items, prefix, count, total, s);
    case 3: return blaunch<Prec, K, 3>(interior, items, prefix, count, total, s);
    case 4: return blaunch<Prec, K, 4>(interior, items, prefix, count, total, s);
    case 6: return blaunch<Prec, K, 6>(interior, items, prefix, count, total, s);
    case 8: return blaunch<Prec, K, 8>(interior, items, prefix, count, total, s);
    default: return hipErrorInvalidValue;
    }
}

template <class Prec>
hipError_t blaunch_prec(int kind, int depth, bool interior, const void* items, const int* prefix, int count,
                        int total, hipStream_t s)
{
    switch (kind) {
    case KIND5: return blaunch_kind<Prec, KIND5>(depth, interior, items, prefix, count, total, s);
    case KIND9: return blaunch_kind<Prec, KIND9>(depth, interior, items, prefix, count, total, s);
    case KIND13: return blaunch_kind<Prec, KIND13>(depth, interior, items, prefix, count, total, s);
    default: return hipErrorInvalidValue;
    }
}

// Pass depths of the persistent kernel (the single-grid defaults).
constexpr int kPD5 = 8, kPD9 = 8, kPD13 = 6;

template <int K, int DEPTH>
int persist_max_tiles_k(const Grid& g)
{
    constexpr int R = KT<K>::R;
    const Decomp dc = make_decomp<R, DEPTH, 2>(g, kPersistMinRows);
    return dc.nstrips * dc.nseg;
}

template <int K, int DEPTH>
int persist_inst_k(const Grid& g, const StepW32& w, int rows, int tile_off, float* const s0[3],
                   float* const s1[3], unsigned char* rec, int* nb, int* rows_used)
{
    constexpr int R = KT<K>::R;
    constexpr int NS = 2 * R + 1, H = R * DEPTH;
    PInst p{};
    rows = fit_rows<R, DEPTH>(g, rows, sizeof(float));
    const Decomp dc = make_decomp<R, DEPTH, 2>(g, rows);
    if (dc.nstrips * dc.nseg > persist_max_tiles_k<K, DEPTH>(g)) return -1;
    // Reach of an item's reads in tiles: the rows it loads (at most
    // y0 - H - NS .. y1 + H + NS + 1; a margin of NS more each way) and the
    // columns x0 .. x0 + 127 of its strip, each mapped into the grid by the
    // boundary rule, and the farthest strip and segment they fall in
    // (cyclic distance on periodic grids).
    constexpr int HP = halo_cols<R, DEPTH>();
    constexpr int SW = kWave * 2 - 2 * HP;
    const bool per = g.periodic != 0;
    auto into = [&](int x, int n) {
        if (per) return ((x % n) + n) % n;
        const int P = 2 * (n - 1);
        int m = ((x % P) + P) % P;
        return m > n - 1 ? P - m : m;
    };
    auto dist = [&](int a, int b, int n) {
        const int d = a > b ? a - b : b - a;
        return per ? std::min(d, n - d) : d;
    };
    int kr = 0, ks = 0;
    for (int s = 0; s < dc.nseg; ++s) {
        const int y0 = s * rows, y1 = std::min(y0 + rows, g.ny);
        for (int y = y0 - H - 2 * NS; y <= y1 - 1 + H + 2 * NS; ++y) kr = std::max(kr, dist(into(y, g.ny) / rows, s, dc.nseg));
    }
    for (int s = 0; s < dc.nstrips; ++s) {
        const int x0 = s * SW - HP;
        for (int x = x0; x < x0 + kWave * 2; ++x) ks = std::max(ks, dist(into(x, g.nx) / SW, s, dc.nstrips));
    }
    p.kr = kr;
    p.ks = ks;
    p.tile_off = tile_off;
    for (int par = 0; par < 2; ++par) {
        SArgs<float>& a = p.a[par];
        float* const* in = par ? s1 : s0;
        float* const* out = par ? s0 : s1;
        a.g = g;
        a.rows = rows;
        a.nstrips = dc.nstrips;
        a.nwork = dc.nstrips * dc.nseg;
        a.in_w0 = in[0];
        a.in_w1 = in[1];
        a.in_p = in[2];
        a.out_w0 = out[0];
        a.out_w1 = out[1];
        a.out_p = out[2];
    }
    p.dc = dc;
    p.w = w;
    p.kind = K;
    p.items = dc.nstrips * dc.nseg;
    p.nb = p.items - dc.ns * dc.ng;
    std::memcpy(rec, &p, sizeof p);
    *nb = p.nb;
    *rows_used = rows;
    return p.items;
}

template <int K, int DEPTH>
const void* persist_fn_k()
{
    return reinterpret_cast<const void*>(&k_stream_persist<K, DEPTH>);
}

const void* persist_fn(int kind)
{
    return kind == KIND5 ? persist_fn_k<KIND5, kPD5>() : kind == KIND9 ? persist_fn_k<KIND9, kPD9>()
                                                                       : persist_fn_k<KIND13, kPD13>();
}

}  // namespace

size_t persist_inst_size() { return sizeof(PInst); }

int persist_depth(int kind) { return kind == KIND5 ? kPD5 : kind == KIND9 ? kPD9 : kPD13; }

int persist_inst(const Grid& g, int kind, const StepW32& w, int rows, int tile_off, float* const s0[3],
                 float* const s1[3], unsigned char* rec, int* nb, int* rows_used)
{
    switch (kind) {
    case KIND5: return persist_inst_k<KIND5, kPD5>(g, w, rows, tile_off, s0, s1, rec, nb, rows_used);
    case KIND9: return persist_inst_k<KIND9, kPD9>(g, w, rows, tile_off, s0, s1, rec, nb, rows_used);
    default: return persist_inst_k<KIND13, kPD13>(g, w, rows, tile_off, s0, s1, rec, nb, rows_used);
    }
}

int persist_max_tiles(const Grid& g, int kind)
{
    switch (kind) {
    case KIND5: return persist_max_tiles_k<KIND5, kPD5>(g);
    case KIND9: return persist_max_tiles_k<KIND9, kPD9>(g);
    default: return persist_max_tiles_k<KIND13, kPD13>(g);
    }
}

int persist_blocks(int kind)
{
    const auto f = kernel_fit(persist_fn(kind));
    return std::max(1, f.first / kWavesPerBlock);
}

hipError_t persist_launch(int kind, const void* insts, const PersistTask* tasks, const int* qt_off, const int* qn,
                          int* ctr, long long wait_ticks, hipStream_t s)
{
    const dim3 grid(persist_blocks(kind)), block(kWave * kWavesPerBlock);
    const PInst* pi = (const PInst*)insts;
    switch (kind) {
    case KIND5: k_stream_persist<KIND5, kPD5><<<grid, block, 0, s>>>(pi, tasks, qt_off, qn, ctr, kPersistQueues, wait_ticks); break;
    case KIND9: k_stream_persist<KIND9, kPD9><<<grid, block, 0, s>>>(pi, tasks, qt_off, qn, ctr, kPersistQueues, wait_ticks); break;
    default: k_stream_persist<KIND13, kPD13><<<grid, block, 0, s>>>(pi, tasks, qt_off, qn, ctr, kPersistQueues, wait_ticks); break;
    }
    return hipGetLastError();
}

hipError_t xcc_probe(int* out, int n, hipStream_t s)
{
    k_xcc_probe<<<n, 64, 0, s>>>(out, n);
    return hipGetLastError();
}

size_t batch_item_size(int precision)
{
    return precision == 0 ? sizeof(BatchItem<PF64>) : sizeof(BatchItem<PF32C>);
}

void batch_tables(int precision, int kind, int depth, int rows, const std::vector<BatchInst>& insts, BatchTables& gen,
                  BatchTables& inr)
{
    if (precision == 0) tables_prec<PF64>(kind, depth, rows, insts, gen, inr);
    else tables_prec<PF32C>(kind, depth, rows, insts, gen, inr);
}

hipError_t batch_launch(int precision, int kind, int depth, bool interior, const void* d_items, const int* d_prefix,
                        int count, int total, hipStream_t s)
{
    if (count <= 0 || total <= 0) return hipSuccess;
    if (precision == 0) return blaunch_prec<PF64>(kind, depth, interior, d_items, d_prefix, count, total, s);
    return blaunch_prec<PF32C>(kind, depth, interior, d_items, d_prefix, count, total, s);
}

hipError_t stream_step_f64(const Grid& g, int kind, const StepW64& w, const StreamShape& sh, const double* p_in,
                           const double* c_in, double* p_out, double* c_out, hipStream_t s)
{
    SArgs<double> a{};
    a.in_w0 = c_in;
    a.in_w1 = nullptr;
    a.in_p = p_in;
    if (sh.depth == 1 && p_out == p_in) {
        a.out_w0 = p_out;  // level k+1 over level k-1
        a.out_w1 = nullptr;
        a.out_p = nullptr;
    } else {
        a.out_w0 = c_out;
        a.out_w1 = nullptr;
        a.out_p = p_out;
    }
    return launch<PF64>(kind, g, w, sh, a, s);
}

hipError_t stream_step_f32c(const Grid& g, int kind, const StepW32& w, const StreamShape& sh, const float* u,
                            const float* lo, const float* d, float* u2, float* lo2, float* d2, hipStream_t s)
{
    SArgs<float> a{};
    a.in_w0 = u;
    a.in_w1 = lo;
    a.in_p = d;
    a.out_w0 = u2;
    a.out_w1 = lo2;
    a.out_p = d2;
    return launch<PF32C>(kind, g, w, sh, a, s);
}

}  // namespace w2d

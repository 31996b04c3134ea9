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

template <class Prec, int K, int DEPTH, int CW>
__global__ __launch_bounds__(kWave* kWavesPerBlock, 2) void k_stream(SArgs<typename Prec::T> a,
                                                                      typename Prec::W w)
{
    using T = typename Prec::T;
    constexpr int R = KT<K>::R;
    constexpr int NS = 2 * R + 1;  // rows in a level's window
    constexpr int NW = Prec::NW;
    constexpr int H = R * DEPTH;   // halo columns on each side
    constexpr int SW = kWave * CW - 2 * H;
    constexpr int E = CW + 2 * R;  // extended row: R neighbours each side

    const int lane = threadIdx.x & (kWave - 1);
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (wid >= a.nwork) return;  // whole wavefronts only
    const int nx = a.g.nx, ny = a.g.ny, ld = a.g.ld;
    const int strip = wid % a.nstrips, seg = wid / a.nstrips;
    const int x0 = strip * SW - H;
    const int xl = x0 + lane * CW;
    const int y0 = seg * a.rows;
    const int y1 = min(y0 + a.rows, ny);

    // Column classes of this lane's CW columns.
    bool ld_ok[CW], st_ok[CW], zero_col[CW];
    int gsrc_lane[CW], gsrc_m[CW];
    bool ghost[CW];
    for (int m = 0; m < CW; ++m) {
        const int x = xl + m;
        ld_ok[m] = (x >= 0 && x < nx);
        st_ok[m] = (x >= x0 + H && x < x0 + H + SW && x < nx);
        ghost[m] = (R == 2) && (x == -1 || x == nx);
        zero_col[m] = !(x >= 1 && x <= nx - 2) && !ghost[m];
        const int src = (x == -1) ? 1 : nx - 2;
        const int off = src - x0;
        gsrc_lane[m] = off / CW;
        gsrc_m[m] = off % CW;
    }
    const bool edge = (x0 <= 0) || (x0 + kWave * CW - 1 >= nx - 1);

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

    const T* inw[2] = {a.in_w0, a.in_w1};
    T* outw[2] = {a.out_w0, a.out_w1};

    // Boundary rule along x on a freshly produced row (centre values only).
    auto fix_columns = [&](T (&v)[NW][E]) {
        if (!edge) return;
#pragma unroll
        for (int f = 0; f < NW; ++f) {
            T g[CW];
#pragma unroll
            for (int m = 0; m < CW; ++m) g[m] = T(0);
            if constexpr (R == 2) {
#pragma unroll
                for (int mm = 0; mm < CW; ++mm) {
#pragma unroll
                    for (int m = 0; m < CW; ++m) {
                        const T s = __shfl(v[f][R + mm], gsrc_lane[m]);
                        if (gsrc_m[m] == mm) g[m] = -s;
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < CW; ++m) {
                if (zero_col[m]) v[f][R + m] = T(0);
                if (ghost[m]) v[f][R + m] = g[m];
            }
        }
    };
    // Fill the R neighbour columns on each side from the adjacent lanes.
    auto extend = [&](T (&v)[NW][E]) {
#pragma unroll
        for (int f = 0; f < NW; ++f) {
#pragma unroll
            for (int e = 0; e < R; ++e) v[f][e] = from_left(v[f][CW + e]);
#pragma unroll
            for (int e = R + CW; e < E; ++e) v[f][e] = from_right(v[f][e - CW]);
        }
    };
    auto zero_row = [&](T (&v)[NW][E]) {
#pragma unroll
        for (int f = 0; f < NW; ++f)
#pragma unroll
            for (int e = 0; e < E; ++e) v[f][e] = T(0);
    };
    auto neg_copy = [&](T (&dst)[NW][E], const T (&src)[NW][E]) {
#pragma unroll
        for (int f = 0; f < NW; ++f)
#pragma unroll
            for (int e = 0; e < E; ++e) dst[f][e] = -src[f][e];
    };

    const bool t1_narrow = (DEPTH == 1);  // only the output region's point field is needed
    // Issue the loads of level-0 row jj (window fields) and of the point
    // field at row jj - R into the given slots.
    // Addresses are clamped into the grid so that every load is in bounds;
    // values from outside the wanted range are then replaced by 0.
    auto issue_loads = [&](int jj, T (&v)[NW][E], T (&p)[CW]) {
        const bool row_ok = (jj >= 0 && jj < ny);
        const int jp = jj - R;
        const bool prow_ok = t1_narrow ? (jp >= y0 && jp < y1) : (jp >= 0 && jp < ny);
        const int jr = row_ok ? jj : 0;
        const int jpr = prow_ok ? jp : 0;
#pragma unroll
        for (int m = 0; m < CW; ++m) {
            const int xr = ld_ok[m] ? xl + m : 0;
            const size_t o = (size_t)jr * ld + xr;
#pragma unroll
            for (int f = 0; f < NW; ++f) {
                const T x = inw[f][o];
                v[f][R + m] = (row_ok && ld_ok[m]) ? x : T(0);
            }
            const bool pok = prow_ok && (t1_narrow ? st_ok[m] : ld_ok[m]);
            const T x = a.in_p[(size_t)jpr * ld + xr];
            p[m] = pok ? x : T(0);
        }
    };

    const int jlo = y0 - H;
    const int jhi = y1 - 1 + H;
    const int jA = floor_div(jlo, NS) * NS;
    issue_loads(jA, win[0][0], pf[0][mod_c(-R, NS)]);

    for (int jb = jA; jb <= jhi; jb += NS) {
#pragma unroll
        for (int ph = 0; ph < NS; ++ph) {
            const int j = jb + ph;
            // 1. Finish level-0 row j (its loads were issued one row ago).
            {
                T(&v)[NW][E] = win[0][ph];
                if (j >= 1 && j <= ny - 2) {
                    fix_columns(v);
                    extend(v);
                } else {
                    zero_row(v);
                }
                if constexpr (R == 2) {
                    if (j == 1) neg_copy(win[0][mod_c(-1, NS)], v);
                    if (j == ny) neg_copy(v, win[0][mod_c(ph - 2, NS)]);
                }
            }
            // 2. Levels 1..DEPTH at rows j - t*R; the next row's loads go out
            //    right after level 1, whose inputs they overwrite.
#pragma unroll
            for (int t = 1; t <= DEPTH; ++t) {
                if (t == 2) {
                    // Slot (ph+1) of level 0 held row j+1-NS = j-2R, last
                    // needed by level 1 at this row.
                    issue_loads(j + 1, win[0][mod_c(ph + 1, NS)], pf[0][mod_c(ph + 1 - R, NS)]);
                }
                const int y = j - t * R;
                if (y < y0 - (DEPTH - t) * R || y > y1 - 1 + (DEPTH - t) * R) continue;
                const int sy = mod_c(ph - t * R, NS);
                const T(&Wc)[NW][E] = win[t - 1][sy];
                const T(&Wn)[NW][E] = win[t - 1][mod_c(ph - t * R + 1, NS)];
                const T(&Ws)[NW][E] = win[t - 1][mod_c(ph - t * R - 1, NS)];
                const T(&Wnn)[NW][E] = win[t - 1][mod_c(ph - t * R + 2, NS)];
                const T(&Wss)[NW][E] = win[t - 1][mod_c(ph - t * R - 2, NS)];
                const T(&Pin)[CW] = pf[t - 1][sy];
                T nv[NW][E];
                T np[CW];
                const bool inside = (y >= 1 && y <= ny - 2);
                if (inside) {
#pragma unroll
                    for (int m = 0; m < CW; ++m) {
                        const int e = R + m;
                        Nbh<T> nb[NW];
#pragma unroll
                        for (int f = 0; f < NW; ++f) {
                            nb[f].C = Wc[f][e];
                            nb[f].E = Wc[f][e + 1];
                            nb[f].W = Wc[f][e - 1];
                            nb[f].N = Wn[f][e];
                            nb[f].S = Ws[f][e];
                            if constexpr (KT<K>::DIAG) {
                                nb[f].NE = Wn[f][e + 1];
                                nb[f].NW = Wn[f][e - 1];
                                nb[f].SE = Ws[f][e + 1];
                                nb[f].SW = Ws[f][e - 1];
                            } else {
                                nb[f].NE = nb[f].NW = nb[f].SE = nb[f].SW = T(0);
                            }
                            if constexpr (KT<K>::AX2) {
                                nb[f].EE = Wc[f][e + 2];
                                nb[f].WW = Wc[f][e - 2];
                                nb[f].NN = Wnn[f][e];
                                nb[f].SS = Wss[f][e];
                            } else {
                                nb[f].EE = nb[f].WW = nb[f].NN = nb[f].SS = T(0);
                            }
                        }
                        if constexpr (NW == 1) {
                            const T s = lap_diff<K>(nb[0], w.w10, w.w11, w.w20);
                            nv[0][e] = (T)f64_update((double)nb[0].C, (double)Pin[m], (double)s);
                            np[m] = nb[0].C;
                        } else {
                            const float su = lap_diff<K>(nb[0], w.w10, w.w11, w.w20);
                            const float sl = lap_sum<K>(nb[1], w.wc, w.w10, w.w11, w.w20);
                            float u2, l2, d2;
                            f32c_update(su, sl, nb[0].C, nb[1].C, Pin[m], u2, l2, d2);
                            nv[0][e] = u2;
                            nv[1][e] = l2;
                            np[m] = d2;
                        }
                    }
                    fix_columns(nv);
                    if (edge) {
#pragma unroll
                        for (int m = 0; m < CW; ++m)
                            if (zero_col[m] || ghost[m]) np[m] = T(0);
                    }
                } else {
#pragma unroll
                    for (int f = 0; f < NW; ++f)
#pragma unroll
                        for (int m = 0; m < CW; ++m) nv[f][R + m] = T(0);
#pragma unroll
                    for (int m = 0; m < CW; ++m) np[m] = T(0);
                }
                if (t < DEPTH) {
                    extend(nv);
                    T(&dst)[NW][E] = win[t][sy];
#pragma unroll
                    for (int f = 0; f < NW; ++f)
#pragma unroll
                        for (int e = 0; e < E; ++e) dst[f][e] = nv[f][e];
#pragma unroll
                    for (int m = 0; m < CW; ++m) pf[t][sy][m] = np[m];
                    if constexpr (R == 2) {
                        if (y == 1) neg_copy(win[t][mod_c(ph - t * R - 2, NS)], dst);
                        if (y == ny) neg_copy(dst, win[t][mod_c(ph - t * R - 2, NS)]);
                    }
                } else if (y >= y0 && y < y1) {
                    // Output row: level DEPTH (and DEPTH-1 for FP64).
#pragma unroll
                    for (int m = 0; m < CW; ++m) {
                        if (!st_ok[m]) continue;
                        const size_t o = (size_t)y * ld + (xl + m);
#pragma unroll
                        for (int f = 0; f < NW; ++f) outw[f][o] = nv[f][R + m];
                        if (a.out_p) a.out_p[o] = np[m];
                    }
                }
            }
            if constexpr (DEPTH == 1) issue_loads(j + 1, win[0][mod_c(ph + 1, NS)], pf[0][mod_c(ph + 1 - R, NS)]);
        }
    }
}

template <class Prec, int K, int DEPTH>
hipError_t launch_depth(const Grid& g, const typename Prec::W& w, int rows, SArgs<typename Prec::T> a,
                        hipStream_t s)
{
    constexpr int CW = 2;
    constexpr int R = KT<K>::R;
    constexpr int SW = kWave * CW - 2 * R * DEPTH;
    static_assert(SW > 0, "strip too narrow");
    a.g = g;
    a.rows = rows;
    a.nstrips = (g.nx + SW - 1) / SW;
    const int nseg = (g.ny + rows - 1) / rows;
    a.nwork = a.nstrips * nseg;
    const int blocks = (a.nwork + kWavesPerBlock - 1) / kWavesPerBlock;
    k_stream<Prec, K, DEPTH, CW><<<blocks, kWave * kWavesPerBlock, 0, s>>>(a, w);
    return hipGetLastError();
}

template <class Prec, int K>
hipError_t launch_kind(const Grid& g, const typename Prec::W& w, const StreamShape& sh, SArgs<typename Prec::T> a,
                       hipStream_t s)
{
    switch (sh.depth) {
    case 1: return launch_depth<Prec, K, 1>(g, w, sh.rows, a, s);
    case 2: return launch_depth<Prec, K, 2>(g, w, sh.rows, a, s);
    case 3: return launch_depth<Prec, K, 3>(g, w, sh.rows, a, s);
    case 4: return launch_depth<Prec, K, 4>(g, w, sh.rows, a, s);
    case 6: return launch_depth<Prec, K, 6>(g, w, sh.rows, a, s);
    case 8: return launch_depth<Prec, K, 8>(g, w, sh.rows, a, s);
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

int stream_columns_per_wave(int) { return kWave * 2; }

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

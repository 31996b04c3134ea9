// Per-node arithmetic of the schemes, shared by every kernel so that all
// launch shapes and kernel variants produce bit-identical results.
//
// The file is compiled with -ffp-contract=off: every operation rounds as
// written, and fused multiply-adds appear only where fma() is spelled out.
#pragma once

#include <hip/hip_runtime.h>

namespace w2d {

// Stencil classes: 5-point (axis neighbours only), 9-point (axis and
// diagonal) and 13-point (axis, diagonal and the axis neighbours two lines
// away).  The isotropic comparison scheme is a 9-point class with other
// weights.
enum Kind : int { KIND5 = 0, KIND9 = 1, KIND13 = 2 };

template <int K>
struct KT {
    static constexpr int R = (K == KIND13) ? 2 : 1;  // stencil radius
    static constexpr bool DIAG = (K != KIND5);
    static constexpr bool AX2 = (K == KIND13);
};

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Values of one node's stencil neighbourhood: centre, axis neighbours
// (E = i+1, W = i-1, N = j+1, S = j-1), diagonals, and axis neighbours two
// lines away.  Unused members are ignored for smaller stencils.
template <typename T>
struct Nbh {
    T C, E, W, N, S, NE, NW, SE, SW, EE, WW, NN, SS;
};

// sum_q w_q delta(q): each rotation sum of Sec. 6.2.1 (eq. notations2) is
// evaluated as a sum of neighbour-minus-centre differences, pairing opposite
// neighbours.  The differences keep the result accurate when the values are
// close (the usual case for a smooth field), which matters in single
// precision.
template <int K, typename T>
__device__ __forceinline__ T lap_diff(const Nbh<T>& v, T w10, T w11, T w20)
{
    const T C = v.C;
    T s = w10 * (((v.E - C) + (v.W - C)) + ((v.N - C) + (v.S - C)));
    if constexpr (KT<K>::DIAG) s = fmaT(w11, ((v.NE - C) + (v.SW - C)) + ((v.NW - C) + (v.SE - C)), s);
    if constexpr (KT<K>::AX2) s = fmaT(w20, ((v.EE - C) + (v.WW - C)) + ((v.NN - C) + (v.SS - C)), s);
    return s;
}

// The same operator as a weighted sum (wc = -4 (w10 + w11 + w20)).  Used
// for the low-order part `lo` of the compensated state, whose own rounding
// is far below the precision that is carried.
template <int K>
__device__ __forceinline__ float lap_sum(const Nbh<float>& v, float wc, float w10, float w11, float w20)
{
    float s = fmaT(w10, (v.E + v.W) + (v.N + v.S), wc * v.C);
    if constexpr (KT<K>::DIAG) s = fmaT(w11, (v.NE + v.NW) + (v.SE + v.SW), s);
    if constexpr (KT<K>::AX2) s = fmaT(w20, (v.EE + v.WW) + (v.NN + v.SS), s);
    return s;
}

// Increment of the compensated level u + lo (single precision):
// sum_q w_q delta(q) applied to u + lo.
//
// 5-point: the four neighbour differences of u (as lap_diff) times the
// two-float weight, plus lap_sum of lo.
//
// 9- and 13-point: regrouped by exact identities between the rotation sums
// and the second differences Dx f = f(i+1) - 2f(i) + f(i-1), Dy likewise:
//   delta(1,0) = Dx + Dy,  delta(1,1) = 2 (Dx + Dy) + Dx Dy,
//   delta(2,0) = Dx Dx + Dy Dy + 4 (Dx + Dy),
// so the increment is wx (Dx + Dy) + w11 Dx Dy + w20 (Dx Dx + Dy Dy) with
// wx = w10 + 2 w11 + 4 w20 (lambda^2 for the schemes of Sec. 6), applied
// as the two-float weight wx + wxl (see StepW32).  Each
// second difference of u is a difference of two neighbour differences,
// which are exact for close values; those of u and of lo are added only
// after they are formed.  The mixed and fourth differences are taken of
// the summed second differences q = Dy u + Dy lo and p = Dx u + Dx lo.  Every
// step is symmetric under negation and under mirroring, so odd-reflected
// data give odd-reflected increments with exact zeros on the mirror lines.
template <typename T>
__device__ __forceinline__ T d2(T a, T c, T b)  // (a - c) - (c - b)
{
    return (a - c) - (c - b);
}

// x times the two-float weight wx + wxl, rounded once.
__device__ __forceinline__ float mul_w2(float wx, float wxl, float x) { return fmaT(wx, x, wxl * x); }

template <int K>
__device__ __forceinline__ float f32c_incr(const Nbh<float>& u, const Nbh<float>& l, float wc, float w10, float w11,
                                           float w20, float wx, float wxl)
{
    if constexpr (K == KIND5) {
        // wx = w10 for this class.
        const float su = mul_w2(wx, wxl, ((u.E - u.C) + (u.W - u.C)) + ((u.N - u.C) + (u.S - u.C)));
        return su + lap_sum<K>(l, wc, w10, w11, w20);
    } else {
        const float q = d2(u.N, u.C, u.S) + d2(l.N, l.C, l.S);
        const float p = d2(u.E, u.C, u.W) + d2(l.E, l.C, l.W);
        const float qE = d2(u.NE, u.E, u.SE) + d2(l.NE, l.E, l.SE);
        const float qW = d2(u.NW, u.W, u.SW) + d2(l.NW, l.W, l.SW);
        float s = fmaT(w11, d2(qE, q, qW), mul_w2(wx, wxl, p + q));
        if constexpr (KT<K>::AX2) {
            const float pE = d2(u.EE, u.E, u.C) + d2(l.EE, l.E, l.C);
            const float pW = d2(u.C, u.W, u.WW) + d2(l.C, l.W, l.WW);
            const float qN = d2(u.NN, u.N, u.C) + d2(l.NN, l.N, l.C);
            const float qS = d2(u.C, u.S, u.SS) + d2(l.C, l.S, l.SS);
            s = fmaT(w20, d2(pE, p, pW) + d2(qN, q, qS), s);
        }
        return s;
    }
}

// The same increment in double precision on one field (the FP64 two-step
// update): the 5-point scheme as lap_diff, the 9- and 13-point schemes
// regrouped as f32c_incr without the lo terms.
template <int K>
__device__ __forceinline__ double f64_incr(const Nbh<double>& u, double w10, double w11, double w20, double wx)
{
    if constexpr (K == KIND5) {
        return lap_diff<K>(u, w10, w11, w20);
    } else {
        const double q = d2(u.N, u.C, u.S);
        const double p = d2(u.E, u.C, u.W);
        double s = fmaT(w11, d2(d2(u.NE, u.E, u.SE), q, d2(u.NW, u.W, u.SW)), wx * (p + q));
        if constexpr (KT<K>::AX2)
            s = fmaT(w20, d2(d2(u.EE, u.E, u.C), p, d2(u.C, u.W, u.WW)) + d2(d2(u.NN, u.N, u.C), q, d2(u.C, u.S, u.SS)), s);
        return s;
    }
}

// FP64 two-step update (Sec. 3, eq. A2): u^{k+1} = 2u^k - u^{k-1} + s.
__device__ __forceinline__ double f64_update(double C, double P, double s) { return ((C + C) - P) + s; }

// Compensated FP32 two-step update.  The level is u + lo, d = u^k - u^{k-1}.
// With s the stencil increment of u + lo: d <- d + s; the new level
// u + lo + d is formed as y = d + lo followed by Dekker's Fast2Sum u + y =
// t + e (t = u + y, e = y - (t - u)), so that t is the new u and e the new
// lo.  The sum is exact whenever |u| >= |y|.  Where u is smaller (near a
// zero crossing of u, where y is largest) t - u rounds to within half an
// ulp of y, so e is off by at most that much: |y| is the change of the level
// over one step, bounded by omega tau max|u| << max|u|, so the loss is far
// below the rounding of an uncompensated single-precision level and does
// not accumulate coherently.  Knuth's branch-free TwoSum would make every
// sum exact at three more operations per update; on coarse 64^2 - 129^2
// grids over 5000 steps both give 1e-7 to 7e-7 of max|u| against FP64.
// Every operation is odd under negation, so reflected data stay reflected.
__device__ __forceinline__ void f32c_update(float s, float u, float lo, float d, float& u2, float& lo2, float& dn2)
{
    const float dn = d + s;
    const float y = dn + lo;
    const float t = u + y;
    lo2 = y - (t - u);
    u2 = t;
    dn2 = dn;
}

// FP64 first step (Sec. 3, eq. A1): u^1 = (u^0 + sum wa delta(u^0)) +
// tau (v^0 + sum wb epsilon(v^0)); sb = 0 for the conventional first step.
__device__ __forceinline__ double first_update(double u0c, double sa, double v0c, double sb, double tau)
{
    return (u0c + sa) + tau * (v0c + sb);
}

// Split of an FP64 level into the compensated FP32 state.
__device__ __forceinline__ void f32c_split(double cur, double prev, float& u, float& lo, float& d)
{
    u = (float)cur;
    lo = (float)(cur - (double)u);
    d = (float)(cur - prev);
}

__device__ __forceinline__ double f32c_join(float u, float lo) { return (double)u + (double)lo; }

}  // namespace w2d

// Schemes built from a caller's stencil and monomial set by the
// construction of Sec. 4-5 (host code only).
//
// Given m stencil nodes x_r (integer offsets in grid steps) and m monomials
// mu_s = x1^a1 x2^a2 with a nonsingular matrix D[s][r] = mu_s(x_r) (the
// unisolvence condition of Sec. 4), the Lagrange basis is
// phi_r = sum_s C[r][s] mu_s with C = D^{-1} (eq. matrix2, Lagrange), and
// the node weights of the operators A and B of Sec. 3 are A phi_r and
// B phi_r (Sec. 5).  Both operators act on a polynomial through the Taylor
// series of the wave solution (the identity that Sec. 5's exact integrals
// over the disk satisfy monomial by monomial):
//   A f = sum_j (c tau)^{2j} / (2j)! Lap^j f,
//   B f = sum_j tau^{2j+1} c^{2j} / (2j+1)! Lap^j f,
// so on mu_s centred at the node (h = 1) only the term 2j = a1 + a2
// survives: A mu_s = lambda^{2j} / (2j)! [Lap^j mu_s], and
// B mu_s / tau = lambda^{2j} / (2j+1)! [Lap^j mu_s], with [.] the constant
// that Lap^j leaves of a monomial of degree 2j (0 unless both exponents are
// even).
//
// The weights must be those of a scheme the kernels run: symmetric under
// the eight symmetries of the square and zero more than three lines from
// the centre, so that they are constant on the node classes (q1, q2),
// q1 >= q2 >= 0, q1 <= 3 (the nodes (+-q1, +-q2) and (+-q2, +-q1)).
// Schemes with weight only on (1,0), (1,1), (2,0) run as the 5-, 9- or
// 13-point class; the others as KINDW.  The stability limit is found
// numerically from the two-step symbol (von Neumann): with
// S(theta) = sum_c 2 A_c(lambda) sigma_c(theta) and sigma_c the sum over
// the class's nodes of cos(q . theta) - 1 (sigma_10 = 2 cos t1 + 2 cos t2 -
// 4, sigma_11 = 4 cos t1 cos t2 - 4, sigma_20 = 2 cos 2t1 + 2 cos 2t2 - 4,
// and for an eight-node class 4 cos q1t1 cos q2t2 + 4 cos q2t1 cos q1t2 -
// 8), the update u^{k+1} - 2u^k + u^{k-1} = S u^k keeps every mode bounded
// iff -4 <= S <= 0 for all theta.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "host.h"

namespace w2d_host {
namespace {

using w2d::KIND13;
using w2d::KIND5;
using w2d::KIND9;
using w2d::KINDW;
using w2d::kWideClasses;

constexpr int kQ[kWideClasses][2] = {{1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}, {3, 0}, {3, 1}, {3, 2}, {3, 3}};

constexpr int kMaxNodes = 64;
constexpr int kMaxExp = 12;

std::mutex g_mu;
std::vector<CustomScheme> g_schemes;

// Constant left by Lap^j on x1^a x2^b with a + b = 2j, by repeated
// application of Lap (x1^a x2^b) = a(a-1) x1^(a-2) x2^b + b(b-1) x1^a x2^(b-2).
double lap_constant(int a, int b)
{
    std::map<std::pair<int, int>, double> p{{{a, b}, 1.0}};
    while (!p.empty() && (p.begin()->first.first + p.begin()->first.second) > 0) {
        std::map<std::pair<int, int>, double> q;
        for (const auto& kv : p) {
            const int e1 = kv.first.first, e2 = kv.first.second;
            if (e1 >= 2) q[{e1 - 2, e2}] += kv.second * e1 * (e1 - 1);
            if (e2 >= 2) q[{e1, e2 - 2}] += kv.second * e2 * (e2 - 1);
        }
        p.swap(q);
    }
    const auto it = p.find({0, 0});
    return it == p.end() ? 0.0 : it->second;
}

double factorial(int n)
{
    double f = 1.0;
    for (int k = 2; k <= n; ++k) f *= k;
    return f;
}

// C = D^{-1} (row-major, n x n) by Gauss-Jordan elimination with partial
// pivoting; false when D is singular.
bool invert(std::vector<double> D, int n, std::vector<double>& C)
{
    C.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) C[(size_t)i * n + i] = 1.0;
    double scale = 0.0;
    for (double v : D) scale = std::max(scale, std::fabs(v));
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(D[(size_t)r * n + col]) > std::fabs(D[(size_t)piv * n + col])) piv = r;
        if (std::fabs(D[(size_t)piv * n + col]) <= 1e-12 * scale) return false;
        if (piv != col)
            for (int k = 0; k < n; ++k) {
                std::swap(D[(size_t)piv * n + k], D[(size_t)col * n + k]);
                std::swap(C[(size_t)piv * n + k], C[(size_t)col * n + k]);
            }
        const double p = D[(size_t)col * n + col];
        for (int k = 0; k < n; ++k) {
            D[(size_t)col * n + k] /= p;
            C[(size_t)col * n + k] /= p;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double f = D[(size_t)r * n + col];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                D[(size_t)r * n + k] -= f * D[(size_t)col * n + k];
                C[(size_t)r * n + k] -= f * C[(size_t)col * n + k];
            }
        }
    }
    return true;
}

double poly_eval(const double* p, int deg, double x)
{
    double s = 0.0;
    for (int k = deg; k >= 0; --k) s = s * x + p[k];
    return s;
}

// Two-step symbol extremes over theta in [0, pi]^2 at Courant number lam:
// a grid, then a local refinement of the grid's extreme points.
void symbol_range(const CustomScheme& s, double lam, double* smin, double* smax)
{
    double w[kWideClasses];
    for (int c = 0; c < kWideClasses; ++c) w[c] = 2.0 * poly_eval(s.a[c], CustomScheme::kDeg, lam);
    auto S = [&](double t1, double t2) {
        double v = 0.0;
        for (int c = 0; c < kWideClasses; ++c) {
            if (w[c] == 0.0) continue;
            const int q1 = kQ[c][0], q2 = kQ[c][1];
            double sig;
            if (q2 == 0) sig = 2.0 * std::cos(q1 * t1) + 2.0 * std::cos(q1 * t2) - 4.0;
            else if (q1 == q2) sig = 4.0 * std::cos(q1 * t1) * std::cos(q1 * t2) - 4.0;
            else sig = 4.0 * std::cos(q1 * t1) * std::cos(q2 * t2) + 4.0 * std::cos(q2 * t1) * std::cos(q1 * t2) - 8.0;
            v += w[c] * sig;
        }
        return v;
    };
    constexpr int N = 128;
    const double dt = M_PI / N;
    double lo = 0.0, hi = 0.0;
    int ilo = 0, jlo = 0, ihi = 0, jhi = 0;
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= i; ++j) {  // S is symmetric in (t1, t2)
            const double v = S(i * dt, j * dt);
            if (v < lo) { lo = v; ilo = i; jlo = j; }
            if (v > hi) { hi = v; ihi = i; jhi = j; }
        }
    // Coordinate search around each extreme point, within the square.
    auto refine = [&](int i, int j, double sign) {
        double t1 = i * dt, t2 = j * dt, best = sign * S(t1, t2), step = dt;
        for (int it = 0; it < 60 && step > 1e-13; ++it) {
            bool moved = false;
            const double d[4][2] = {{step, 0}, {-step, 0}, {0, step}, {0, -step}};
            for (const auto& dd : d) {
                const double u1 = std::min(M_PI, std::max(0.0, t1 + dd[0]));
                const double u2 = std::min(M_PI, std::max(0.0, t2 + dd[1]));
                const double v = sign * S(u1, u2);
                if (v > best) {
                    best = v;
                    t1 = u1;
                    t2 = u2;
                    moved = true;
                }
            }
            if (!moved) step *= 0.5;
        }
        return sign * best;
    };
    *smin = std::min(lo, refine(ilo, jlo, -1.0));
    *smax = std::max(hi, refine(ihi, jhi, 1.0));
}

bool stable_at(const CustomScheme& s, double lam)
{
    double smin, smax;
    symbol_range(s, lam, &smin, &smax);
    return smin >= -4.0 * (1.0 + 1e-13) && smax <= 4e-13;
}

// Largest lambda in (0, 4] below which the two-step update is stable: a
// scan in steps of 1/256, then bisection to 1e-12.
double stability_limit(const CustomScheme& s)
{
    double ok = 0.0, bad = -1.0;
    for (int k = 1; k <= 1024; ++k) {
        const double lam = k / 256.0;
        if (stable_at(s, lam)) ok = lam;
        else {
            bad = lam;
            break;
        }
    }
    if (bad < 0.0) return ok;
    while (bad - ok > 1e-12 * bad) {
        const double mid = 0.5 * (ok + bad);
        if (stable_at(s, mid)) ok = mid;
        else bad = mid;
    }
    return ok;
}

// Index of the class of node (q1, q2) in kQ; -1 for the centre,
// kWideClasses for a node more than three lines out.
int class_of(int q1, int q2)
{
    const int a = std::abs(q1), b = std::abs(q2);
    const int hi = std::max(a, b), lo = std::min(a, b);
    if (hi == 0) return -1;
    for (int c = 0; c < kWideClasses; ++c)
        if (kQ[c][0] == hi && kQ[c][1] == lo) return c;
    return kWideClasses;
}

int class_size(int c) { return (kQ[c][1] == 0 || kQ[c][1] == kQ[c][0]) ? 4 : 8; }

}  // namespace

int custom_scheme_create(int m, const int32_t* nodes, const int32_t* exps, int* id)
{
    if (m < 1 || m > kMaxNodes) return fail(WAVE2D_EINVAL, "m must be in [1, %d] (got %d)", kMaxNodes, m);
    if (!nodes || !exps || !id) return fail(WAVE2D_EINVAL, "nodes, exps and scheme must not be NULL");
    for (int r = 0; r < m; ++r) {
        if (std::abs(nodes[2 * r]) > 8 || std::abs(nodes[2 * r + 1]) > 8)
            return fail(WAVE2D_EINVAL, "node %d (%d, %d) is more than 8 steps away", r, nodes[2 * r], nodes[2 * r + 1]);
        if (exps[2 * r] < 0 || exps[2 * r + 1] < 0 || exps[2 * r] + exps[2 * r + 1] > kMaxExp)
            return fail(WAVE2D_EINVAL, "monomial %d (%d, %d): exponents must be >= 0 with degree <= %d", r,
                        exps[2 * r], exps[2 * r + 1], kMaxExp);
        for (int t = 0; t < r; ++t) {
            if (nodes[2 * t] == nodes[2 * r] && nodes[2 * t + 1] == nodes[2 * r + 1])
                return fail(WAVE2D_EINVAL, "node (%d, %d) appears twice", nodes[2 * r], nodes[2 * r + 1]);
            if (exps[2 * t] == exps[2 * r] && exps[2 * t + 1] == exps[2 * r + 1])
                return fail(WAVE2D_EINVAL, "monomial (%d, %d) appears twice", exps[2 * r], exps[2 * r + 1]);
        }
    }
    // D[s][r] = mu_s(x_r) (eq. matrix1), C = D^{-1} (eq. matrix2).
    std::vector<double> D((size_t)m * m), C;
    for (int s = 0; s < m; ++s)
        for (int r = 0; r < m; ++r)
            D[(size_t)s * m + r] = std::pow((double)nodes[2 * r], exps[2 * s]) * std::pow((double)nodes[2 * r + 1], exps[2 * s + 1]);
    if (!invert(D, m, C)) return fail(WAVE2D_EINVAL, "the stencil is not unisolvent for these monomials (D is singular)");
    // With D[s][t] = mu_s(x_t), phi_r = sum_s K[r][s] mu_s has
    // phi_r(x_t) = (K D)[r][t] = delta_rt for K = D^{-1} = C.  Node weights
    // as polynomials in lambda: A phi_r and B phi_r / tau.
    std::vector<double> Aw((size_t)m * (CustomScheme::kDeg + 1), 0.0), Bw(Aw.size(), 0.0);
    for (int s = 0; s < m; ++s) {
        const int a1 = exps[2 * s], a2 = exps[2 * s + 1];
        if ((a1 | a2) & 1) continue;  // odd powers average out over the disk
        const int deg = a1 + a2;
        if (deg > CustomScheme::kDeg) return fail(WAVE2D_EINVAL, "monomial degree %d exceeds %d", deg, CustomScheme::kDeg);
        const double k = lap_constant(a1, a2);
        const double ka = k / factorial(deg), kb = k / factorial(deg + 1);
        for (int r = 0; r < m; ++r) {
            const double cr = C[(size_t)r * m + s];
            Aw[(size_t)r * (CustomScheme::kDeg + 1) + deg] += cr * ka;
            Bw[(size_t)r * (CustomScheme::kDeg + 1) + deg] += cr * kb;
        }
    }
    // Lagrange property, as a check of the solve.
    for (int r = 0; r < m; ++r)
        for (int t = 0; t < m; ++t) {
            double v = 0.0;
            for (int s = 0; s < m; ++s) v += C[(size_t)r * m + s] * D[(size_t)s * m + t];
            if (std::fabs(v - (r == t ? 1.0 : 0.0)) > 1e-9)
                return fail(WAVE2D_EINVAL, "Lagrange basis check failed at node %d (ill-conditioned stencil)", r);
        }
    // Classes: every node of a class carries the same polynomials; nodes
    // outside the kernels' classes must carry zero weight.
    CustomScheme cs{};
    bool seen[kWideClasses] = {};
    double scale = 0.0;
    for (double v : Aw) scale = std::max(scale, std::fabs(v));
    for (double v : Bw) scale = std::max(scale, std::fabs(v));
    const double tol = 1e-10 * std::max(1.0, scale);
    // The kernels write each update as the centre value plus weighted
    // differences, which needs the weights of all nodes to reproduce
    // constants: A 1 = 1 and B 1 = tau (true when the monomials include 1).
    for (int k = 0; k <= CustomScheme::kDeg; ++k) {
        double sa = 0.0, sb = 0.0;
        for (int r = 0; r < m; ++r) {
            sa += Aw[(size_t)r * (CustomScheme::kDeg + 1) + k];
            sb += Bw[(size_t)r * (CustomScheme::kDeg + 1) + k];
        }
        const double want = (k == 0) ? 1.0 : 0.0;
        if (std::fabs(sa - want) > tol || std::fabs(sb - want) > tol)
            return fail(WAVE2D_EINVAL, "the weights do not reproduce constants (include the monomial 1)");
    }
    auto is_zero = [&](int r) {
        const double* pa = &Aw[(size_t)r * (CustomScheme::kDeg + 1)];
        const double* pb = &Bw[(size_t)r * (CustomScheme::kDeg + 1)];
        for (int k = 0; k <= CustomScheme::kDeg; ++k)
            if (std::fabs(pa[k]) > tol || std::fabs(pb[k]) > tol) return false;
        return true;
    };
    for (int r = 0; r < m; ++r)
        if (class_of(nodes[2 * r], nodes[2 * r + 1]) == kWideClasses && !is_zero(r))
            return fail(WAVE2D_EINVAL, "node (%d, %d) has nonzero weight more than three lines from the centre",
                        nodes[2 * r], nodes[2 * r + 1]);
    // Each class: every node equals the class's first node; a class with
    // weight needs all of its four or eight nodes.
    for (int c = 0; c < kWideClasses; ++c) {
        int ref = -1, count = 0;
        for (int r = 0; r < m; ++r) {
            if (class_of(nodes[2 * r], nodes[2 * r + 1]) != c) continue;
            ++count;
            if (ref < 0) {
                ref = r;
                continue;
            }
            const double* pa = &Aw[(size_t)r * (CustomScheme::kDeg + 1)];
            const double* pb = &Bw[(size_t)r * (CustomScheme::kDeg + 1)];
            const double* qa = &Aw[(size_t)ref * (CustomScheme::kDeg + 1)];
            const double* qb = &Bw[(size_t)ref * (CustomScheme::kDeg + 1)];
            for (int k = 0; k <= CustomScheme::kDeg; ++k)
                if (std::fabs(pa[k] - qa[k]) > tol || std::fabs(pb[k] - qb[k]) > tol)
                    return fail(WAVE2D_EINVAL, "weights are not symmetric: node (%d, %d) differs from its class",
                                nodes[2 * r], nodes[2 * r + 1]);
        }
        if (ref < 0 || is_zero(ref)) continue;
        if (count != class_size(c))
            return fail(WAVE2D_EINVAL, "class (%d, %d) carries weight but the stencil has %d of its %d nodes", kQ[c][0],
                        kQ[c][1], count, class_size(c));
        seen[c] = true;
        std::copy(&Aw[(size_t)ref * (CustomScheme::kDeg + 1)], &Aw[(size_t)ref * (CustomScheme::kDeg + 1)] + CustomScheme::kDeg + 1, cs.a[c]);
        std::copy(&Bw[(size_t)ref * (CustomScheme::kDeg + 1)], &Bw[(size_t)ref * (CustomScheme::kDeg + 1)] + CustomScheme::kDeg + 1, cs.b[c]);
    }
    for (int c = 0; c < kWideClasses; ++c)
        for (int k = 0; k <= CustomScheme::kDeg; ++k) {
            if (std::fabs(cs.a[c][k]) <= tol) cs.a[c][k] = 0.0;
            if (std::fabs(cs.b[c][k]) <= tol) cs.b[c][k] = 0.0;
        }
    bool any = false;
    for (int c = 0; c < kWideClasses; ++c)
        for (int k = 0; k <= CustomScheme::kDeg; ++k) any = any || cs.a[c][k] != 0.0;
    if (!any) return fail(WAVE2D_EINVAL, "the scheme has no stencil weights");
    bool wide = false;
    for (int c = 3; c < kWideClasses; ++c) wide = wide || seen[c];
    cs.kind = wide ? KINDW : seen[2] ? KIND13 : (seen[1] ? KIND9 : KIND5);
    cs.lambda_max = stability_limit(cs);
    if (!(cs.lambda_max > 0.0)) return fail(WAVE2D_EINVAL, "the scheme is unstable for every Courant number");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_schemes.size() >= 256) return fail(WAVE2D_EINVAL, "too many custom schemes (256)");
    g_schemes.push_back(cs);
    *id = kCustomBase + (int)g_schemes.size() - 1;
    return WAVE2D_OK;
}

bool custom_scheme(int id, CustomScheme* out)
{
    if (id < kCustomBase) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    const size_t k = (size_t)(id - kCustomBase);
    if (k >= g_schemes.size()) return false;
    *out = g_schemes[k];
    return true;
}

}  // namespace w2d_host

// C ABI of the wave2d library: argument validation, scheme weights,
// workspace management and the launch sequences of the entry points
// declared in include/wave2d.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "host.h"

using namespace w2d;

namespace w2d_host {

thread_local std::string g_last_error;

// Largest grid side: keeps every launch grid within the hardware limits.
constexpr int64_t kMaxSide = int64_t(1) << 18;
// Row stride limit: the streaming kernels address a segment's rows through
// 32-bit buffer offsets.
constexpr int64_t kMaxLd = int64_t(1) << 22;

int fail(int status, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(WAVE2D_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}


int kind_of(int scheme)
{
    switch (scheme) {
    case WAVE2D_P5: return KIND5;
    case WAVE2D_P9: return KIND9;
    case WAVE2D_C9: return KIND9;
    case WAVE2D_P13: return KIND13;
    default: {
        CustomScheme cs;
        return custom_scheme(scheme, &cs) ? cs.kind : -1;
    }
    }
}

// Tuning slot of a scheme; schemes built by wave2d_scheme_create share the
// slot of the paper's scheme with the same stencil class.
int scheme_index(int scheme)
{
    switch (scheme) {
    case WAVE2D_P5: return 0;
    case WAVE2D_P9: return 1;
    case WAVE2D_P13: return 2;
    case WAVE2D_C9: return 3;
    default: {
        // KINDW schemes run one level per launch: no launch shape to tune.
        CustomScheme cs;
        if (!custom_scheme(scheme, &cs) || cs.kind == KINDW) return -1;
        return cs.kind == KIND5 ? 0 : cs.kind == KIND9 ? 1 : 2;
    }
    }
}

// Scheme id whose built-in defaults a scheme uses (the paper's scheme of
// the same stencil class for built schemes).
int tuning_scheme(int scheme)
{
    const int si = scheme_index(scheme);
    if (si < 0 || scheme < kCustomBase) return scheme;
    return si == 0 ? WAVE2D_P5 : si == 1 ? WAVE2D_P9 : WAVE2D_P13;
}

// Node weights of the A and B operators for one node of each class (the
// order of Params: axis at distance 1, diagonal, axis at distance 2, then
// the classes out to three lines, which only built schemes use); B divided
// by tau.
//   five-point:  A: lambda^2/2 (Sec. 6.1, eq. A6); B: lambda^2/6 (eq. B6)
//   nine-point:  A: lambda^2/2 - lambda^4/6, lambda^4/12 (eq. A11)
//                B: lambda^2/6 - lambda^4/30, lambda^4/60 (eq. B11)
//   13-point:    eq. comp13.1 expanded per node:
//                A: lambda^2 (2 - lambda^2)/3, lambda^4/12, lambda^2 (lambda^2 - 1)/24
//                B: lambda^2 (10 - 3 lambda^2)/45, lambda^4/60, lambda^2 (3 lambda^2 - 5)/360
//   isotropic:   eq. comp9.1b / comp9.2b: A: lambda^2/3, lambda^2/12; no B stencil.
// The two-step weights are twice the A weights (Sec. 3, eq. A2).
bool node_weights(int scheme, double lam, double wa[kWideClasses], double wb[kWideClasses], bool* has_b)
{
    const double l2 = lam * lam, l4 = l2 * l2;
    *has_b = true;
    for (int c = 0; c < kWideClasses; ++c) wa[c] = wb[c] = 0.0;
    switch (scheme) {
    case WAVE2D_P5:
        wa[0] = l2 / 2.0; wa[1] = 0.0; wa[2] = 0.0;
        wb[0] = l2 / 6.0; wb[1] = 0.0; wb[2] = 0.0;
        return true;
    case WAVE2D_P9:
        wa[0] = l2 / 2.0 - l4 / 6.0; wa[1] = l4 / 12.0; wa[2] = 0.0;
        wb[0] = l2 / 6.0 - l4 / 30.0; wb[1] = l4 / 60.0; wb[2] = 0.0;
        return true;
    case WAVE2D_P13:
        wa[0] = l2 * (2.0 - l2) / 3.0; wa[1] = l4 / 12.0; wa[2] = l2 * (l2 - 1.0) / 24.0;
        wb[0] = l2 * (10.0 - 3.0 * l2) / 45.0; wb[1] = l4 / 60.0; wb[2] = l2 * (3.0 * l2 - 5.0) / 360.0;
        return true;
    case WAVE2D_C9:
        wa[0] = l2 / 3.0; wa[1] = l2 / 12.0; wa[2] = 0.0;
        wb[0] = wb[1] = wb[2] = 0.0;
        *has_b = false;
        return true;
    default: {
        // Built schemes: the polynomials of the Sec. 4-5 construction.
        CustomScheme cs;
        if (!custom_scheme(scheme, &cs)) return false;
        for (int c = 0; c < kWideClasses; ++c) {
            double sa = 0.0, sb = 0.0;
            for (int k = CustomScheme::kDeg; k >= 0; --k) {
                sa = sa * lam + cs.a[c][k];
                sb = sb * lam + cs.b[c][k];
            }
            wa[c] = sa;
            wb[c] = sb;
        }
        return true;
    }
    }
}

double lambda_max_of(int scheme)
{
    switch (scheme) {
    case WAVE2D_P5: return std::sqrt(0.5);
    case WAVE2D_P9: return std::sqrt((3.0 - std::sqrt(3.0)) * 0.5);
    case WAVE2D_P13: return std::sqrt(0.5);
    case WAVE2D_C9: return std::sqrt(0.75);
    default: {
        CustomScheme cs;
        return custom_scheme(scheme, &cs) ? cs.lambda_max : -1.0;
    }
    }
}


int check_finite_pos(double v, const char* name)
{
    if (!(std::isfinite(v) && v > 0.0)) return fail(WAVE2D_EINVAL, "%s must be finite and > 0 (got %g)", name, v);
    return WAVE2D_OK;
}

int validate(int64_t nx, int64_t ny, int64_t ld, double h, double tau, double c, int scheme, uint32_t flags,
             Params* p)
{
    const uint32_t known = WAVE2D_FIRST_CONVENTIONAL | WAVE2D_ALLOW_UNSTABLE | WAVE2D_KERNEL_SIMPLE | WAVE2D_PERIODIC;
    if (flags & ~known) return fail(WAVE2D_EINVAL, "unknown flag bits 0x%x", flags & ~known);
    if (nx < 3 || ny < 3) return fail(WAVE2D_EINVAL, "grid must have at least 3 x 3 nodes (got %lld x %lld)",
                                      (long long)nx, (long long)ny);
    if (ld < nx) return fail(WAVE2D_EINVAL, "ld (%lld) < nx (%lld)", (long long)ld, (long long)nx);
    if (nx > kMaxSide || ny > kMaxSide)
        return fail(WAVE2D_EINVAL, "grid side exceeds %d nodes", kMaxSide);
    if (ld > kMaxLd) return fail(WAVE2D_EINVAL, "ld (%lld) exceeds %lld", (long long)ld, (long long)kMaxLd);
    if (ld > (int64_t(1) << 31) / ny || ld * ny >= (int64_t(1) << 31))
        return fail(WAVE2D_EINVAL, "grid too large: ld*ny must be < 2^31");
    int r;
    if ((r = check_finite_pos(h, "h")) || (r = check_finite_pos(tau, "tau")) || (r = check_finite_pos(c, "c")))
        return r;
    p->scheme = scheme;
    p->kind = kind_of(scheme);
    if (p->kind < 0) return fail(WAVE2D_EINVAL, "unknown scheme %d", scheme);
    p->g = Grid{(int)nx, (int)ny, (int)ld, (flags & WAVE2D_PERIODIC) ? 1 : 0};
    if (p->g.periodic) {
        const int rr = radius_of_kind(p->kind);
        if (nx < 2 * rr + 1 || ny < 2 * rr + 1)
            return fail(WAVE2D_EINVAL, "periodic grids need at least %d x %d nodes for scheme %d", 2 * rr + 1,
                        2 * rr + 1, scheme);
    }
    p->lam = c * tau / h;
    const double lmax = lambda_max_of(scheme);
    if (!(flags & WAVE2D_ALLOW_UNSTABLE) && p->lam > lmax * (1.0 + 1e-12))
        return fail(WAVE2D_EUNSTABLE, "Courant number %.17g exceeds the stability limit %.17g of scheme %d",
                    p->lam, lmax, scheme);
    node_weights(scheme, p->lam, p->wa, p->wb, &p->has_b);
    return WAVE2D_OK;
}

// Periodic grids run the temporally blocked kernels only when no lane's
// column pair straddles the wrap (even nx) and the whole grid fits one
// buffer range; other periodic grids use the one-node-per-thread kernels.
bool stream_ok(const Grid& g, size_t elt)
{
    if (!g.periodic) return true;
    return (g.nx % 2 == 0) && (uint64_t)g.ld * (uint64_t)g.ny * elt < (uint64_t(1) << 31);
}

StepW64 step_w64(const Params& p)
{
    return StepW64{2.0 * p.wa[0], 2.0 * p.wa[1], 2.0 * p.wa[2], 2.0 * p.wa[0] + 4.0 * p.wa[1] + 8.0 * p.wa[2]};
}

StepW32 step_w32(const Params& p)
{
    StepW32 w;
    w.w10 = (float)(2.0 * p.wa[0]);
    w.w11 = (float)(2.0 * p.wa[1]);
    w.w20 = (float)(2.0 * p.wa[2]);
    w.wc = -4.0f * (w.w10 + w.w11 + w.w20);
    const double wx = 2.0 * p.wa[0] + 4.0 * p.wa[1] + 8.0 * p.wa[2];
    w.wx = (float)wx;
    w.wxl = (float)(wx - (double)w.wx);
    return w;
}

int radius_of_kind(int kind) { return kind == KINDW ? 3 : kind == KIND13 ? 2 : 1; }

WideW64 wide_w64(const Params& p)
{
    WideW64 w;
    for (int c = 0; c < kWideClasses; ++c) w.w[c] = 2.0 * p.wa[c];
    return w;
}

WideW32 wide_w32(const Params& p)
{
    WideW32 w;
    for (int c = 0; c < kWideClasses; ++c) {
        const double x = 2.0 * p.wa[c];
        w.w[c] = (float)x;
        w.wl[c] = (float)(x - (double)w.w[c]);
    }
    return w;
}

WideFirstW wide_first_w(const Params& p, uint32_t flags, double tau)
{
    WideFirstW w;
    for (int c = 0; c < kWideClasses; ++c) {
        w.a[c] = p.wa[c];
        w.b[c] = p.wb[c];
    }
    w.tau = tau;
    w.poisson = (p.has_b && !(flags & WAVE2D_FIRST_CONVENTIONAL)) ? 1 : 0;
    return w;
}

FirstW first_w(const Params& p, uint32_t flags, double tau)
{
    FirstW w;
    w.a10 = p.wa[0]; w.a11 = p.wa[1]; w.a20 = p.wa[2];
    w.b10 = p.wb[0]; w.b11 = p.wb[1]; w.b20 = p.wb[2];
    w.tau = tau;
    w.poisson = (p.has_b && !(flags & WAVE2D_FIRST_CONVENTIONAL)) ? 1 : 0;
    return w;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

size_t grid_bytes(const Grid& g, size_t elt) { return ((size_t)g.ld * (g.ny - 1) + g.nx) * elt; }

int check_ptrs(const Grid& g, std::initializer_list<std::pair<const void*, size_t>> arrs)
{
    std::vector<std::pair<const void*, size_t>> v(arrs);
    for (size_t i = 0; i < v.size(); ++i) {
        if (!v[i].first) return fail(WAVE2D_EINVAL, "array argument %zu is NULL", i);
        for (size_t k = 0; k < i; ++k)
            if (overlap(v[i].first, grid_bytes(g, v[i].second), v[k].first, grid_bytes(g, v[k].second)))
                return fail(WAVE2D_EINVAL, "array arguments %zu and %zu overlap", k, i);
    }
    return WAVE2D_OK;
}

// ---- tuning --------------------------------------------------------------------

std::mutex g_tune_mu;
struct TuneEntry {
    bool set;
    wave2d_tuning t;
};
TuneEntry g_tune[2][4] = {};

// Default segment height for a grid.  A pass costs about rows + 2 R depth
// phases per work item (the item recomputes R depth rows of its neighbours
// above and below) and its items run in rounds of the device's resident
// wave slots.  Heights are chosen so the items fill about 1.5 rounds when
// three or more waves share a SIMD (a half-full last round still keeps
// 1.5 waves per SIMD issuing) and 2 rounds with fewer, within
// [max(8, 2 R depth), 64] rows.  Measured on MI355X, compensated 9-point,
// depth 6 (3 waves per SIMD): 4097^2 best at 30-32 rows (1.5-1.6 rounds;
// 694 GLUP/s in one round, 793 in two), 2049^2 best at 12-16 rows, 8193^2
// at 48-64.
int fill_rows(int precision, int kind, int depth, int64_t nx, int64_t ny)
{
    const ShapeFit f = stream_shape_fit(precision, kind, depth);
    if (f.slots < 1 || f.strip_cols < 1) return 32;
    const int64_t nstrips = (nx + f.strip_cols - 1) / f.strip_cols;
    const int64_t lo = std::max(8, 2 * f.halo_rows);
    if (f.simd_waves >= 3) {
        const int64_t segs = std::max<int64_t>(1, (int64_t)(1.5 * f.slots) / nstrips);
        const int64_t r = (ny + segs - 1) / segs;
        return (int)std::min<int64_t>(64, std::max<int64_t>(lo, r));
    }
    // Two waves per SIMD: the longest segments whose work items fill a
    // whole number of rounds of the resident waves (a launch takes
    // ceil(items / slots) item times, and longer segments recompute fewer
    // warm-up rows).  Measured on 4097^2: one round (75 rows) beats two
    // (38) by 3-7% for the compensated 5- and 9-point kernels and the
    // double-precision 9-point one (its 5-point kernel prefers two rounds),
    // and for the 13-point kernels 81 rows (one round) beats 44 (1.8
    // rounds) by 4-11%.  Very tall segments lose again: on 6001^2 the
    // compensated 9-point kernel ran 4% slower at 163 rows (one round) than
    // at 82 (two), hence the cap.
    constexpr int64_t kMaxRows = 128;
    for (int64_t k = 1; k <= 64; ++k) {
        const int64_t segs = k * f.slots / nstrips;
        if (segs < 1) continue;
        const int64_t r = (ny + segs - 1) / segs;
        if (r <= kMaxRows) return (int)std::max(lo, r);
    }
    return (int)std::max<int64_t>(lo, 64);
}

// Shapes measured fastest on MI355X (256 CUs) for the grid sizes of the
// standard workloads: sweeps of depth and of every segment height near the
// best, repeated (the height of the last, partial segment of a column
// makes neighbouring heights differ by up to 10%), per-pass rates of
// back-to-back passes (one launch each) after an untimed warm-up.  Used only on devices with the same CU count.
struct MeasuredShape {
    int precision, scheme;
    int64_t nx, ny;
    wave2d_tuning t;
};
const MeasuredShape kMeasured[] = {
    {WAVE2D_F32C, WAVE2D_P9, 4097, 4097, {8, 75}},    // 938 GLUP/s per pass (38 rows: 906)
    {WAVE2D_F32C, WAVE2D_P9, 8193, 8193, {8, 100}},   // 1121 (68 rows: 1070)
    {WAVE2D_F32C, WAVE2D_P9, 2049, 2049, {6, 19}},    // 654 (20 rows: 625)
    {WAVE2D_F32C, WAVE2D_P5, 4097, 4097, {8, 75}},    // 975 (40 rows: 911)
    {WAVE2D_F32C, WAVE2D_P13, 4097, 4097, {6, 81}},   // 612 (44 rows: 551)
    {WAVE2D_F32C, WAVE2D_P13, 8193, 8193, {6, 161}},  // 796 (112 rows: 771)
    {WAVE2D_F64, WAVE2D_P9, 4097, 4097, {8, 75}},     // 890 (40 rows: 848)
    {WAVE2D_F64, WAVE2D_P5, 4097, 4097, {8, 38}},     // 966 (75 rows: 918)
    {WAVE2D_F64, WAVE2D_P9, 8193, 8193, {8, 149}},    // 1028 (100 rows: 1005)
    {WAVE2D_F64, WAVE2D_P5, 8193, 8193, {8, 149}},    // 1056 (100 rows: 1044)
    {WAVE2D_F64, WAVE2D_P13, 4097, 4097, {6, 81}},    // 548 (56 rows: 528)
    {WAVE2D_F64, WAVE2D_P13, 8193, 8193, {6, 161}},   // 696 (128 rows: 662)
    {WAVE2D_F64, WAVE2D_P13, 2049, 2049, {4, 20}},    // 337 (24 rows: 303)
};

int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 0;
    (void)hipGetLastError();
    return cus;
}

// Depths measured fastest on MI355X (depth x rows sweeps of the streaming
// kernels on 2049^2 to 8193^2 grids); overridable per process.  Without a
// grid size the height is 8, the least segment height batched launches
// start from.
wave2d_tuning default_tuning(int precision, int scheme_in, int64_t nx, int64_t ny)
{
    const int scheme = tuning_scheme(scheme_in);
    for (const MeasuredShape& m : kMeasured)
        if (m.precision == precision && m.scheme == scheme && m.nx == nx && m.ny == ny && device_cus() == 256)
            return m.t;
    // The double-precision 13-point kernel at depth 6 holds 254 VGPRs (two
    // waves per SIMD, as at depth 4); the deeper pass pays off once the grid
    // gives every SIMD several segments (measured: 4097^2 and 8193^2 faster
    // at depth 6, 2049^2 at depth 4).
    int depth;
    if (precision == WAVE2D_F32C) depth = (scheme == WAVE2D_P13) ? 6 : 8;
    else if (scheme == WAVE2D_P13) depth = (nx * ny >= (int64_t(1) << 23)) ? 6 : 4;
    else depth = 8;
    const int rows = (nx > 0 && ny > 0) ? fill_rows(precision, kind_of(scheme), depth, nx, ny) : 8;
    return wave2d_tuning{depth, rows};
}

// Shapes the autotuner measured for particular grid sizes.
std::map<std::tuple<int, int, int64_t, int64_t>, wave2d_tuning> g_tune_size;

void set_tuning_entry(int precision, int scheme, const wave2d_tuning& t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const int si = scheme_index(scheme);
    if (si < 0) return;
    g_tune[precision][si].set = true;
    g_tune[precision][si].t = t;
}

void set_tuning_size_entry(int precision, int scheme, int64_t nx, int64_t ny, const wave2d_tuning& t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_size[std::make_tuple(precision, scheme, nx, ny)] = t;
}

// Shapes kept across processes: with WAVE2D_TUNE_CACHE naming a file, each
// line "precision scheme nx ny depth rows" is loaded before the first
// lookup, and every autotuned shape is appended.  Lines that do not parse,
// unknown or run-time-built schemes and unsupported shapes are skipped.
std::once_flag g_cache_once;

bool cacheable(int precision, int scheme, const wave2d_tuning& t)
{
    const bool paper = scheme == WAVE2D_P5 || scheme == WAVE2D_P9 || scheme == WAVE2D_P13 || scheme == WAVE2D_C9;
    return (precision == WAVE2D_F64 || precision == WAVE2D_F32C) && paper && stream_depth_supported(t.depth) &&
           t.rows >= 1;
}

void load_tune_cache()
{
    const char* path = std::getenv("WAVE2D_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        int prec, scheme, depth, rows;
        long long nx, ny;
        if (std::sscanf(line, "%d %d %lld %lld %d %d", &prec, &scheme, &nx, &ny, &depth, &rows) != 6) continue;
        const wave2d_tuning t{depth, rows};
        if (nx < 3 || ny < 3 || !cacheable(prec, scheme, t)) continue;
        set_tuning_size_entry(prec, scheme, nx, ny, t);
    }
    std::fclose(f);
}

void save_tune_cache(int precision, int scheme, int64_t nx, int64_t ny, const wave2d_tuning& t)
{
    const char* path = std::getenv("WAVE2D_TUNE_CACHE");
    if (!path || !*path || !cacheable(precision, scheme, t)) return;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%d %d %lld %lld %d %d\n", precision, scheme, (long long)nx, (long long)ny, t.depth, t.rows);
    std::fclose(f);
}

wave2d_tuning tuning_for(int precision, int scheme, int64_t nx, int64_t ny)
{
    std::call_once(g_cache_once, load_tune_cache);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_size.find(std::make_tuple(precision, scheme, nx, ny));
    if (it != g_tune_size.end()) return it->second;
    const int si = scheme_index(scheme);
    if (si >= 0 && g_tune[precision][si].set) return g_tune[precision][si].t;
    return default_tuning(precision, scheme, nx, ny);
}

// ---- library-owned device buffers ---------------------------------------------

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_buf_mu;
std::map<std::pair<int, hipStream_t>, DevBuf> g_work;  // per (device, stream)
std::map<int, DevBuf> g_part;                          // norms partials per device
std::map<std::pair<int, hipStream_t>, Fork> g_fork;    // side stream per (device, stream)
std::map<int, double*> g_host;                         // pinned host results per device

int get_device(int* dev)
{
    W2D_HIP(hipGetDevice(dev));
    return WAVE2D_OK;
}

int library_work(hipStream_t s, size_t need, void** out)
{
    int dev, r;
    if ((r = get_device(&dev))) return r;
    std::lock_guard<std::mutex> lk(g_buf_mu);
    DevBuf& b = g_work[{dev, s}];
    if (b.bytes < need) {
        if (b.ptr) {
            // Earlier calls on this stream may still use the old buffer.
            W2D_HIP(hipStreamSynchronize(s));
            W2D_HIP(hipFree(b.ptr));
            b.ptr = nullptr;
            b.bytes = 0;
        }
        hipError_t e = hipMalloc(&b.ptr, need);
        if (e != hipSuccess) {
            b.ptr = nullptr;
            (void)hipGetLastError();
            return fail(WAVE2D_ENOMEM, "workspace of %zu bytes: %s", need, hipGetErrorString(e));
        }
        b.bytes = need;
    }
    *out = b.ptr;
    return WAVE2D_OK;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Side stream and fork/join events for the boundary-strip kernels of calls
// on stream s (default priority, created on first use).
int side_of(hipStream_t s, const Fork** out)
{
    int dev, r;
    if ((r = get_device(&dev))) return r;
    std::lock_guard<std::mutex> lk(g_buf_mu);
    auto it = g_fork.find({dev, s});
    if (it == g_fork.end()) {
        Fork f{};
        W2D_HIP(hipStreamCreateWithFlags(&f.side, hipStreamNonBlocking));
        W2D_HIP(hipEventCreateWithFlags(&f.ev_fork, hipEventDisableTiming));
        W2D_HIP(hipEventCreateWithFlags(&f.ev_join, hipEventDisableTiming));
        it = g_fork.emplace(std::make_pair(dev, s), f).first;
    }
    *out = &it->second;
    return WAVE2D_OK;
}

size_t work_bytes_of(int precision, const Grid& g)
{
    const size_t n = (size_t)g.ld * g.ny;
    if (precision == WAVE2D_F64) return 2 * align256(n * sizeof(double));
    return 3 * align256(n * sizeof(float));
}

int resolve_work(int precision, const Grid& g, void* work, size_t work_bytes, hipStream_t s, char** base)
{
    const size_t need = work_bytes_of(precision, g);
    if (work) {
        if (work_bytes < need)
            return fail(WAVE2D_EINVAL, "workspace too small: %zu < %zu bytes", work_bytes, need);
        *base = (char*)work;
        return WAVE2D_OK;
    }
    void* p;
    int r = library_work(s, need, &p);
    if (r) return r;
    *base = (char*)p;
    return WAVE2D_OK;
}

// Depths of consecutive passes for `steps` levels at most `depth` per pass,
// using only supported depths; the count is made even when possible so that
// a ping-pong sequence ends in the caller's buffers.
std::vector<int> plan_passes(int64_t steps, int depth, bool* needs_copy)
{
    std::vector<int> v;
    if (!stream_depth_supported(depth)) depth = 1;
    int64_t left = steps;
    while (left >= depth) {
        v.push_back(depth);
        left -= depth;
    }
    static const int sup[] = {8, 6, 4, 3, 2, 1};
    while (left > 0) {
        for (int d : sup)
            if (d <= left && stream_depth_supported(d)) {
                v.push_back(d);
                left -= d;
                break;
            }
    }
    *needs_copy = false;
    if (v.size() % 2 == 1) {
        // Split one pass of depth >= 2 into two supported depths.
        bool split = false;
        for (size_t k = v.size(); k-- > 0;) {
            const int d = v[k];
            if (d < 2) continue;
            int a = d / 2, b = d - d / 2;
            if (!stream_depth_supported(a) || !stream_depth_supported(b)) continue;
            v[k] = a;
            v.insert(v.begin() + k + 1, b);
            split = true;
            break;
        }
        if (!split) *needs_copy = true;
    }
    return v;
}

// ---- pass sequences ----------------------------------------------------------

// FP64: (up, uc) = (u^{k-1}, u^k) -> (u^{k+steps-1}, u^{k+steps}) in place.
int run_steps_f64(const Params& p, uint32_t flags, int64_t steps, double* up, double* uc, void* work,
                  size_t work_bytes, hipStream_t s)
{
    if (steps == 0) return WAVE2D_OK;
    const Grid& g = p.g;
    if (p.kind == KINDW) {
        // One level per launch, in place: level k+1 overwrites level k-1.
        const WideW64 ww = wide_w64(p);
        double* a = up;
        double* b = uc;
        for (int64_t k = 0; k < steps; ++k) {
            W2D_HIP(wide_step_f64(g, ww, a, b, a, s));
            std::swap(a, b);
        }
        if (steps % 2) W2D_HIP(swap_f64(g, up, uc, s));
        return WAVE2D_OK;
    }
    const StepW64 w = step_w64(p);
    const wave2d_tuning tn = tuning_for(WAVE2D_F64, p.scheme, g.nx, g.ny);
    const bool simple = (flags & WAVE2D_KERNEL_SIMPLE) || !stream_ok(g, sizeof(double));
    if (simple || tn.depth == 1 || steps == 1) {
        // In place: level k+1 overwrites level k-1, then the roles swap.
        double* a = up;
        double* b = uc;
        const StreamShape sh{1, tn.rows};
        for (int64_t k = 0; k < steps; ++k) {
            if (simple) W2D_HIP(simple_step_f64(g, p.kind, w, a, b, a, s));
            else W2D_HIP(stream_step_f64(g, p.kind, w, sh, a, b, a, nullptr, s));
            std::swap(a, b);
        }
        if (steps % 2) W2D_HIP(swap_f64(g, up, uc, s));
        return WAVE2D_OK;
    }
    char* base;
    int r = resolve_work(WAVE2D_F64, g, work, work_bytes, s, &base);
    if (r) return r;
    const size_t stride = align256((size_t)g.ld * g.ny * sizeof(double));
    double* wp = (double*)base;
    double* wc = (double*)(base + stride);
    bool needs_copy;
    const std::vector<int> passes = plan_passes(steps, tn.depth, &needs_copy);
    double *ip = up, *ic = uc, *op = wp, *oc = wc;
    for (int d : passes) {
        const StreamShape sh{d, tn.rows};
        W2D_HIP(stream_step_f64(g, p.kind, w, sh, ip, ic, op, oc, s));
        std::swap(ip, op);
        std::swap(ic, oc);
    }
    if (ip != up) W2D_HIP(copy_f64x2(g, ip, ic, up, uc, s));
    return WAVE2D_OK;
}

// Compensated FP32: state (u, lo, d) advanced `steps` levels in place.
int run_steps_f32c(const Params& p, uint32_t flags, int64_t steps, float* u, float* lo, float* d, void* work,
                   size_t work_bytes, hipStream_t s)
{
    if (steps == 0) return WAVE2D_OK;
    const StepW32 w = step_w32(p);
    const Grid& g = p.g;
    char* base;
    int r = resolve_work(WAVE2D_F32C, g, work, work_bytes, s, &base);
    if (r) return r;
    const size_t stride = align256((size_t)g.ld * g.ny * sizeof(float));
    float* wu = (float*)base;
    float* wl = (float*)(base + stride);
    float* wd = (float*)(base + 2 * stride);
    if (p.kind == KINDW) {
        const WideW32 ww = wide_w32(p);
        float *iu = u, *il = lo, *id = d, *ou = wu, *ol = wl, *od = wd;
        for (int64_t k = 0; k < steps; ++k) {
            W2D_HIP(wide_step_f32c(g, ww, iu, il, id, ou, ol, od, s));
            std::swap(iu, ou);
            std::swap(il, ol);
            std::swap(id, od);
        }
        if (iu != u) W2D_HIP(copy_f32x3(g, iu, il, id, u, lo, d, s));
        return WAVE2D_OK;
    }
    const bool simple = (flags & WAVE2D_KERNEL_SIMPLE) || !stream_ok(g, sizeof(float));
    const wave2d_tuning tn = tuning_for(WAVE2D_F32C, p.scheme, g.nx, g.ny);
    bool needs_copy = false;
    std::vector<int> passes;
    if (simple) passes.assign((size_t)steps, 1);
    else passes = plan_passes(steps, tn.depth, &needs_copy);
    float *iu = u, *il = lo, *id = d, *ou = wu, *ol = wl, *od = wd;
    for (int dd : passes) {
        if (simple) W2D_HIP(simple_step_f32c(g, p.kind, w, iu, il, id, ou, ol, od, s));
        else W2D_HIP(stream_step_f32c(g, p.kind, w, StreamShape{dd, tn.rows}, iu, il, id, ou, ol, od, s));
        std::swap(iu, ou);
        std::swap(il, ol);
        std::swap(id, od);
    }
    if (iu != u) W2D_HIP(copy_f32x3(g, iu, il, id, u, lo, d, s));
    return WAVE2D_OK;
}

// FP64 first step (eq. A1) with the kernels of the scheme's class.
int first_step_any(const Params& p, uint32_t flags, double tau, const double* u0, const double* v0, double* u1,
                   hipStream_t s)
{
    if (p.kind == KINDW) W2D_HIP(wide_first_step(p.g, wide_first_w(p, flags, tau), u0, v0, u1, s));
    else W2D_HIP(simple_first_step(p.g, p.kind, first_w(p, flags, tau), u0, v0, u1, s));
    return WAVE2D_OK;
}

struct HostSlot {
    double* part;
    double* host;
};

int norm_slot(hipStream_t, HostSlot* hs)
{
    int dev, r;
    if ((r = get_device(&dev))) return r;
    std::lock_guard<std::mutex> lk(g_buf_mu);
    DevBuf& b = g_part[dev];
    const size_t need = (size_t)(norms_blocks() + 1) * 4 * sizeof(double);
    if (!b.ptr) {
        hipError_t e = hipMalloc(&b.ptr, need);
        if (e != hipSuccess) {
            b.ptr = nullptr;
            (void)hipGetLastError();
            return fail(WAVE2D_ENOMEM, "norm scratch: %s", hipGetErrorString(e));
        }
        b.bytes = need;
    }
    double*& h = g_host[dev];
    if (!h) {
        hipError_t e = hipHostMalloc((void**)&h, 4 * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) {
            h = nullptr;
            (void)hipGetLastError();
            return fail(WAVE2D_ENOMEM, "pinned host buffer: %s", hipGetErrorString(e));
        }
    }
    hs->part = (double*)b.ptr;
    hs->host = h;
    return WAVE2D_OK;
}

std::mutex g_norm_mu;  // the per-device norm scratch is shared by all streams

int check_grid_only(int64_t nx, int64_t ny, int64_t ld, Grid* g)
{
    if (nx < 1 || ny < 1) return fail(WAVE2D_EINVAL, "empty grid");
    if (nx > kMaxSide || ny > kMaxSide) return fail(WAVE2D_EINVAL, "grid side exceeds %d nodes", kMaxSide);
    if (ld < nx) return fail(WAVE2D_EINVAL, "ld (%lld) < nx (%lld)", (long long)ld, (long long)nx);
    if (ld > kMaxLd) return fail(WAVE2D_EINVAL, "ld (%lld) exceeds %lld", (long long)ld, (long long)kMaxLd);
    if (ld * ny >= (int64_t(1) << 31)) return fail(WAVE2D_EINVAL, "grid too large: ld*ny must be < 2^31");
    *g = Grid{(int)nx, (int)ny, (int)ld};
    return WAVE2D_OK;
}

}  // namespace w2d_host

using namespace w2d_host;

// ======================= exported entry points =================================

extern "C" {

double wave2d_lambda_max(int scheme) { return lambda_max_of(scheme); }

int wave2d_scheme_create(int32_t m, const int32_t* nodes, const int32_t* exps, int* scheme)
{
    return custom_scheme_create(m, nodes, exps, scheme);
}

int wave2d_class_weights(int scheme, uint32_t flags, double lambda, int32_t nclass, double* w2, double* wa,
                         double* wb)
{
    double a[kWideClasses], b[kWideClasses];
    bool hb;
    if (!(std::isfinite(lambda) && lambda >= 0.0)) return fail(WAVE2D_EINVAL, "lambda must be finite and >= 0");
    if (nclass < 1 || nclass > kWideClasses) return fail(WAVE2D_EINVAL, "nclass must be in [1, %d]", kWideClasses);
    if (!node_weights(scheme, lambda, a, b, &hb)) return fail(WAVE2D_EINVAL, "unknown scheme %d", scheme);
    for (int q = nclass; q < kWideClasses; ++q)
        if (a[q] != 0.0 || b[q] != 0.0)
            return fail(WAVE2D_EINVAL, "scheme %d has weight in class %d, beyond the %d requested", scheme, q, nclass);
    const bool poisson = hb && !(flags & WAVE2D_FIRST_CONVENTIONAL);
    for (int q = 0; q < nclass; ++q) {
        if (w2) w2[q] = 2.0 * a[q];
        if (wa) wa[q] = a[q];
        if (wb) wb[q] = poisson ? b[q] : 0.0;
    }
    return WAVE2D_OK;
}

int wave2d_weights(int scheme, uint32_t flags, double lambda, double w2[3], double wa[3], double wb[3])
{
    return wave2d_class_weights(scheme, flags, lambda, 3, w2, wa, wb);
}

const char* wave2d_status_str(int status)
{
    switch (status) {
    case WAVE2D_OK: return "WAVE2D_OK";
    case WAVE2D_EINVAL: return "WAVE2D_EINVAL";
    case WAVE2D_EUNSTABLE: return "WAVE2D_EUNSTABLE";
    case WAVE2D_ENOMEM: return "WAVE2D_ENOMEM";
    case WAVE2D_EDEVICE: return "WAVE2D_EDEVICE";
    case WAVE2D_EBUSY: return "WAVE2D_EBUSY";
    case WAVE2D_ENOTFOUND: return "WAVE2D_ENOTFOUND";
    default: return "WAVE2D_UNKNOWN";
    }
}

const char* wave2d_last_error(void) { return g_last_error.c_str(); }

size_t wave2d_work_bytes(int precision, int64_t nx, int64_t ny, int64_t ld)
{
    if ((precision != WAVE2D_F64 && precision != WAVE2D_F32C) || nx < 1 || ny < 1 || ld < nx) return 0;
    return work_bytes_of(precision, Grid{(int)nx, (int)ny, (int)ld});
}

int wave2d_first_step(int64_t nx, int64_t ny, int64_t ld, double h, double tau, double c, int scheme,
                      uint32_t flags, const double* u0, const double* v0, double* u1, void* stream)
{
    Params p;
    int r = validate(nx, ny, ld, h, tau, c, scheme, flags, &p);
    if (r) return r;
    if ((r = check_ptrs(p.g, {{u0, 8}, {v0, 8}, {u1, 8}}))) return r;
    return first_step_any(p, flags, tau, u0, v0, u1, (hipStream_t)stream);
}

int wave2d_step(int64_t nx, int64_t ny, int64_t ld, double h, double tau, double c, int scheme, uint32_t flags,
                int64_t steps, double* u_prev, double* u_cur, void* work, size_t work_bytes, void* stream)
{
    Params p;
    int r = validate(nx, ny, ld, h, tau, c, scheme, flags, &p);
    if (r) return r;
    if (steps < 0) return fail(WAVE2D_EINVAL, "steps must be >= 0");
    if ((r = check_ptrs(p.g, {{u_prev, 8}, {u_cur, 8}}))) return r;
    return run_steps_f64(p, flags, steps, u_prev, u_cur, work, work_bytes, (hipStream_t)stream);
}

int wave2d_run(int64_t nx, int64_t ny, int64_t ld, double h, double tau, double c, int scheme, uint32_t flags,
               int64_t steps, const double* u0, const double* v0, double* u_prev_out, double* u_out, void* work,
               size_t work_bytes, void* stream)
{
    Params p;
    int r = validate(nx, ny, ld, h, tau, c, scheme, flags, &p);
    if (r) return r;
    if (steps < 1) return fail(WAVE2D_EINVAL, "steps must be >= 1");
    if ((r = check_ptrs(p.g, {{u0, 8}, {v0, 8}, {u_prev_out, 8}, {u_out, 8}}))) return r;
    hipStream_t s = (hipStream_t)stream;
    W2D_HIP(copy_interior_f64(p.g, u0, u_prev_out, s));
    if ((r = first_step_any(p, flags, tau, u0, v0, u_out, s))) return r;
    return run_steps_f64(p, flags, steps - 1, u_prev_out, u_out, work, work_bytes, s);
}

int wave2d_f32c_init(int64_t nx, int64_t ny, int64_t ld, const double* u_prev, const double* u_cur, float* u,
                     float* lo, float* d, void* stream)
{
    Grid g;
    int r = check_grid_only(nx, ny, ld, &g);
    if (r) return r;
    if ((r = check_ptrs(g, {{u_prev, 8}, {u_cur, 8}, {u, 4}, {lo, 4}, {d, 4}}))) return r;
    W2D_HIP(f32c_init(g, u_prev, u_cur, u, lo, d, (hipStream_t)stream));
    return WAVE2D_OK;
}

int wave2d_f32c_step(int64_t nx, int64_t ny, int64_t ld, double h, double tau, double c, int scheme,
                     uint32_t flags, int64_t steps, float* u, float* lo, float* d, void* work, size_t work_bytes,
                     void* stream)
{
    Params p;
    int r = validate(nx, ny, ld, h, tau, c, scheme, flags, &p);
    if (r) return r;
    if (steps < 0) return fail(WAVE2D_EINVAL, "steps must be >= 0");
    if ((r = check_ptrs(p.g, {{u, 4}, {lo, 4}, {d, 4}}))) return r;
    return run_steps_f32c(p, flags, steps, u, lo, d, work, work_bytes, (hipStream_t)stream);
}

int wave2d_f32c_export(int64_t nx, int64_t ny, int64_t ld, const float* u, const float* lo, double* out,
                       void* stream)
{
    Grid g;
    int r = check_grid_only(nx, ny, ld, &g);
    if (r) return r;
    if ((r = check_ptrs(g, {{u, 4}, {lo, 4}, {out, 8}}))) return r;
    W2D_HIP(f32c_export(g, u, lo, out, (hipStream_t)stream));
    return WAVE2D_OK;
}

int wave2d_f32c_run(int64_t nx, int64_t ny, int64_t ld, double h, double tau, double c, int scheme,
                    uint32_t flags, int64_t steps, const double* u0, const double* v0, float* u, float* lo,
                    float* d, void* work, size_t work_bytes, void* stream)
{
    Params p;
    int r = validate(nx, ny, ld, h, tau, c, scheme, flags, &p);
    if (r) return r;
    if (steps < 1) return fail(WAVE2D_EINVAL, "steps must be >= 1");
    if ((r = check_ptrs(p.g, {{u0, 8}, {v0, 8}, {u, 4}, {lo, 4}, {d, 4}}))) return r;
    hipStream_t s = (hipStream_t)stream;
    if (p.kind == KINDW) W2D_HIP(wide_first_step_f32c(p.g, wide_first_w(p, flags, tau), u0, v0, u, lo, d, s));
    else W2D_HIP(simple_first_step_f32c(p.g, p.kind, first_w(p, flags, tau), u0, v0, u, lo, d, s));
    return run_steps_f32c(p, flags, steps - 1, u, lo, d, work, work_bytes, s);
}

int wave2d_norms(int64_t nx, int64_t ny, int64_t ld, const double* a, const double* b, double out[4],
                 void* stream)
{
    Grid g;
    int r = check_grid_only(nx, ny, ld, &g);
    if (r) return r;
    if (!out) return fail(WAVE2D_EINVAL, "out is NULL");
    if (!a || !b) return fail(WAVE2D_EINVAL, "array argument is NULL");
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_norm_mu);
    HostSlot hs;
    if ((r = norm_slot(s, &hs))) return r;
    W2D_HIP(norms_f64(g, a, b, hs.part, s));
    W2D_HIP(hipMemcpyAsync(hs.host, hs.part + 4 * norms_blocks(), 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    W2D_HIP(hipStreamSynchronize(s));
    memcpy(out, hs.host, 4 * sizeof(double));
    return WAVE2D_OK;
}

int wave2d_f32c_norms(int64_t nx, int64_t ny, int64_t ld, const float* u, const float* lo, const double* b,
                      double out[4], void* stream)
{
    Grid g;
    int r = check_grid_only(nx, ny, ld, &g);
    if (r) return r;
    if (!out) return fail(WAVE2D_EINVAL, "out is NULL");
    if (!u || !lo || !b) return fail(WAVE2D_EINVAL, "array argument is NULL");
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_norm_mu);
    HostSlot hs;
    if ((r = norm_slot(s, &hs))) return r;
    W2D_HIP(norms_f32c(g, u, lo, b, hs.part, s));
    W2D_HIP(hipMemcpyAsync(hs.host, hs.part + 4 * norms_blocks(), 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    W2D_HIP(hipStreamSynchronize(s));
    memcpy(out, hs.host, 4 * sizeof(double));
    return WAVE2D_OK;
}

int wave2d_set_tuning(int precision, int scheme, const wave2d_tuning* t)
{
    if (precision != WAVE2D_F64 && precision != WAVE2D_F32C) return fail(WAVE2D_EINVAL, "unknown precision");
    if (kind_of(scheme) == KINDW) return fail(WAVE2D_EINVAL, "scheme %d runs one level per launch: no tuning", scheme);
    const int si = scheme_index(scheme);
    if (si < 0) return fail(WAVE2D_EINVAL, "unknown scheme %d", scheme);
    if (t) {
        if (!stream_depth_supported(t->depth)) return fail(WAVE2D_EINVAL, "unsupported depth %d", t->depth);
        if (t->rows < 1) return fail(WAVE2D_EINVAL, "rows must be >= 1");
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[precision][si].set = (t != nullptr);
    if (t) g_tune[precision][si].t = *t;
    // An override or reset applies to every grid size.
    for (auto it = g_tune_size.begin(); it != g_tune_size.end();) {
        if (std::get<0>(it->first) == precision && std::get<1>(it->first) == scheme) it = g_tune_size.erase(it);
        else ++it;
    }
    return WAVE2D_OK;
}

int wave2d_get_tuning(int precision, int scheme, int64_t nx, int64_t ny, wave2d_tuning* t)
{
    if (precision != WAVE2D_F64 && precision != WAVE2D_F32C) return fail(WAVE2D_EINVAL, "unknown precision");
    if (kind_of(scheme) == KINDW) return fail(WAVE2D_EINVAL, "scheme %d runs one level per launch: no tuning", scheme);
    if (scheme_index(scheme) < 0) return fail(WAVE2D_EINVAL, "unknown scheme %d", scheme);
    if (!t) return fail(WAVE2D_EINVAL, "t is NULL");
    *t = tuning_for(precision, scheme, nx, ny);
    return WAVE2D_OK;
}

int wave2d_release(void)
{
    std::lock_guard<std::mutex> lk(g_buf_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_work) {
        if (kv.second.ptr) {
            (void)hipSetDevice(kv.first.first);
            (void)hipFree(kv.second.ptr);
        }
    }
    g_work.clear();
    for (auto& kv : g_part) {
        if (kv.second.ptr) {
            (void)hipSetDevice(kv.first);
            (void)hipFree(kv.second.ptr);
        }
    }
    g_part.clear();
    for (auto& kv : g_fork) {
        (void)hipSetDevice(kv.first.first);
        (void)hipStreamSynchronize(kv.second.side);
        (void)hipStreamDestroy(kv.second.side);
        (void)hipEventDestroy(kv.second.ev_fork);
        (void)hipEventDestroy(kv.second.ev_join);
    }
    g_fork.clear();
    for (auto& kv : g_host)
        if (kv.second) (void)hipHostFree(kv.second);
    g_host.clear();
    (void)hipSetDevice(cur);
    return WAVE2D_OK;
}

}  // extern "C"

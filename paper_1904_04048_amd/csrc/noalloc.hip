// Allocation-free variant of wave2d_f32c_step for callers that cannot
// allocate device memory (code under stream capture, tight serving loops).
//
// The second state the multi-pass sequence ping-pongs through lives in a
// fixed device array of this file (kNoAllocBytes) instead of a library or
// caller buffer.  Its device address is looked up once per device and kept;
// the name `scratch` itself is a host-side stand-in and is never passed to
// a kernel.  Nothing here calls hipMalloc or hipFree.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host.h"

namespace {

constexpr size_t kNoAllocBytes = WAVE2D_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the
// first call made with that device current).
int scratch_ptr(void** out)
{
    int dev = 0, r;
    if ((r = w2d_host::get_device(&dev))) return r;
    if (dev < 0 || dev >= kMaxDevices) return w2d_host::fail(WAVE2D_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return w2d_host::hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return WAVE2D_OK;
}

}  // namespace

extern "C" {

int wave2d_f32c_step_noalloc(int64_t nx, int64_t ny, int64_t ld, double h, double tau, double c, int scheme,
                             uint32_t flags, int64_t steps, float* u, float* lo, float* d, void* stream)
{
    using namespace w2d_host;
    Params p;
    int r = validate(nx, ny, ld, h, tau, c, scheme, flags, &p);
    if (r) return r;
    if (steps < 0) return fail(WAVE2D_EINVAL, "steps must be >= 0");
    if ((r = check_ptrs(p.g, {{u, 4}, {lo, 4}, {d, 4}}))) return r;
    const size_t need = work_bytes_of(WAVE2D_F32C, p.g);
    if (need > kNoAllocBytes)
        return fail(WAVE2D_EINVAL, "grid %lld x %lld (ld %lld) needs %zu bytes of scratch; the fixed array holds %zu",
                    (long long)nx, (long long)ny, (long long)ld, need, kNoAllocBytes);
    void* work;
    if ((r = scratch_ptr(&work))) return r;
    return run_steps_f32c(p, flags, steps, u, lo, d, work, kNoAllocBytes, (hipStream_t)stream);
}

}  // extern "C"

// The integration entry that allocates nothing: the work-queue heads, the
// FP32-to-FP64 hand-back list and the per-state counters of the wavefront
// kernels live in one file-scope device array of fixed size instead of
// buffers the handle allocates on demand.  Each device the library runs on
// holds its own copy of the array for the life of the process; its device
// address is looked up once per device with that device current and used for
// every launch (the array's name is only a host-side stand-in).
#include <hip/hip_runtime.h>
#include <mutex>

#include "rk_internal.h"

namespace {

constexpr int64_t kMaxStates = 262144;        // states per call
constexpr int kQueueInts = 64;                // queue heads, padded to 256 bytes
constexpr size_t kScratchInts = (size_t)kQueueInts + (size_t)kMaxStates * (1 + rk::kNumCounters);

__device__ __align__(256) int32_t scratch[kScratchInts];   // 11.5 MB per device

constexpr int kMaxDevices = 64;
std::mutex g_mu;
int32_t *g_ptr[kMaxDevices] = {};

// device address of this device's copy of the array (looked up on first use)
int scratch_ptr(int32_t **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return rk_fail(RK_EHIP, "radau_integrate_noalloc: hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return rk_fail(RK_EINVAL, "radau_integrate_noalloc: device index too large");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return rk_fail(RK_EHIP, "radau_integrate_noalloc: hipGetSymbolAddress of the static workspace failed");
        }
        g_ptr[dev] = static_cast<int32_t *>(p);
    }
    *out = g_ptr[dev];
    return RK_OK;
}

}  // namespace

extern "C" int radau_integrate_noalloc(rk_mech *mech, int64_t n_states, double dt, const double *d_y_in,
                                       double *d_y_out, double atol, double rtol, void *stream) {
    if (n_states > kMaxStates)
        return rk_fail(RK_EINVAL, "radau_integrate_noalloc: at most 262144 states per call");
    int32_t *base = nullptr;
    const int rc = scratch_ptr(&base);
    if (rc != RK_OK) return rc;
    rk::Work w;
    w.queue = base;
    w.fb_list = base + kQueueInts;
    w.counters = base + kQueueInts + kMaxStates;
    w.allow_predictor = false;
    return rk_integrate_common(mech, n_states, dt, d_y_in, d_y_out, atol, rtol, stream, &w);
}

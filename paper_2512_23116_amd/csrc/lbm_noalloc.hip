// lbm_noalloc.hip — the theta histogram without any device allocation, for
// callers that cannot allocate device memory (code that runs while a HIP graph
// is being captured elsewhere in the process, tight serving loops, harnesses
// that forbid hipMalloc).
//
// lbm_theta_histogram keeps its counts in a device buffer it allocates on its
// first call.  This variant counts into `scratch`, a file-scope device array of
// a fixed size (kNoallocMaxBins + 3 64-bit counters, 32.8 KB) that every GPU the
// library runs on holds until the process ends.  Host code never uses the
// array's name as an address (on the host it is only a stand-in for the
// symbol): the device address is looked up once per device with
// hipGetSymbolAddress and kept in `g_scratch`.  Calls on one device share its
// array; each call clears the counters it uses with a fill kernel before
// counting, and two calls that overlap on one device race.
#include <cmath>
#include <mutex>

#include "lbm_internal.hpp"

namespace {

constexpr int kNoallocMaxBins = 4096;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned long long scratch[kNoallocMaxBins + 3];

std::mutex g_scratch_mu;
unsigned long long* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on `dev` (the current device); looked up on
// the first call on that device.
hipError_t scratch_on(int dev, unsigned long long** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = (unsigned long long*)p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

__global__ __launch_bounds__(256) void k_zero_counts(unsigned long long* c, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) c[i] = 0ull;
}

lbm_status set_err(lbm_handle* h, lbm_status st, const char* m) {
    h->err = m;
    return st;
}

lbm_status hip_err(lbm_handle* h, hipError_t e, const char* what) {
    h->err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? LBM_ERR_OUT_OF_MEMORY : LBM_ERR_DEVICE;
}

}  // namespace

extern "C" lbm_status lbm_theta_histogram_noalloc(lbm_handle* h, double lo, double hi,
                                                  int32_t nbins, int64_t* counts) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (!counts) return set_err(h, LBM_ERR_INVALID_ARG, "counts is NULL");
    if (nbins < 1 || nbins > kNoallocMaxBins)
        return set_err(h, LBM_ERR_INVALID_ARG,
                       "nbins must be 1..4096 (the size of the static device scratch)");
    if (!(std::isfinite(lo) && std::isfinite(hi) && hi > lo))
        return set_err(h, LBM_ERR_INVALID_ARG, "need finite lo < hi");
    if (!h->initialized) return set_err(h, LBM_ERR_STATE, "state not initialised");
    if (h->device < 0 || h->device >= kMaxDevices)
        return set_err(h, LBM_ERR_DEVICE, "device index beyond the scratch table");
    // the symbol lookup and the launches run with the handle's device current
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != h->device) e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_err(h, e, "hipSetDevice");
    unsigned long long* c = nullptr;
    const int n = nbins + 3;
    e = scratch_on(h->device, &c);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_zero_counts, dim3((n + 255) / 256), dim3(256), 0, h->stream, c, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = lbm::launch_theta_hist(h->cfg.precision, lbm::current_pattern(h), lbm::current_args(h),
                                   lo, (double)nbins / (hi - lo), nbins, c, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(counts, c, (size_t)n * sizeof(int64_t), hipMemcpyDeviceToHost,
                           h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (prev >= 0 && prev != h->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_err(h, e, "theta histogram (static scratch)");
    return LBM_OK;
}

// Allocation-free one-shot correlation (include/xcorr.h,
// xcorr_correlate_static): the running sums of an integration that spans
// several launches live in a file-scope device array held by the library, so
// the call allocates nothing.  Each GPU the library runs on holds its own
// copy of the array (at its own address) until the process ends.
#include "xcorr.h"
#include "xcorr_internal.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

namespace {

constexpr size_t kScratchBytes = XCORR_STATIC_SCRATCH_BYTES;

// The running sums of the static entry point.  In host code this name is a
// stand-in, not a device address: kernels receive the address looked up per
// device below.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of this GPU's copy of `scratch`, looked up once per device
// (with that device current) on its first call.
int scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return xc::api_error(XCORR_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return xc::api_error(XCORR_E_DEVICE, "device index outside the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return xc::api_error(XCORR_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return XCORR_OK;
}

}  // namespace

extern "C" int xcorr_correlate_static(const xcorr_config *cfg, const void *d_volts, int64_t n_samples, void *d_out,
                                      int64_t *n_integrated, void *stream)
{
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc)
        return rc;
    return xc::correlate_once(cfg, ws, kScratchBytes, d_volts, n_samples, d_out, n_integrated,
                              reinterpret_cast<hipStream_t>(stream));
}

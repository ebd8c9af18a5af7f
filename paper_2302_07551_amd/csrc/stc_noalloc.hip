// Allocation-free residual: stc_residual_noalloc stages its padded vector and
// partial sums in a static device array instead of the handle's arena, for
// callers that cannot allocate device memory.
#include <mutex>

#include "stc_internal.h"

namespace {

// Staging of stc_residual_noalloc on each GPU the library runs on (held until
// the process ends).  Host code never uses this name as an address: it takes
// the device's copy from hipGetSymbolAddress.
constexpr size_t kScratchBytes = STC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device copy of scratch on `device` (the current device), looked up once
// per device.
stc_status scratch_on(int device, void **out) {
    if (device < 0 || device >= kMaxDevices)
        return stc::report_error(STC_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return stc::report_error(STC_EDEVICE, "hipGetSymbolAddress of the static staging "
                                                  "array failed");
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return STC_OK;
}

}  // namespace

extern "C" stc_status stc_residual_noalloc(stc_handle *h, const double *x, double *res_1) {
    int device = -1;
    if (hipGetDevice(&device) != hipSuccess)
        return stc::report_error(STC_EDEVICE, "hipGetDevice failed");
    void *ptr = nullptr;
    const stc_status rc = scratch_on(device, &ptr);
    if (rc != STC_OK) return rc;
    return stc::residual_into(h, x, res_1, device, static_cast<char *>(ptr), kScratchBytes);
}

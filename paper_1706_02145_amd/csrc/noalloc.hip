// Allocation-free coupling mat-vec (celes_apply_W_noalloc): the mat-vec's
// scratch (source sums/differences and source-chunk partial sums) lives in a
// fixed file-scope device array instead of memory the library allocates, for
// callers that cannot allocate (stream capture, serving loops).
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)CELES_NOALLOC_SCRATCH_BYTES;

// One copy per device, held until the process ends.  Host code must never
// pass this name to a kernel: it is a host-side stand-in.  The device
// address comes from hipGetSymbolAddress, per device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// device address of `scratch` on `device`, looked up once per device with
// that device current (the caller's current device is restored)
int scratch_ptr(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return CELES_E_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return CELES_E_DEVICE;
        if (cur != device && hipSetDevice(device) != hipSuccess) return CELES_E_DEVICE;
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) return CELES_E_DEVICE;
        g_ptr[device] = p;
    }
    *out = g_ptr[device];
    return CELES_OK;
}

}  // namespace

extern "C" int celes_apply_W_noalloc(celes_handle* h, int precision, int K, const void* x_dev, void* y_dev,
                                     void* stream) {
    return celes_guard([&] {
        if (!h) return CELES_E_ARG;
        if (K < 1 || !x_dev || !y_dev) {
            h->err = "K < 1 or null device pointer";
            return CELES_E_ARG;
        }
        void* p = nullptr;
        const int rc = scratch_ptr(h->opt.device, &p);
        if (rc != CELES_OK) {
            h->err = "cannot resolve the fixed scratch buffer on this device";
            return rc;
        }
        return matvec_on_scratch(h, precision, K, x_dev, y_dev, (hipStream_t)stream, p, kScratchBytes);
    });
}

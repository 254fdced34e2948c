// Private definitions shared by the library's translation units: the
// problem handle and a small owning device buffer.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/celes.h"
#include "device_common.hpp"
#include "host_math.hpp"
#include "precond.hpp"

// No C++ exception crosses the C ABI: every entry point that allocates on
// the host runs its body through this guard (host allocation failure ->
// CELES_E_OOM, anything else -> CELES_E_DEVICE).
template <typename F>
int celes_guard(F&& body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return CELES_E_OOM;
    } catch (...) {
        return CELES_E_DEVICE;
    }
}

namespace celes {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    bool ensure(size_t b) {
        if (b <= bytes && p) return true;
        release();
        if (hipMalloc(&p, b) != hipSuccess) {
            p = nullptr;
            return false;
        }
        bytes = b;
        return true;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

}  // namespace celes

struct celes_handle {
    using DevBuf = celes::DevBuf;
    using cplx = celes::cplx;

    celes_options opt;
    int64_t N = 0;
    int L = 0, nmax = 0, half = 0;
    double n0 = 1, wavelength = 0, k = 0;
    std::vector<double> pos;     // [N][3]
    std::vector<double> radius;  // [N]
    std::vector<cplx> nsph;      // [N]
    std::vector<cplx> tq;        // [N][2][L]
    // Hankel table
    double lut_lo = 0, lut_dr = 1;
    int64_t lut_n = 0;
    // device data
    DevBuf d_px, d_py, d_pz, d_tq64, d_tq32, d_lut64, d_lut32;
    DevBuf d_mrec;               // block-entry records of the matrix-core mat-vec (lmax <= 4)
    DevBuf d_xsd, d_part;        // mat-vec scratch
    DevBuf d_ffb, d_ffdir, d_ffc;  // far-field sums: coefficients, directions, sums
    // incident field / solution (host, canonical layout [K][N][nmax])
    int K = 0;
    std::vector<cplx> a_in;
    // incident description (for the near field): plane waves or one Gaussian beam
    bool gaussian = false;
    std::vector<double> pw_beta, pw_alpha;
    std::vector<int> pw_pol;
    std::vector<cplx> pw_E0;
    double g_waist = 0, g_focus[3] = {0, 0, 0}, g_alpha = 0;
    cplx g_E0 = 1.0;
    std::vector<cplx> b;
    bool have_solution = false;
    // solver scratch
    DevBuf d_V, d_w, d_z, d_r, d_x, d_rhs, d_h, d_partial, d_V32, d_w32, d_z32, d_r32, d_x32;
    // preconditioner
    std::unique_ptr<celes::BlockPrecond> pre;
    uint64_t pre_gen = 0;        // bumped whenever the preconditioner is rebuilt or removed
    int target_blocks = 0;       // mat-vec work split (0: default); forced by tests through the environment
    int tuned_blocks[2] = {0, 0};  // autotuned work split per precision (FP64, complex64); 0: not tuned
    // celes_kernel_timing: HIP events around each coupling-kernel launch
    bool time_kernels = false;
    std::vector<hipEvent_t> tev;  // pairs (begin, end), reused
    size_t tev_used = 0;
    std::string err;
    ~celes_handle() {
        for (hipEvent_t e : tev) (void)hipEventDestroy(e);
    }
};

// y = W x for K right-hand sides on the VALU coupling kernel, with the
// source sums/differences and chunk partial sums in the caller-given device
// buffer scratch [scratch_bytes]: no allocation, no timing events
int matvec_on_scratch(celes_handle* h, int precision, int K, const void* x, void* y, hipStream_t s, void* scratch,
                      size_t scratch_bytes);

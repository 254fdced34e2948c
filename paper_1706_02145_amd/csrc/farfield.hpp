// Far-field sphere sums on the device (Appendix D): for every direction
// rhat_d and multipole n, c_n(d) = sum_i e^{-ik rhat_d . r_i} b^i_n, the part of
// the scattered far field that couples all spheres; the angular functions
// f_n(theta, phi) are applied to c on the host.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "device_common.hpp"

namespace celes {

// px, py, pz: [N] sphere centres; b: [N][nmax] coefficients of one right-hand
// side; dirs: [ndir][3] unit vectors; c: [ndir][nmax] output.  All device
// pointers; enqueued on s.  Returns 0 or -1 (launch error).
int ff_sums_launch(const double* px, const double* py, const double* pz, const cx<double>* b, int64_t N, int nmax,
                   const double* dirs, int64_t ndir, double k, cx<double>* c, hipStream_t s);

}  // namespace celes

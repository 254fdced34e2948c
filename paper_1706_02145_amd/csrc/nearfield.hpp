// Near field on the device (Section 2.1 and Appendix A.1): the scattered
// field sum_i sum_n b^i_n Psi^(3)_n(r - r_i) and plane-wave superpositions
// (plane-wave incidence, the angular spectrum of a Gaussian beam) at
// arbitrary points.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "device_common.hpp"

namespace celes {

// E [npt][3] = sum over spheres of the outgoing SVWF expansion with
// coefficients b [N][nmax] (one right-hand side), at pts [npt][3].  Device
// pointers, enqueued on s.  Returns 0, -1 (launch error) or -2 (L outside
// 1..6).  Points must lie outside every sphere; a point at a sphere's centre
// gets no contribution from that sphere.
int nf_scattered_launch(const double* px, const double* py, const double* pz, const cx<double>* b, int64_t N, int L,
                        const double* pts, int64_t npt, double k, cx<double>* E, hipStream_t s);

// E [npt][3] += sum_q amp_q e^{i kv_q . (p - origin)} for nn plane waves with
// wave vectors kv [nn][3] and complex amplitude vectors amp [nn][3].
int nf_planewaves_launch(const double* kv, const cx<double>* amp, int64_t nn, double ox, double oy, double oz,
                         const double* pts, int64_t npt, cx<double>* E, hipStream_t s);

}  // namespace celes

// Host-side special functions and coefficient tables of the T-matrix method.
// Everything here is FP64 (long double where cancellation matters) and runs
// once per problem; the device kernels consume the resulting tables.
#pragma once
#include <complex>
#include <vector>
#include <cstdint>

namespace celes {

using cplx = std::complex<double>;

inline int half_of(int L) { return L * (L + 2); }
inline int nmax_of(int L) { return 2 * L * (L + 2); }
// index of (l, m) inside one polarisation block: l(l+1) + m - 1
inline int lm_index(int l, int m) { return l * (l + 1) + m - 1; }

// Wigner 3j symbol (Racah formula, long double accumulation)
double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3);

// Translation coefficients of Appendix A.2.  a5 is real; b5 is purely
// imaginary and b5im returns its imaginary part.
double a5_coef(int l, int m, int lp, int mp, int p);
double b5im_coef(int l, int m, int lp, int mp, int p);

// Normalized associated Legendre functions without Condon-Shortley phase,
// P_l^m(cos t) for 0 <= m <= l <= lmax, from cos t and sin t (>= 0).
// out[l*(lmax+1) + m].
void legendre_table(int lmax, double ct, double st, double* out);
// pi_l^m(t) = P_l^m / sin t and tau_l^m(t) = dP_l^m(cos t)/dt, valid at the poles.
void pi_tau(int l, int m, double theta, double* pi, double* tau);

// spherical Hankel h_p(x) = j_p + i y_p, p = 0..pmax, real x > 0, and
// d/dx h_p(x).
void sph_hankel(int pmax, double x, cplx* h, cplx* dh);

// Mie T-matrix entries (Appendix B) for size parameter x = kR and relative
// index m: Q[0][l-1] = Q_{1l}, Q[1][l-1] = Q_{2l}.
void mie_Q(int L, double x, cplx m, cplx* Q1, cplx* Q2);

// Gauss-Legendre nodes/weights on [-1, 1]
void gauss_legendre(int n, double* x, double* w);

// B^dagger_{nj}(beta) of the PVWF-to-SVWF expansion (Appendix A.2, eq. B with
// every explicit i replaced by -i).
cplx b_dagger(int tau, int l, int m, int j, double beta);

}  // namespace celes

// Near-field kernels: one lane per evaluation point, the sources (spheres or
// plane waves) staged in LDS tiles and read as broadcasts, FP64 throughout.
//
// Scattered field of one sphere at r = p - r_i (spherical coordinates of r):
//   Psi_1lm = e_lm h_l(kr) (i m pi_l^|m| e_theta - tau_l^|m| e_phi)
//   Psi_2lm = e_lm [l(l+1) h_l(kr)/(kr) P_l^|m| e_r
//                   + (kr h_{l-1} - l h_l)/(kr) (tau_l^|m| e_theta + i m pi_l^|m| e_phi)]
// with e_lm = e^{i m phi} / sqrt(2 l (l+1)), h_l the spherical Hankel function
// of the first kind (h_0, h_1 from one sincos, then the upward recurrence),
// P_l^m the normalized associated Legendre function without Condon-Shortley
// phase, pi = m P / sin(theta), tau = dP/dtheta.  P_l^m = sin^m R_l^m with R
// a polynomial in cos(theta): R and dR/dcos follow the three-term recurrence
// in l, which keeps pi and tau finite on the axis.
#include "nearfield.hpp"

namespace celes {
namespace {

constexpr int NF_THREADS = 128;
constexpr int NF_TILE = 32;

template <int L>
__global__ void __launch_bounds__(NF_THREADS)
    nf_scattered_kernel(const double* __restrict__ px, const double* __restrict__ py, const double* __restrict__ pz,
                        const cx<double>* __restrict__ b, int64_t N, const double* __restrict__ pts, int64_t npt,
                        double k, cx<double>* __restrict__ E) {
    constexpr int HALF = L * (L + 2), NMAX = 2 * HALF;
    __shared__ double spos[NF_TILE][3];
    __shared__ cx<double> sb[NF_TILE][NMAX];
    const int64_t q = (int64_t)blockIdx.x * NF_THREADS + threadIdx.x;
    double p0 = 0, p1 = 0, p2 = 0;
    if (q < npt) {
        p0 = pts[3 * q];
        p1 = pts[3 * q + 1];
        p2 = pts[3 * q + 2];
    }
    cx<double> Ex = {0, 0}, Ey = {0, 0}, Ez = {0, 0};
    for (int64_t t0 = 0; t0 < N; t0 += NF_TILE) {
        const int nt = (int)min((int64_t)NF_TILE, N - t0);
        __syncthreads();
        for (int e = threadIdx.x; e < nt * NMAX; e += NF_THREADS) sb[e / NMAX][e % NMAX] = b[t0 * NMAX + e];
        for (int e = threadIdx.x; e < nt; e += NF_THREADS) {
            spos[e][0] = px[t0 + e];
            spos[e][1] = py[t0 + e];
            spos[e][2] = pz[t0 + e];
        }
        __syncthreads();
        if (q >= npt) continue;
        for (int s = 0; s < nt; ++s) {
            const double dx = p0 - spos[s][0], dy = p1 - spos[s][1], dz = p2 - spos[s][2];
            const double rho2 = dx * dx + dy * dy, rr = sqrt(rho2 + dz * dz);
            if (!(rr > 0)) continue;
            const double rho = sqrt(rho2);
            const double ct = dz / rr, st = rho / rr;
            const double cp = rho > 0 ? dx / rho : 1.0, sp = rho > 0 ? dy / rho : 0.0;
            const double x = k * rr, inv = 1.0 / x;
            double sn, cs;
            sincos(x, &sn, &cs);
            cx<double> h[L + 1];
            h[0] = {sn * inv, -cs * inv};
            h[1] = {(h[0].re - cs) * inv, (h[0].im - sn) * inv};
#pragma unroll
            for (int l = 1; l < L; ++l)
                h[l + 1] = {(2 * l + 1) * inv * h[l].re - h[l - 1].re, (2 * l + 1) * inv * h[l].im - h[l - 1].im};
            cx<double> Sr = {0, 0}, St = {0, 0}, Sp = {0, 0};
            const cx<double>* bs = sb[s];
            double rmm = 0.70710678118654752440;  // R_0^0 = 1/sqrt(2)
            double stm1 = 1.0;                    // sin^(mu-1) for mu >= 1
            cx<double> eph = {1.0, 0.0};          // e^{i mu phi}
#pragma unroll
            for (int mu = 0; mu <= L; ++mu) {
                if (mu > 0) {
                    rmm *= sqrt((2.0 * mu + 1.0) / (2.0 * mu));
                    if (mu > 1) stm1 *= st;
                    eph = {eph.re * cp - eph.im * sp, eph.re * sp + eph.im * cp};
                }
                // R_l^mu and dR_l^mu/dcos for l = mu .. L
                double R[L + 2], dR[L + 2];
                R[mu] = rmm;
                dR[mu] = 0.0;
                if (mu + 1 <= L) {
                    R[mu + 1] = sqrt(2.0 * mu + 3.0) * ct * rmm;
                    dR[mu + 1] = sqrt(2.0 * mu + 3.0) * rmm;
                }
#pragma unroll
                for (int l = mu + 2; l <= L; ++l) {
                    const double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)mu * mu));
                    const double c = sqrt((2.0 * l + 1.0) * ((l - 1.0) * (l - 1.0) - (double)mu * mu) /
                                          ((2.0 * l - 3.0) * ((double)l * l - (double)mu * mu)));
                    R[l] = a * ct * R[l - 1] - c * R[l - 2];
                    dR[l] = a * (R[l - 1] + ct * dR[l - 1]) - c * dR[l - 2];
                }
#pragma unroll
                for (int l = (mu > 1 ? mu : 1); l <= L; ++l) {
                    const double smu = mu == 0 ? 1.0 : stm1 * st;   // sin^mu
                    const double P = smu * R[l];
                    const double pi = mu == 0 ? 0.0 : stm1 * R[l];
                    const double tau = mu == 0 ? -st * dR[l] : mu * stm1 * ct * R[l] - stm1 * st * st * dR[l];
                    const double nrm = 1.0 / sqrt(2.0 * l * (l + 1));
                    const cx<double> z = h[l];
                    const cx<double> dk = {(x * h[l - 1].re - l * h[l].re) * inv, (x * h[l - 1].im - l * h[l].im) * inv};
                    const cx<double> zr = {l * (l + 1) * z.re * inv * P, l * (l + 1) * z.im * inv * P};
#pragma unroll
                    for (int sg = 0; sg < 2; ++sg) {
                        if (sg == 1 && mu == 0) continue;
                        const int m = sg == 0 ? mu : -mu;
                        // e = e^{i m phi} / sqrt(2l(l+1))
                        const cx<double> e = {eph.re * nrm, (sg == 0 ? eph.im : -eph.im) * nrm};
                        const cx<double> b1 = cmul(bs[l * (l + 1) + m - 1], e);
                        const cx<double> b2 = cmul(bs[HALF + l * (l + 1) + m - 1], e);
                        // tau = 1: z (i m pi e_theta - tau e_phi)
                        const cx<double> zb1 = cmul(b1, z);
                        St.re -= m * pi * zb1.im;
                        St.im += m * pi * zb1.re;
                        Sp.re -= tau * zb1.re;
                        Sp.im -= tau * zb1.im;
                        // tau = 2: zr e_r + dk (tau e_theta + i m pi e_phi)
                        const cx<double> rb = cmul(b2, zr), db = cmul(b2, dk);
                        Sr.re += rb.re;
                        Sr.im += rb.im;
                        St.re += tau * db.re;
                        St.im += tau * db.im;
                        Sp.re -= m * pi * db.im;
                        Sp.im += m * pi * db.re;
                    }
                }
            }
            const double er0 = st * cp, er1 = st * sp, er2 = ct;
            const double et0 = ct * cp, et1 = ct * sp, et2 = -st;
            const double ep0 = -sp, ep1 = cp;
            Ex.re += Sr.re * er0 + St.re * et0 + Sp.re * ep0;
            Ex.im += Sr.im * er0 + St.im * et0 + Sp.im * ep0;
            Ey.re += Sr.re * er1 + St.re * et1 + Sp.re * ep1;
            Ey.im += Sr.im * er1 + St.im * et1 + Sp.im * ep1;
            Ez.re += Sr.re * er2 + St.re * et2;
            Ez.im += Sr.im * er2 + St.im * et2;
        }
    }
    if (q < npt) {
        E[3 * q] = Ex;
        E[3 * q + 1] = Ey;
        E[3 * q + 2] = Ez;
    }
}

constexpr int PW_TILE = 64;

__global__ void __launch_bounds__(NF_THREADS)
    nf_planewaves_kernel(const double* __restrict__ kv, const cx<double>* __restrict__ amp, int64_t nn, double ox,
                         double oy, double oz, const double* __restrict__ pts, int64_t npt,
                         cx<double>* __restrict__ E) {
    __shared__ double sk[PW_TILE][3];
    __shared__ cx<double> sa[PW_TILE][3];
    const int64_t q = (int64_t)blockIdx.x * NF_THREADS + threadIdx.x;
    double r0 = 0, r1 = 0, r2 = 0;
    if (q < npt) {
        r0 = pts[3 * q] - ox;
        r1 = pts[3 * q + 1] - oy;
        r2 = pts[3 * q + 2] - oz;
    }
    cx<double> acc[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t t0 = 0; t0 < nn; t0 += PW_TILE) {
        const int nt = (int)min((int64_t)PW_TILE, nn - t0);
        __syncthreads();
        for (int e = threadIdx.x; e < nt * 3; e += NF_THREADS) {
            sk[e / 3][e % 3] = kv[t0 * 3 + e];
            sa[e / 3][e % 3] = amp[t0 * 3 + e];
        }
        __syncthreads();
        if (q >= npt) continue;
        for (int s = 0; s < nt; ++s) {
            double sn, cs;
            sincos(sk[s][0] * r0 + sk[s][1] * r1 + sk[s][2] * r2, &sn, &cs);
            const cx<double> ph = {cs, sn};
#pragma unroll
            for (int a = 0; a < 3; ++a) cfma(acc[a], sa[s][a], ph);
        }
    }
    if (q < npt)
        for (int a = 0; a < 3; ++a) {
            E[3 * q + a].re += acc[a].re;
            E[3 * q + a].im += acc[a].im;
        }
}

template <int L>
int launch_L(const double* px, const double* py, const double* pz, const cx<double>* b, int64_t N,
             const double* pts, int64_t npt, double k, cx<double>* E, hipStream_t s) {
    hipLaunchKernelGGL(nf_scattered_kernel<L>, dim3((unsigned)((npt + NF_THREADS - 1) / NF_THREADS)),
                       dim3(NF_THREADS), 0, s, px, py, pz, b, N, pts, npt, k, E);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int nf_scattered_launch(const double* px, const double* py, const double* pz, const cx<double>* b, int64_t N, int L,
                        const double* pts, int64_t npt, double k, cx<double>* E, hipStream_t s) {
    if (npt <= 0) return 0;
    switch (L) {
        case 1: return launch_L<1>(px, py, pz, b, N, pts, npt, k, E, s);
        case 2: return launch_L<2>(px, py, pz, b, N, pts, npt, k, E, s);
        case 3: return launch_L<3>(px, py, pz, b, N, pts, npt, k, E, s);
        case 4: return launch_L<4>(px, py, pz, b, N, pts, npt, k, E, s);
        case 5: return launch_L<5>(px, py, pz, b, N, pts, npt, k, E, s);
        case 6: return launch_L<6>(px, py, pz, b, N, pts, npt, k, E, s);
        default: return -2;
    }
}

int nf_planewaves_launch(const double* kv, const cx<double>* amp, int64_t nn, double ox, double oy, double oz,
                         const double* pts, int64_t npt, cx<double>* E, hipStream_t s) {
    if (npt <= 0 || nn <= 0) return 0;
    hipLaunchKernelGGL(nf_planewaves_kernel, dim3((unsigned)((npt + NF_THREADS - 1) / NF_THREADS)), dim3(NF_THREADS),
                       0, s, kv, amp, nn, ox, oy, oz, pts, npt, E);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace celes

// Coupling mat-vec W x by rotation, translation along z and rotation back
// (the O(lmax^3) translation that the paper's Discussion, Section 5, names
// for larger lmax), hand-written for gfx950.
//
// For a pair with displacement d = |d| (sin t cos f, sin t sin f, cos t) the
// translation operator factorises as A(d) = U A(|d| z) U^H, U the rotation
// of the SVWF basis taking z to d: block-diagonal in (tau, l),
//   U^l_{m m''} = e^{i m f} c_m c_{m''} d^l_{m m''}(t),  c_m = (-1)^m (m > 0), 1 (m <= 0),
// and A(|d| z) couples only equal m.  The coupling block of the mat-vec is
// A^T (Section 2.2: W^{ii'}_{nn'} = A_{n'n}), so per pair
//   y_i += conj(U) A_z^T U^T x_j
// on the polarisation sums/differences s = x_1 + x_2 (with A + iB) and
// d = x_1 - x_2 (with A - iB), one pass each (blockIdx.z).
//
// Wigner's d at an arbitrary angle is never evaluated: with
// Delta^l = d^l(pi/2) (compile-time constants) and P = diag(i^m),
//   d^l(t) = P Delta^T diag(e^{-ikt}) Delta P^*,
// so each rotation is two constant real matrix products around a diagonal
// phase.  The unit factors i^m c_m and the phases e^{imf} combine into powers
// of q = -i e^{if}; the factors between the two rotations combine into
// (-1)^m on the axial translation.
//
// Mapping as in the direct kernel: one lane per receiving sphere, a block
// walks a chunk of sources staged in LDS tiles (broadcast reads), partial sums
// per (chunk, pass) in the same layout, reduced by the same finish kernel.
#include <hip/hip_runtime.h>
#include <type_traits>

#include "device_common.hpp"
#include "wx_plan.hpp"
#include "wx_launch.hpp"

#ifndef CELES_WX_L
#error "define CELES_WX_L (1..6)"
#endif

namespace celes {

using namespace plan;

namespace rtr {

constexpr int BLOCK = 64;   // receivers per block (one wave)
constexpr int TILE = 16;    // sources per LDS tile

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

// d^l_{k m}(pi/2) by Wigner's sum: at pi/2 every cos/sin power is 2^{-l/...}
// so that d = 2^{-l} sqrt((l+k)!(l-k)!(l+m)!(l-m)!) / (2l)! *
// sum_j (-1)^{k-m+j} (2l)! / ((l+m-j)! j! (k-m+j)! (l-k-j)!), an integer sum
constexpr double delta(int l, int k, int m) {
    double s = 0.0;
    for (int j = 0; j <= 2 * l; ++j) {
        const int a = l + m - j, b = k - m + j, c = l - k - j;
        if (a < 0 || b < 0 || c < 0) continue;
        const double multi = cfact(2 * l) / (cfact(a) * cfact(j) * cfact(b) * cfact(c));
        s += (((k - m + j) % 2 + 2) % 2 ? -1.0 : 1.0) * multi;
    }
    double p2 = 1.0;
    for (int i = 0; i < l; ++i) p2 *= 2.0;
    return s * csqrt(cfact(l + k) * cfact(l - k) * cfact(l + m) * cfact(l - m)) / (cfact(2 * l) * p2);
}

// axial translation coefficient of the p term: a5 (or Im b5) at m' = m,
// source (l', m) first, times P_p^0(1) = sqrt((2p+1)/2)
constexpr double za(int lp, int l, int m, int p) { return ca5(lp, m, l, m, p) * csqrt((2.0 * p + 1.0) / 2.0); }
constexpr double zb(int lp, int l, int m, int p) { return cb5im(lp, m, l, m, p) * csqrt((2.0 * p + 1.0) / 2.0); }

constexpr int off(int l, int m) { return l * (l + 1) + m - 1; }

// g = Delta^l u (rows k, columns m), constant real matrix on complex
// vectors.  Delta_{k,-m} = (-1)^{l+k} Delta_{k,m}, so with S_m = u_m + u_{-m}
// and D_m = u_m - u_{-m} each output sums over m >= 0 only:
//   g_k = Delta_{k0} u_0 + sum_{m>0} Delta_{km} (l+k even ? S_m : D_m)
template <typename T, int l>
__device__ __forceinline__ void delta_mul(const cx<T> (&u)[2 * l + 1], cx<T> (&g)[2 * l + 1]) {
    cx<T> S[l + 1], D[l + 1];
    sfor<1, l + 1>([&](auto M_) {
        constexpr int m = decltype(M_)::value;
        S[m] = {u[l + m].re + u[l - m].re, u[l + m].im + u[l - m].im};
        D[m] = {u[l + m].re - u[l - m].re, u[l + m].im - u[l - m].im};
    });
    sfor<-l, l + 1>([&](auto K_) {
        constexpr int k = decltype(K_)::value;
        constexpr bool even = ((l + k) & 1) == 0;
        cx<T> acc = {0, 0};
        constexpr double c0 = delta(l, k, 0);
        if constexpr (c0 != 0.0) acc = {(T)c0 * u[l].re, (T)c0 * u[l].im};
        sfor<1, l + 1>([&](auto M_) {
            constexpr int m = decltype(M_)::value;
            constexpr double c = delta(l, k, m);
            if constexpr (c != 0.0) {
                const cx<T>& v = even ? S[m] : D[m];
                acc.re = fma((T)c, v.re, acc.re);
                acc.im = fma((T)c, v.im, acc.im);
            }
        });
        g[k + l] = acc;
    });
}

// w = Delta^T g.  Delta_{-k,m} = (-1)^{l+m} Delta_{k,m}, so with
// P_k = g_k + g_{-k} and Q_k = g_k - g_{-k}:
//   w_m = Delta_{0m} g_0 + sum_{k>0} Delta_{km} (l+m even ? P_k : Q_k)
template <typename T, int l>
__device__ __forceinline__ void delta_tmul(const cx<T> (&g)[2 * l + 1], cx<T> (&w)[2 * l + 1]) {
    cx<T> Pk[l + 1], Qk[l + 1];
    sfor<1, l + 1>([&](auto K_) {
        constexpr int k = decltype(K_)::value;
        Pk[k] = {g[l + k].re + g[l - k].re, g[l + k].im + g[l - k].im};
        Qk[k] = {g[l + k].re - g[l - k].re, g[l + k].im - g[l - k].im};
    });
    sfor<-l, l + 1>([&](auto M_) {
        constexpr int m = decltype(M_)::value;
        constexpr bool even = ((l + m) & 1) == 0;
        cx<T> acc = {0, 0};
        constexpr double c0 = delta(l, 0, m);
        if constexpr (c0 != 0.0) acc = {(T)c0 * g[l].re, (T)c0 * g[l].im};
        sfor<1, l + 1>([&](auto K_) {
            constexpr int k = decltype(K_)::value;
            constexpr double c = delta(l, k, m);
            if constexpr (c != 0.0) {
                const cx<T>& v = even ? Pk[k] : Qk[k];
                acc.re = fma((T)c, v.re, acc.re);
                acc.im = fma((T)c, v.im, acc.im);
            }
        });
        w[m + l] = acc;
    });
}

// g_k *= e^{-ik t}: ep[k] = e^{ik t} for k >= 0
template <typename T, int l, int LL>
__device__ __forceinline__ void theta_phase(cx<T> (&g)[2 * l + 1], const cx<T> (&ep)[LL + 1]) {
    sfor<1, l + 1>([&](auto K_) {
        constexpr int k = decltype(K_)::value;
        g[l + k] = cmulc(g[l + k], ep[k]);     // e^{-ikt}
        g[l - k] = cmul(g[l - k], ep[k]);      // e^{+ikt}
    });
}

// The rotated source vector lives in registers, or, where registers would
// spill (FP64 at lmax >= 5), in per-lane LDS slots [entry][lane].
template <typename T, int L>
constexpr bool t_in_lds() { return sizeof(T) == 8 && L >= 5; }

template <typename T, int L, bool LDS>
struct RotVec;
template <typename T, int L>
struct RotVec<T, L, false> {
    cx<T> r[L * (L + 2)];
    __device__ __forceinline__ RotVec(cx<T>*) {}
    __device__ __forceinline__ cx<T> get(int c) const { return r[c]; }
    __device__ __forceinline__ void set(int c, cx<T> v) { r[c] = v; }
};
template <typename T, int L>
struct RotVec<T, L, true> {
    cx<T>* s;   // this lane's column of [entry][BLOCK]
    __device__ __forceinline__ RotVec(cx<T>* lane_slots) : s(lane_slots) {}
    __device__ __forceinline__ cx<T> get(int c) const { return s[c * BLOCK]; }
    __device__ __forceinline__ void set(int c, cx<T> v) { s[c * BLOCK] = v; }
};

// one pair: y += conj(U) A_z^{+-T} U^T v  (SG = +1: A + iB, SG = -1: A - iB)
template <typename T, int L, int SG>
__device__ __forceinline__ void rtr_pair(const cx<T>* __restrict__ v, const cx<T> (&h)[2 * L + 1],
                                         const cx<T> (&qp)[L + 1], const cx<T> (&ep)[L + 1],
                                         cx<T> (&y)[L * (L + 2)], cx<T>* lane_slots) {
    // ---- rotate into the pair frame: t = U^T v, without its last unit
    // factor (folded into the axial step) ----
    RotVec<T, L, t_in_lds<T, L>()> t(lane_slots);
    sfor<1, L + 1>([&](auto LP_) {
        constexpr int l = decltype(LP_)::value;
        cx<T> u[2 * l + 1], g[2 * l + 1], w[2 * l + 1];
        u[l] = v[off(l, 0)];
        sfor<1, l + 1>([&](auto M_) {
            constexpr int m = decltype(M_)::value;
            u[l + m] = cmul(qp[m], v[off(l, m)]);                    // q^m v_m
            const cx<T> b = cmulc(v[off(l, -m)], qp[m]);              // conj(q^m) v_{-m}
            u[l - m] = (m & 1) ? cx<T>{-b.re, -b.im} : b;             // (-1)^m
        });
        delta_mul<T, l>(u, g);
        theta_phase<T, l, L>(g, ep);
        delta_tmul<T, l>(g, w);
        sfor<0, 2 * l + 1>([&](auto C_) { t.set(off(l, decltype(C_)::value - l), w[decltype(C_)::value]); });
    });
    // ---- translate along z (m-diagonal) and rotate back, output degree by degree ----
    sfor<1, L + 1>([&](auto L_) {
        constexpr int l = decltype(L_)::value;
        cx<T> z[2 * l + 1], g[2 * l + 1], w[2 * l + 1];
        // A_z is even and B_z odd under m -> -m (Appendix A.2 mirror
        // symmetry): one pair of p sums serves m and -m
        sfor<0, l + 1>([&](auto M_) {
            constexpr int m = decltype(M_)::value;
            cx<T> accp = {0, 0}, accm = {0, 0};
            sfor<(m > 1 ? m : 1), L + 1>([&](auto LQ_) {
                constexpr int lp = decltype(LQ_)::value;
                // A_z and B_z entry (source (lp, m), receiver (l, m))
                cx<T> A = {0, 0}, B = {0, 0};
                sfor<0, 2 * L + 1>([&](auto P_) {
                    constexpr int p = decltype(P_)::value;
                    constexpr double ca = za(lp, l, m, p), cb = zb(lp, l, m, p);
                    if constexpr (ca != 0.0) {
                        A.re = fma((T)ca, h[p].re, A.re);
                        A.im = fma((T)ca, h[p].im, A.im);
                    }
                    if constexpr (cb != 0.0) {
                        B.re = fma((T)cb, h[p].re, B.re);
                        B.im = fma((T)cb, h[p].im, B.im);
                    }
                });
                // coefficients (-1)^m (A +- iB) for +m and (-1)^m (A -+ iB) for -m:
                // the (-1)^m is the two rotations' unit factors
                constexpr T sa = (T)((m & 1) ? -1 : 1);
                constexpr T sg = (T)SG * sa;
                const cx<T> cp = {sa * A.re - sg * B.im, sa * A.im + sg * B.re};
                cfma(accp, cp, t.get(off(lp, m)));
                if constexpr (m > 0) {
                    const cx<T> cm = {sa * A.re + sg * B.im, sa * A.im - sg * B.re};
                    cfma(accm, cm, t.get(off(lp, -m)));
                }
            });
            z[l + m] = accp;
            if constexpr (m > 0) z[l - m] = accm;
        });
        delta_mul<T, l>(z, g);
        theta_phase<T, l, L>(g, ep);
        delta_tmul<T, l>(g, w);
        y[off(l, 0)].re += w[l].re;
        y[off(l, 0)].im += w[l].im;
        sfor<1, l + 1>([&](auto M_) {
            constexpr int m = decltype(M_)::value;
            // y_m += (-1)^m conj(q^m) w_m,  y_{-m} += q^m w_{-m}
            const cx<T> a = cmulc(w[l + m], qp[m]);
            if constexpr (m & 1) {
                y[off(l, m)].re -= a.re;
                y[off(l, m)].im -= a.im;
            } else {
                y[off(l, m)].re += a.re;
                y[off(l, m)].im += a.im;
            }
            cfma(y[off(l, -m)], qp[m], w[l - m]);
        });
    });
}

template <typename T, int P>
__device__ __forceinline__ void hankel_lut(double d, double inv_kd, const LutView<T>& lut, cx<T> (&h)[P + 1]) {
    double s = (d - lut.d_lo) * lut.inv_dr;
    int q = (int)s;
    q = q < 0 ? 0 : (q >= lut.n_int ? lut.n_int - 1 : q);
    T tt = (T)(s - (double)q);
    const cx<T>* c = lut.coef + (size_t)q * 8;
#pragma unroll
    for (int p = 0; p <= (P < 1 ? P : 1); ++p) {
        cx<T> c0 = c[4 * p], c1 = c[4 * p + 1], c2 = c[4 * p + 2], c3 = c[4 * p + 3];
        h[p].re = fma(fma(fma(c3.re, tt, c2.re), tt, c1.re), tt, c0.re);
        h[p].im = fma(fma(fma(c3.im, tt, c2.im), tt, c1.im), tt, c0.im);
    }
    const T fi = (T)inv_kd;
#pragma unroll
    for (int p = 1; p < P; ++p) {
        T f = (T)(2 * p + 1) * fi;
        h[p + 1] = {f * h[p].re - h[p - 1].re, f * h[p].im - h[p - 1].im};
    }
}

template <typename T, int P>
__device__ __forceinline__ void hankel_direct(double kd, cx<T> (&h)[P + 1]) {
    double s, c;
    sincos(kd, &s, &c);
    const double inv = 1.0 / kd;
    const double h0r = s * inv, h0i = -c * inv;
    h[0] = {(T)h0r, (T)h0i};
    if constexpr (P >= 1) h[1] = {(T)((h0r - c) * inv), (T)((h0i - s) * inv)};
    const T fi = (T)inv;
#pragma unroll
    for (int p = 1; p < P; ++p) {
        T f = (T)(2 * p + 1) * fi;
        h[p + 1] = {f * h[p].re - h[p - 1].re, f * h[p].im - h[p - 1].im};
    }
}

template <typename T, int L, int HMODE, int SG>
__device__ __forceinline__ void rtr_block(const WxArgs<T>& a, cx<T>* tile, cx<T>* slots, int bx, int chunk, int k) {
    constexpr int HALF = L * (L + 2);
    constexpr int PASS = SG > 0 ? 0 : 1;   // s (x_1 + x_2) or d (x_1 - x_2)
    const int i = bx * BLOCK + threadIdx.x;
    const bool active = i < a.n;
    const double xi = active ? a.px[i] : 0.0;
    const double yi = active ? a.py[i] : 0.0;
    const double zi = active ? a.pz[i] : 0.0;
    cx<T> y[HALF];
#pragma unroll
    for (int c = 0; c < HALF; ++c) y[c] = {0, 0};
    const int j0 = chunk * a.chunk_len;
    const int j1 = min(a.n, j0 + a.chunk_len);
    for (int t0 = j0; t0 < j1; t0 += TILE) {
        const int nt = min(TILE, j1 - t0);
        __syncthreads();
        for (int e = threadIdx.x; e < nt * HALF; e += BLOCK) {
            const int jj = e / HALF, r = e % HALF;
            tile[e] = a.xsd[((size_t)(t0 + jj) * a.nrhs + k) * (2 * HALF) + PASS * HALF + r];
        }
        __syncthreads();
        for (int jj = 0; jj < nt; ++jj) {
            const int j = t0 + jj;
            if (!active || j == i) continue;
            const double dx = xi - a.px[j], dy = yi - a.py[j], dz = zi - a.pz[j];
            const double rho2 = dx * dx + dy * dy;
            const double r = sqrt(rho2 + dz * dz);
            const double inv_r = 1.0 / r;
            const double rho = sqrt(rho2);
            double cf = 1.0, sf = 0.0;
            if (rho > 0.0) {
                const double ir = 1.0 / rho;
                cf = dx * ir;
                sf = dy * ir;
            }
            cx<T> h[2 * L + 1];
            if constexpr (HMODE == 0)
                hankel_lut<T, 2 * L>(r, inv_r * a.lut.inv_k, a.lut, h);
            else
                hankel_direct<T, 2 * L>(a.k * r, h);
            // powers of q = -i e^{if} and of e^{it}
            cx<T> qp[L + 1], ep[L + 1];
            qp[0] = {1, 0};
            ep[0] = {1, 0};
            const cx<T> q1 = {(T)sf, (T)(-cf)};
            const cx<T> e1 = {(T)(dz * inv_r), (T)(rho * inv_r)};
#pragma unroll
            for (int m = 1; m <= L; ++m) {
                qp[m] = cmul(qp[m - 1], q1);
                ep[m] = cmul(ep[m - 1], e1);
            }
            rtr_pair<T, L, SG>(tile + jj * HALF, h, qp, ep, y, slots + threadIdx.x);
        }
    }
    if (!active) return;
    cx<T>* out = a.part + ((size_t)chunk * a.nrhs + k) * (2 * HALF) * a.ldp;
#pragma unroll
    for (int c = 0; c < HALF; ++c) out[(size_t)(PASS * HALF + c) * a.ldp + i] = y[c];
}

// waves per SIMD the compiler must leave room for: three for the complex64
// kernel at lmax 4 (168 VGPRs and 36 B of spill per lane instead of 240
// VGPRs: 28.0 vs 29.2 ms per W x on the 20,000-sphere slab, same bits);
// elsewhere no constraint (lmax 5-6 measured slower with it)
template <typename T, int L>
constexpr int rtr_min_waves() { return sizeof(T) == 4 && L == 4 ? 3 : 1; }

// grid: (receiver tiles, source chunks, 2 passes x right-hand sides)
template <typename T, int L, int HMODE>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(rtr_min_waves<T, L>())))
void wx_rtr_kernel(WxArgs<T> a) {
    constexpr int HALF = L * (L + 2);
    __shared__ cx<T> tile[TILE * HALF];
    __shared__ cx<T> slots[t_in_lds<T, L>() ? HALF * BLOCK : 1];
    const int k = blockIdx.z >> 1;
    if ((blockIdx.z & 1) == 0)
        rtr_block<T, L, HMODE, 1>(a, tile, slots, blockIdx.x, blockIdx.y, k);
    else
        rtr_block<T, L, HMODE, -1>(a, tile, slots, blockIdx.x, blockIdx.y, k);
}

// Persistent multi-problem variant (batches): as the direct scheme's batch
// kernel, every block repeatedly claims the next work item (problem p,
// receiver tile, source chunk, pass x right-hand side) from a counter that
// must be zero at launch; items of problem p are numbered
// [item_off[p], item_off[p+1]).  Items of converged systems are skipped.
// Every block exits once the counter passes the last item.
template <typename T, int L, int HMODE>
__global__ __launch_bounds__(BLOCK) void wx_rtr_batch_kernel(const WxArgs<T>* __restrict__ args,
                                                             const int* __restrict__ item_off,
                                                             const int* __restrict__ nbx,
                                                             const int* __restrict__ nchunk, int nprob,
                                                             int* __restrict__ counter) {
    constexpr int HALF = L * (L + 2);
    __shared__ cx<T> tile[TILE * HALF];
    __shared__ cx<T> slots[t_in_lds<T, L>() ? HALF * BLOCK : 1];
    __shared__ int s_item;
    const int total = item_off[nprob];
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= total) break;
        int p = 0;
        while (item_off[p + 1] <= item) ++p;
        const int local = item - item_off[p];
        const int bxn = nbx[p], chn = nchunk[p];
        const int bx = local % bxn;
        const int chunk = (local / bxn) % chn;
        const int z = local / (bxn * chn);
        const int k = z >> 1;
        const WxArgs<T> a = args[p];
        if (a.active && a.active[a.sys0 + k] == 0) continue;
        if ((z & 1) == 0)
            rtr_block<T, L, HMODE, 1>(a, tile, slots, bx, chunk, k);
        else
            rtr_block<T, L, HMODE, -1>(a, tile, slots, bx, chunk, k);
    }
}

}  // namespace rtr

template <typename T, int L>
void wx_rtr_batch_run_L(const WxArgs<T>* args, const int* item_off, const int* nbx, const int* nchunk, int nprob,
                        int* counter, int nblocks, int hmode, hipStream_t s) {
    if constexpr (L > 4) {
        return;       // batches are compiled for cut-offs up to 4
    } else {
        if (hmode == 0)
            hipLaunchKernelGGL((rtr::wx_rtr_batch_kernel<T, L, 0>), dim3(nblocks), dim3(rtr::BLOCK), 0, s, args,
                               item_off, nbx, nchunk, nprob, counter);
        else
            hipLaunchKernelGGL((rtr::wx_rtr_batch_kernel<T, L, 1>), dim3(nblocks), dim3(rtr::BLOCK), 0, s, args,
                               item_off, nbx, nchunk, nprob, counter);
    }
}
template void wx_rtr_batch_run_L<double, CELES_WX_L>(const WxArgs<double>*, const int*, const int*, const int*, int,
                                                     int*, int, int, hipStream_t);
template void wx_rtr_batch_run_L<float, CELES_WX_L>(const WxArgs<float>*, const int*, const int*, const int*, int,
                                                    int*, int, int, hipStream_t);

template <typename T, int L>
void wx_rtr_run_L(const WxArgs<T>& a, int hmode, int nchunk, hipStream_t s) {
    dim3 grid((a.n + rtr::BLOCK - 1) / rtr::BLOCK, nchunk, 2 * a.nrhs);
    if (hmode == 0)
        hipLaunchKernelGGL((rtr::wx_rtr_kernel<T, L, 0>), grid, dim3(rtr::BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL((rtr::wx_rtr_kernel<T, L, 1>), grid, dim3(rtr::BLOCK), 0, s, a);
}
template void wx_rtr_run_L<double, CELES_WX_L>(const WxArgs<double>&, int, int, hipStream_t);
template void wx_rtr_run_L<float, CELES_WX_L>(const WxArgs<float>&, int, int, hipStream_t);

}  // namespace celes

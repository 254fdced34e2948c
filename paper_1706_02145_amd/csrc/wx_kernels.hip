// Coupling mat-vec W x evaluated on the fly (paper, Section 2.2 eq. a and
// Section 3.2.2), hand-written for gfx950.
//
// Mapping.  One lane = one receiving sphere i; a wave walks a contiguous
// chunk of source spheres i' that is uniform across the wave, so all source
// data (position and the source coefficients) comes in through scalar loads
// and the VALU works only on per-lane pair quantities.  Work on one pair is
// split into passes by the receiving |m| = M0 (a kernel instantiation per
// pass): a pass keeps only its own accumulators live, which is what lets the
// FP64 L = 4 kernel run without spilling, and it reuses every reduced
// translation coefficient for m = +M0 and m = -M0.
//
// Polarisation structure.  With x_1, x_2 the tau = 1, 2 halves of a source
// vector, the block [[A, B], [B, A]] acts as (A + B)(x_1 + x_2) and
// (A - B)(x_1 - x_2).  The kernels therefore consume s = x_1 + x_2 and
// d = x_1 - x_2 and produce y_1 + y_2 and y_1 - y_2; prep/finish kernels
// convert.  b5 is purely imaginary (b5 = i b5im), so A +- B = A +- i B'.
//
// Split over sources.  Each (receiver tile, source chunk) writes its partial
// sums to part[chunk][k][i]; wx_finish reduces over chunks in a fixed order
// (deterministic), converts back to (tau, l, m) and applies the optional
// y = x - T (W x) epilogue of eq. M.
#include <hip/hip_runtime.h>
#include <type_traits>

#include "device_common.hpp"
#include "wx_plan.hpp"
#include "wx_launch.hpp"

#define WX_BLOCK WX_BLOCK_SIZE   // receivers per block (4 waves share one source tile)
#define WX_TILE WX_TILE_SIZE     // sources per LDS tile

// This translation unit instantiates the kernels of one multipole cut-off,
// CELES_WX_L, so that the cut-offs compile in parallel.
#ifndef CELES_WX_L
#error "define CELES_WX_L (1..6)"
#endif

namespace celes {

using namespace plan;

// compile-time loop: f(integral_constant<int, B>), ..., f(integral_constant<int, E-1>)
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

// ---------------------------------------------------------------------------
// spherical Hankel functions h_p(kd), p = 0..2L
// ---------------------------------------------------------------------------
template <typename T, int P>
__device__ __forceinline__ void hankel_direct(double kd, cx<T> (&h)[P + 1]) {
    // h_0 = -i e^{ix}/x, h_1 = -e^{ix}(x + i)/x^2, h_{p+1} = (2p+1)/x h_p - h_{p-1}
    double s, c;
    sincos(kd, &s, &c);
    double inv = 1.0 / kd;
    double h0r = s * inv, h0i = -c * inv;
    double h1r = (h0r - c) * inv;   // (s/x - c)/x
    double h1i = (h0i - s) * inv;   // (-c/x - s)/x
    if constexpr (sizeof(T) == 8) {
        h[0] = {h0r, h0i};
        if constexpr (P >= 1) h[1] = {h1r, h1i};
#pragma unroll
        for (int p = 1; p < P; ++p) {
            double f = (2.0 * p + 1.0) * inv;
            h[p + 1] = {f * h[p].re - h[p - 1].re, f * h[p].im - h[p - 1].im};
        }
    } else {
        float fi = (float)inv;
        h[0] = {(float)h0r, (float)h0i};
        if constexpr (P >= 1) h[1] = {(float)h1r, (float)h1i};
#pragma unroll
        for (int p = 1; p < P; ++p) {
            float f = (2.0f * p + 1.0f) * fi;
            h[p + 1] = {f * h[p].re - h[p - 1].re, f * h[p].im - h[p - 1].im};
        }
    }
}

template <typename T, int P>
__device__ __forceinline__ void hankel_lut(double d, double inv_kd, const LutView<T>& lut, cx<T> (&h)[P + 1]) {
    // h_0 and h_1: cubic Hermite on [d_q, d_q + dr], coefficients in Horner
    // order c0..c3 of t (one 128-byte row per interval in FP64); higher
    // orders by the upward recurrence, as in hankel_direct
    double s = (d - lut.d_lo) * lut.inv_dr;
    int q = (int)s;
    q = q < 0 ? 0 : (q >= lut.n_int ? lut.n_int - 1 : q);
    T t = (T)(s - (double)q);
    const cx<T>* c = lut.coef + (size_t)q * 8;
#pragma unroll
    for (int p = 0; p <= (P < 1 ? P : 1); ++p) {
        cx<T> c0 = c[4 * p], c1 = c[4 * p + 1], c2 = c[4 * p + 2], c3 = c[4 * p + 3];
        h[p].re = fma(fma(fma(c3.re, t, c2.re), t, c1.re), t, c0.re);
        h[p].im = fma(fma(fma(c3.im, t, c2.im), t, c1.im), t, c0.im);
    }
    const T fi = (T)inv_kd;
#pragma unroll
    for (int p = 1; p < P; ++p) {
        T f = (T)(2 * p + 1) * fi;
        h[p + 1] = {f * h[p].re - h[p - 1].re, f * h[p].im - h[p - 1].im};
    }
}

// ---------------------------------------------------------------------------
// accumulation of one receiving |m| = M0 for one (mu, Legendre column) step
// ---------------------------------------------------------------------------
template <typename T, int L, int KB, int M0, int mu>
__device__ __forceinline__ void pass_mu_step(const cx<T>* xs, const cx<T> (&H)[2 * L + 1], cx<T> emu,
                                             cx<T> (&accP)[KB][L], cx<T> (&accM)[KB][L], cx<T> (&accPm)[KB][L],
                                             cx<T> (&accMm)[KB][L]) {
    constexpr int HALF = L * (L + 2);
    constexpr int LLO = l_lo(M0);
    constexpr bool MIRROR = M0 > 0;
    sfor<0, 2>([&](auto SG_) {
        constexpr int sgn = decltype(SG_)::value == 0 ? 1 : -1;
        if constexpr (branch(L, M0, mu, sgn)) {
            constexpr int mp = M0 + sgn * mu;
            constexpr bool two = MIRROR || mu > 0;
            const cx<T> rot = sgn > 0 ? emu : cx<T>{emu.re, -emu.im};
            const cx<T> rotc = {rot.re, -rot.im};
            sfor<lp_lo(mp), L + 1>([&](auto LP_) {
                constexpr int lp = decltype(LP_)::value;
                // keep the group's LDS reads next to their use (bounded live range)
                __builtin_amdgcn_sched_barrier(0);
                // source coefficients of (l', m') and of the mirror (l', -m'),
                // for each right-hand side of the block (tile row = [KB][2 HALF])
                cx<T> ts[KB], td[KB], us[KB], ud[KB];
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const cx<T>* xk = xs + kb * (2 * HALF);
                    ts[kb] = cmul(rot, xk[lp * (lp + 1) + mp - 1]);
                    td[kb] = cmul(rot, xk[HALF + lp * (lp + 1) + mp - 1]);
                    if constexpr (two) {
                        us[kb] = cmul(rotc, xk[lp * (lp + 1) - mp - 1]);
                        ud[kb] = cmul(rotc, xk[HALF + lp * (lp + 1) - mp - 1]);
                    }
                }
                sfor<LLO, L + 1>([&](auto LL_) {
                    constexpr int l = decltype(LL_)::value;
                    constexpr int pa0 = pa_lo(l, lp, mu), nA = na(l, lp, mu);
                    constexpr int pb0 = pb_lo(l, lp, mu), nB = nb(l, lp, mu);
                    cx<T> A = {0, 0}, B = {0, 0};
                    sfor<0, nA>([&](auto QA_) {
                        constexpr int t = decltype(QA_)::value;
                        constexpr double cv = ca5(lp, mp, l, M0, pa0 + 2 * t);
                        const T c = (T)cv;
                        A.re = fma(c, H[pa0 + 2 * t].re, A.re);
                        A.im = fma(c, H[pa0 + 2 * t].im, A.im);
                    });
                    sfor<0, nB>([&](auto QB_) {
                        constexpr int t = decltype(QB_)::value;
                        constexpr double cv = cb5im(lp, mp, l, M0, pb0 + 2 * t);
                        const T c = (T)cv;
                        B.re = fma(c, H[pb0 + 2 * t].re, B.re);
                        B.im = fma(c, H[pb0 + 2 * t].im, B.im);
                    });
                    // P = A + iB, Q = A - iB
                    const cx<T> Pv = {A.re - B.im, A.im + B.re};
                    const cx<T> Qv = {A.re + B.im, A.im - B.re};
                    constexpr int q = l - LLO;
#pragma unroll
                    for (int kb = 0; kb < KB; ++kb) {
                        cfma(accP[kb][q], Pv, ts[kb]);
                        cfma(accM[kb][q], Qv, td[kb]);
                        if constexpr (MIRROR) {
                            cfma(accPm[kb][q], Qv, us[kb]);
                            cfma(accMm[kb][q], Pv, ud[kb]);
                        } else if constexpr (two) {
                            cfma(accP[kb][q], Qv, us[kb]);
                            cfma(accM[kb][q], Pv, ud[kb]);
                        }
                    }
                });
            });
        }
    });
}

// partial sums: part[chunk][k][kk][i] for right-hand side k = k0 + kb
template <typename T, int L, int KB, int M0>
__device__ __forceinline__ void pass_store(const WxArgs<T>& a, int chunk, int k0, int i,
                                           const cx<T> (&accP)[KB][L], const cx<T> (&accM)[KB][L],
                                           const cx<T> (&accPm)[KB][L], const cx<T> (&accMm)[KB][L]) {
    constexpr int HALF = L * (L + 2);
    constexpr int LLO = l_lo(M0);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        cx<T>* out = a.part + ((size_t)chunk * a.nrhs + k0 + kb) * (2 * HALF) * a.ldp;
#pragma unroll
        for (int l = LLO; l <= L; ++l) {
            const int q = l - LLO;
            out[(size_t)(l * (l + 1) + M0 - 1) * a.ldp + i] = accP[kb][q];
            out[(size_t)(HALF + l * (l + 1) + M0 - 1) * a.ldp + i] = accM[kb][q];
            if constexpr (M0 > 0) {
                out[(size_t)(l * (l + 1) - M0 - 1) * a.ldp + i] = accPm[kb][q];
                out[(size_t)(HALF + l * (l + 1) - M0 - 1) * a.ldp + i] = accMm[kb][q];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// one group of passes (receiving |m| = MA, and MB >= 0 if present) of the
// coupling mat-vec over one (receiver tile, source chunk); the pair
// geometry, the Hankel functions and the Legendre columns are computed once
// per pair and shared by the passes of the group
// ---------------------------------------------------------------------------
template <typename T, int L, int KB, int HMODE, int MA, int MB>
__device__ __forceinline__ void wx_group(const WxArgs<T>& a, cx<T>* tile, int k0, int bx, int chunk) {
    constexpr int HALF = L * (L + 2);
    constexpr int P2 = 2 * L;
    constexpr bool HASB = MB >= 0;
    constexpr int MUMAX = HASB ? imax(mu_max(L, MA), mu_max(L, MB)) : mu_max(L, MA);

    const int i = bx * WX_BLOCK + threadIdx.x;
    const bool active = i < a.n;
    const double xi = active ? a.px[i] : 0.0;
    const double yi = active ? a.py[i] : 0.0;
    const double zi = active ? a.pz[i] : 0.0;

    cx<T> aP[KB][L], aM[KB][L], aPm[KB][L], aMm[KB][L];
    cx<T> bP[KB][L], bM[KB][L], bPm[KB][L], bMm[KB][L];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int q = 0; q < L; ++q) {
            aP[kb][q] = aM[kb][q] = aPm[kb][q] = aMm[kb][q] = {0, 0};
            bP[kb][q] = bM[kb][q] = bPm[kb][q] = bMm[kb][q] = {0, 0};
        }

    const int j0 = chunk * a.chunk_len;
    const int j1 = min(a.n, j0 + a.chunk_len);
    for (int t0 = j0; t0 < j1; t0 += WX_TILE) {
        const int nt = min(WX_TILE, j1 - t0);
        __syncthreads();
        {
            // tile[jj][kb][e] <- xsd[t0 + jj][k0 + kb][e]  (xsd is [N][nrhs][2 HALF])
            const int row = KB * 2 * HALF;
            for (int e = threadIdx.x; e < nt * row; e += WX_BLOCK) {
                const int jj = e / row, r = e % row;
                tile[e] = a.xsd[((size_t)(t0 + jj) * a.nrhs + k0) * (2 * HALF) + r];
            }
        }
        __syncthreads();
        for (int jj = 0; jj < nt; ++jj) {
            const int j = t0 + jj;
            if (!active || j == i) continue;
            // ---- pair geometry (FP64) ----
            const double dx = xi - a.px[j], dy = yi - a.py[j], dz = zi - a.pz[j];
            const double rho2 = dx * dx + dy * dy;
            const double r = sqrt(rho2 + dz * dz);
            const double inv_r = 1.0 / r;
            const double rho = sqrt(rho2);
            const T ct = (T)(dz * inv_r), st = (T)(rho * inv_r);
            T cph = 1, sph = 0;
            if (rho > 0.0) {
                const double ir = 1.0 / rho;
                cph = (T)(dx * ir);
                sph = (T)(dy * ir);
            }
            // ---- radial functions ----
            cx<T> h[P2 + 1];
            if constexpr (HMODE == 0)
                hankel_lut<T, P2>(r, inv_r * a.lut.inv_k, a.lut, h);
            else
                hankel_direct<T, P2>(a.k * r, h);

            const cx<T>* xs = tile + jj * (KB * 2 * HALF);
            const cx<T> e1 = {cph, sph};
            cx<T> emu = {1, 0};
            T pmm = (T)0.70710678118654752440;   // P_0^0
            sfor<0, MUMAX + 1>([&](auto MU_) {
                constexpr int mu = decltype(MU_)::value;
                if constexpr (mu > 0) {
                    constexpr double cd = leg_diag(mu);
                    pmm = (T)cd * st * pmm;
                    emu = cmul(emu, e1);
                }
                // Legendre column P_p^mu, p = mu..2L, and H_p = h_p P_p^mu
                T Pc[P2 + 1];
                cx<T> H[P2 + 1];
                sfor<mu, P2 + 1>([&](auto PP_) {
                    constexpr int p = decltype(PP_)::value;
                    if constexpr (p == mu) {
                        Pc[p] = pmm;
                    } else if constexpr (p == mu + 1) {
                        constexpr double cs = leg_sub(mu);
                        Pc[p] = (T)cs * ct * pmm;
                    } else {
                        constexpr double ca = leg_a(p, mu), cb = leg_b(p, mu);
                        Pc[p] = (T)ca * ct * Pc[p - 1] - (T)cb * Pc[p - 2];
                    }
                    H[p] = {h[p].re * Pc[p], h[p].im * Pc[p]};
                });
                if constexpr (mu <= mu_max(L, MA)) pass_mu_step<T, L, KB, MA, mu>(xs, H, emu, aP, aM, aPm, aMm);
                if constexpr (HASB) {
                    if constexpr (mu <= mu_max(L, MB)) pass_mu_step<T, L, KB, MB, mu>(xs, H, emu, bP, bM, bPm, bMm);
                }
            });
        }
    }
    if (!active) return;
    pass_store<T, L, KB, MA>(a, chunk, k0, i, aP, aM, aPm, aMm);
    if constexpr (HASB) pass_store<T, L, KB, MB>(a, chunk, k0, i, bP, bM, bPm, bMm);
}

// Pass groups per cut-off, heaviest first (blockIdx.z indexes the group, so
// the heaviest blocks are dispatched first).  Groups share one pair set-up;
// each combines passes so that the groups carry about equal work and no more
// accumulators than the |m| = 1 pass alone (FP64: within 256 VGPRs, two
// waves per SIMD).  Per-pair work of pass M0 at L = 4, in flops: 3036, 5648,
// 4428, 3120, 1816 for M0 = 0..4, hence {0,3}, {2,4}, {1}.
template <int L>
struct Groups;
template <> struct Groups<1> { static constexpr int n = 1; static constexpr int a[1] = {0}; static constexpr int b[1] = {1}; };
template <> struct Groups<2> { static constexpr int n = 2; static constexpr int a[2] = {0, 1}; static constexpr int b[2] = {2, -1}; };
template <> struct Groups<3> { static constexpr int n = 3; static constexpr int a[3] = {1, 0, 2}; static constexpr int b[3] = {-1, 3, -1}; };
template <> struct Groups<4> { static constexpr int n = 3; static constexpr int a[3] = {2, 0, 1}; static constexpr int b[3] = {4, 3, -1}; };
template <> struct Groups<5> { static constexpr int n = 4; static constexpr int a[4] = {3, 2, 1, 0}; static constexpr int b[4] = {4, 5, -1, -1}; };
template <> struct Groups<6> { static constexpr int n = 4; static constexpr int a[4] = {3, 2, 0, 1}; static constexpr int b[4] = {5, 6, 4, -1}; };

// blockIdx.z = g + G * kblock: pass group g, right-hand sides kblock*KB .. +KB
template <typename T, int L, int KB, int HMODE>
__global__ __launch_bounds__(WX_BLOCK) void wx_fused_kernel(WxArgs<T> a) {
    constexpr int HALF = L * (L + 2);
    // source tile staged in LDS; every lane reads the same element (broadcast)
    __shared__ cx<T> tile[WX_TILE * KB * 2 * HALF];
    const int g = blockIdx.z % Groups<L>::n;
    const int k0 = (blockIdx.z / Groups<L>::n) * KB;
    sfor<0, Groups<L>::n>([&](auto G_) {
        constexpr int gi = decltype(G_)::value;
        if (g == gi) wx_group<T, L, KB, HMODE, Groups<L>::a[gi], Groups<L>::b[gi]>(a, tile, k0, blockIdx.x, blockIdx.y);
    });
}

// Persistent multi-problem variant: the grid is sized to the machine and
// every block repeatedly claims the next work item (problem p, receiver
// tile, source chunk, pass group, right-hand-side block) from a counter.
// Items of problem p are numbered [item_off[p], item_off[p+1]); the counter
// must be zero at launch.  Every block exits once the counter passes the
// last item.
template <typename T, int L, int KB, int HMODE>
__global__ __launch_bounds__(WX_BLOCK) void wx_batch_kernel(const WxArgs<T>* __restrict__ args,
                                                            const int* __restrict__ item_off,
                                                            const int* __restrict__ nbx,
                                                            const int* __restrict__ nchunk, int nprob,
                                                            int* __restrict__ counter) {
    constexpr int HALF = L * (L + 2);
    constexpr int G = Groups<L>::n;
    __shared__ cx<T> tile[WX_TILE * KB * 2 * HALF];
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
        const int g = z % G, k0 = (z / G) * KB;
        const WxArgs<T> a = args[p];
        if (a.active) {
            bool any = false;
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) any = any || a.active[a.sys0 + k0 + kb] != 0;
            if (!any) continue;
        }
        sfor<0, G>([&](auto G_) {
            constexpr int gi = decltype(G_)::value;
            if (g == gi) wx_group<T, L, KB, HMODE, Groups<L>::a[gi], Groups<L>::b[gi]>(a, tile, k0, bx, chunk);
        });
    }
}

template <typename T, int L, int KB>
static void launch_batch_kb(const WxArgs<T>* args, const int* item_off, const int* nbx, const int* nchunk,
                            int nprob, int* counter, int nblocks, int hmode, hipStream_t s) {
    if (hmode == 0)
        hipLaunchKernelGGL((wx_batch_kernel<T, L, KB, 0>), dim3(nblocks), dim3(WX_BLOCK), 0, s, args, item_off, nbx,
                           nchunk, nprob, counter);
    else
        hipLaunchKernelGGL((wx_batch_kernel<T, L, KB, 1>), dim3(nblocks), dim3(WX_BLOCK), 0, s, args, item_off, nbx,
                           nchunk, nprob, counter);
}

// right-hand-side block widths compiled per precision and cut-off
template <typename T, int L>
constexpr int max_kb() {
    if constexpr (L > 4) return 1;
    else if constexpr (sizeof(T) == 8) return L <= 3 ? 2 : 1;
    else return 4;
}

template <typename T, int L, int KB>
static void launch_kb(const WxArgs<T>& a, int hmode, int nchunk, hipStream_t s) {
    dim3 grid((a.n + WX_BLOCK - 1) / WX_BLOCK, nchunk, Groups<L>::n * (a.nrhs / KB));
    if (hmode == 0)
        hipLaunchKernelGGL((wx_fused_kernel<T, L, KB, 0>), grid, dim3(WX_BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL((wx_fused_kernel<T, L, KB, 1>), grid, dim3(WX_BLOCK), 0, s, a);
}

template <typename T, int L>
void wx_run_L(const WxArgs<T>& a, int hmode, int nchunk, hipStream_t s) {
    // a.kb has been chosen by the host among 1, 2, 4 (<= max_kb) and divides a.nrhs
    if constexpr (max_kb<T, L>() >= 4) {
        if (a.kb == 4) return launch_kb<T, L, 4>(a, hmode, nchunk, s);
    }
    if constexpr (max_kb<T, L>() >= 2) {
        if (a.kb == 2) return launch_kb<T, L, 2>(a, hmode, nchunk, s);
    }
    launch_kb<T, L, 1>(a, hmode, nchunk, s);
}

// batches are compiled for cut-offs up to 4 (the persistent kernel would
// double the compile time of the larger cut-offs)
template <typename T, int L>
void wx_batch_run_L(const WxArgs<T>* args, const int* item_off, const int* nbx, const int* nchunk, int nprob,
                    int* counter, int nblocks, int kb, int hmode, hipStream_t s) {
    if constexpr (L > 4) {
        return;
    } else {
    if constexpr (max_kb<T, L>() >= 4) {
        if (kb == 4) return launch_batch_kb<T, L, 4>(args, item_off, nbx, nchunk, nprob, counter, nblocks, hmode, s);
    }
    if constexpr (max_kb<T, L>() >= 2) {
        if (kb == 2) return launch_batch_kb<T, L, 2>(args, item_off, nbx, nchunk, nprob, counter, nblocks, hmode, s);
    }
    launch_batch_kb<T, L, 1>(args, item_off, nbx, nchunk, nprob, counter, nblocks, hmode, s);
    }
}
template void wx_batch_run_L<double, CELES_WX_L>(const WxArgs<double>*, const int*, const int*, const int*, int, int*,
                                                 int, int, int, hipStream_t);
template void wx_batch_run_L<float, CELES_WX_L>(const WxArgs<float>*, const int*, const int*, const int*, int, int*,
                                                int, int, int, hipStream_t);

template <typename T, int L>
int wx_max_kb_L() { return max_kb<T, L>(); }
template int wx_max_kb_L<double, CELES_WX_L>();
template int wx_max_kb_L<float, CELES_WX_L>();

template <int L>
int wx_num_groups_L() { return Groups<L>::n; }
template int wx_num_groups_L<CELES_WX_L>();

template void wx_run_L<double, CELES_WX_L>(const WxArgs<double>&, int, int, hipStream_t);
template void wx_run_L<float, CELES_WX_L>(const WxArgs<float>&, int, int, hipStream_t);

}  // namespace celes

// Coupling mat-vec W x for a block of right-hand sides on the matrix cores
// (paper, Section 2.2 eq. a and Section 3.2.2; complex64, lmax <= 4).
//
// Mapping.  One wave = one receiving sphere i; the four waves of a block share
// the LDS-staged source vectors of a tile of sources.  For every pair (i, j)
// the wave
//   1. evaluates the pair geometry, h_p(kd), the Legendre columns and the
//      azimuthal phases once (wave-uniform) and leaves H_p^mu = h_p P_p^mu and
//      e^{ik phi} in a wave-private LDS area;
//   2. builds the two reduced HALF x HALF blocks
//        P = e^{i(m'-m) phi} (A~ + i B~),   Q = e^{i(m'-m) phi} (A~ - i B~),
//      A~ = sum_p a5(l',m'|l,m|p) H_p^{|m'-m|}, B~ likewise with b5 / i,
//      lane-parallel from a host-built record table, and writes them in real
//      form [[Re, -Im], [Im, Re]] into LDS in matrix-core operand order.  One
//      record serves an entry and its mirror (m, m' -> -m, -m'): a5 is even
//      and b5 odd under the mirror (Appendix A.2), so with Y = A~ + i B~ and
//      X = A~ - i B~ the mirror entry has P = conj(ph) X and Q = conj(ph) Y;
//   3. applies P to the source's s = x1 + x2 and Q to d = x1 - x2 for all the
//      block's right-hand sides: two (R x R) x (R x KN) real products,
//      R = 2 HALF rounded up to 16, with v_mfma_f32_16x16x4f32, accumulating
//      in registers over the source chunk.
// The partial sums go to the layout of the VALU kernels and are reduced by the
// same finish kernel.
#include <hip/hip_runtime.h>
#include <type_traits>

#include "device_common.hpp"
#include "wx_plan.hpp"
#include "wx_mfma.hpp"

namespace celes {

using namespace plan;

typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

template <int B, int E, typename F>
__device__ __forceinline__ void mfor(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        mfor<B + 1, E>(f);
    }
}

// Two operand forms.  Real form: the complex HALF x HALF block as one real
// matrix [[Re, -Im], [Im, Re]] of order R = 2 HALF (padded to 16), one
// product with [Re x; Im x].  Three-product form (Gauss), used where the
// complex order pads to 16 with little waste (lmax 3: HALF = 15): the three
// real products Re(P) Re(x), Im(P) Im(x) and (Re P + Im P)(Re x + Im x) of
// order HALF padded to 16 give Re = T1 - T2 and Im = T3 - T1 - T2 with three
// quarters of the real-form multiplies.
template <int L>
struct MShape {
    static constexpr int HALF = L * (L + 2);
    static constexpr bool G3 = L == 3;                     // three-product form
    static constexpr int NMAT = G3 ? 3 : 1;                // operand matrices per half
    static constexpr int NMX = G3 ? 2 : 1;                 // source matrices staged per half (Re + Im
                                                           // of the three-product form is formed in registers)
    static constexpr int R = G3 ? (HALF + 15) / 16 * 16 : (2 * HALF + 15) / 16 * 16;   // matrix order
    static constexpr int MT = R / 16;                      // 16-row tiles
    static constexpr int KS = R / 4;                       // k-steps of 4
    static constexpr int KQ = KS / 4;                      // float4 groups of k-steps
    static constexpr int MSZ = MT * 64 * KS;               // floats of one operand matrix
    static constexpr int E = HALF * HALF;                  // reduced block entries
    static constexpr int P2 = 2 * L;
    static constexpr int HS = wxm_h_stride(L);             // H row stride: p = 0..2L
    static constexpr int NPH = 4 * L + 1;                  // e^{ik phi}, k = -2L..2L
    static constexpr int TA = L + 1, TB = L;               // padded term counts of A~ and B~
    static constexpr int EC = (E + L * L) / 2;             // records: entry pairs under the mirror
    static_assert(KS % 4 == 0, "k-steps come in float4 groups");
    static_assert(5 + TA + TB <= WXM_REC, "record too short");
    static_assert(NMAT * MSZ <= 65536, "operand offsets must fit 16 bits");
};

// h_p(kd), p = 0..2L, in FP32 from the FP64 distance: h_0, h_1 from the
// two-order table (HMODE 0) or from sin/cos (HMODE 1), higher orders by the
// upward recurrence h_{p+1} = (2p+1)/x h_p - h_{p-1}
template <int L, int HMODE>
__device__ __forceinline__ void pair_hankel(double r, double inv_r, const WxMfmaArgs& a, cx<float> (&h)[2 * L + 1]) {
    constexpr int P = 2 * L;
    float fi;
    if constexpr (HMODE == 0) {
        const double s = (r - a.lut.d_lo) * a.lut.inv_dr;
        int q = (int)s;
        q = q < 0 ? 0 : (q >= a.lut.n_int ? a.lut.n_int - 1 : q);
        const float t = (float)(s - (double)q);
        const cx<float>* c = a.lut.coef + (size_t)q * 8;
#pragma unroll
        for (int p = 0; p <= 1; ++p) {
            const cx<float> c0 = c[4 * p], c1 = c[4 * p + 1], c2 = c[4 * p + 2], c3 = c[4 * p + 3];
            h[p].re = fmaf(fmaf(fmaf(c3.re, t, c2.re), t, c1.re), t, c0.re);
            h[p].im = fmaf(fmaf(fmaf(c3.im, t, c2.im), t, c1.im), t, c0.im);
        }
        fi = (float)(inv_r * a.lut.inv_k);
    } else {
        const double kd = a.k * r;
        double s, c;
        sincos(kd, &s, &c);
        const double inv = 1.0 / kd;
        const double h0r = s * inv, h0i = -c * inv;
        h[0] = {(float)h0r, (float)h0i};
        h[1] = {(float)((h0r - c) * inv), (float)((h0i - s) * inv)};
        fi = (float)inv;
    }
#pragma unroll
    for (int p = 1; p < P; ++p) {
        const float f = (float)(2 * p + 1) * fi;
        h[p + 1] = {f * h[p].re - h[p - 1].re, f * h[p].im - h[p - 1].im};
    }
}

// one block-entry record, decoded: H offsets of the first A~ / B~ terms,
// phase index, mirror flag, packed operand offsets, coefficients
template <int L>
struct EntryRec {
    int head, w01, w23, m01, m23;
    float c[2 * L + 1];
};

template <int L>
__device__ __forceinline__ void load_rec(const float* r, EntryRec<L>& e) {
    e.head = __float_as_int(r[0]);
    e.w01 = __float_as_int(r[1]);
    e.w23 = __float_as_int(r[2]);
    e.m01 = __float_as_int(r[3]);
    e.m23 = __float_as_int(r[4]);
#pragma unroll
    for (int q = 0; q <= 2 * L; ++q) e.c[q] = r[5 + q];
}

// P, Q of one record (and of its mirror) into the wave's real-form operands
template <int L>
__device__ __forceinline__ void build_entry(const EntryRec<L>& e, const cx<float>* sh, const cx<float>* sp, float* aP,
                                            float* aQ) {
    constexpr int TA = L + 1, TB = L;
    const int hA = e.head & 1023, hB = (e.head >> 10) & 1023, iph = (e.head >> 20) & 1023;
    cx<float> A = {0.f, 0.f}, B = {0.f, 0.f};
#pragma unroll
    for (int q = 0; q < TA; ++q) {
        const cx<float> hh = sh[hA + 2 * q];
        A.re = fmaf(e.c[q], hh.re, A.re);
        A.im = fmaf(e.c[q], hh.im, A.im);
    }
#pragma unroll
    for (int q = 0; q < TB; ++q) {
        const cx<float> hh = sh[hB + 2 * q];
        B.re = fmaf(e.c[TA + q], hh.re, B.re);
        B.im = fmaf(e.c[TA + q], hh.im, B.im);
    }
    const cx<float> ph = sp[iph];
    const cx<float> Y = {A.re - B.im, A.im + B.re};   // A~ + i B~
    const cx<float> X = {A.re + B.im, A.im - B.re};   // A~ - i B~
    // real-form positions (n, n'), (n+H, n'+H) <- Re; (n, n'+H) <- -Im; (n+H, n') <- Im
    auto put = [&](int w01, int w23, cx<float> vp, cx<float> vq) {
        const int o0 = w01 & 0xffff, o1 = (int)((unsigned)w01 >> 16);
        const int o2 = w23 & 0xffff, o3 = (int)((unsigned)w23 >> 16);
        aP[o0] = vp.re;
        aP[o1] = vp.re;
        aP[o2] = -vp.im;
        aP[o3] = vp.im;
        aQ[o0] = vq.re;
        aQ[o1] = vq.re;
        aQ[o2] = -vq.im;
        aQ[o3] = vq.im;
    };
    if constexpr (MShape<L>::G3) {
        // three-product form: Re, Im and Re + Im at one offset of three matrices
        constexpr int M1 = MShape<L>::MSZ;
        auto put3 = [&](int o, cx<float> vp, cx<float> vq) {
            aP[o] = vp.re;
            aP[o + M1] = vp.im;
            aP[o + 2 * M1] = vp.re + vp.im;
            aQ[o] = vq.re;
            aQ[o + M1] = vq.im;
            aQ[o + 2 * M1] = vq.re + vq.im;
        };
        put3(e.w01, cmul(ph, Y), cmul(ph, X));
        if ((e.head >> 30) & 1) {
            const cx<float> phc = {ph.re, -ph.im};
            put3(e.m01, cmul(phc, X), cmul(phc, Y));
        }
    } else {
        put(e.w01, e.w23, cmul(ph, Y), cmul(ph, X));
        if ((e.head >> 30) & 1) {
            const cx<float> phc = {ph.re, -ph.im};
            put(e.m01, e.m23, cmul(phc, X), cmul(phc, Y));
        }
    }
}

template <int L, int NT, int HMODE>
__global__ __launch_bounds__(256) void wx_mfma_kernel(WxMfmaArgs a) {
    using S = MShape<L>;
    constexpr int HALF = S::HALF, MT = S::MT, KS = S::KS, KQ = S::KQ, P2 = S::P2, NMAT = S::NMAT;
    constexpr int HS = S::HS, NPH = S::NPH, EC = S::EC;
    constexpr int KN = 16 * NT;                 // right-hand sides per block
    constexpr int TS = 2;                       // sources per staged tile of B operands
    // sources per set-up tile: one per lane group of GW = 64 / TSU >= 2L + 1
    // lanes; 4 for the narrower blocks, whose occupancy larger tables would cut
    constexpr int TSU = NT == 4 && P2 + 1 <= 8 ? 8 : 4;
    constexpr int GW = 64 / TSU;
    static_assert(GW >= P2 + 1, "a lane group holds the 2L + 1 set-up lanes");
    constexpr int AH = NMAT * S::MSZ;           // floats of one block's operand matrices (R x R each)
    constexpr int XM = NT * 64 * KS;            // floats of one source operand matrix (R x KN)
    constexpr int XH = S::NMX * XM;             // floats of one staged source half
    constexpr int EPL = (EC + 63) / 64;         // records per lane
    constexpr bool REGREC = EPL <= 2;           // records live in registers (lmax <= 3)
    constexpr int HT = (P2 + 1) * HS;           // complex H entries per source
    constexpr int HTAIL = P2 + 1;               // zeroed entries after the last table (reads past a row)

    __shared__ __attribute__((aligned(16))) float s_rec[REGREC ? 4 : EC * WXM_REC];
    __shared__ __attribute__((aligned(16))) float s_x[TS * 2 * XH];
    __shared__ __attribute__((aligned(16))) float s_a[4 * 2 * AH];
    __shared__ cx<float> s_h[4 * TSU * HT + HTAIL];
    __shared__ cx<float> s_ph[4 * TSU * NPH];
    __shared__ double s_pos[TSU * 3];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int i = blockIdx.x * 4 + wv;
    const bool active = i < a.n;
    const int chunk = blockIdx.y;
    const int k0 = blockIdx.z * KN;
    if (a.active) {
        // batches: nothing to do once every system of this block has converged
        int any = 0;
        for (int c = 0; c < KN; ++c) any |= a.active[a.sys0 + k0 + c];
        if (!any) return;
    }

    if constexpr (!REGREC)
        for (int e = tid; e < EC * WXM_REC; e += 256) s_rec[e] = a.rec[e];
    for (int e = tid; e < 4 * 2 * AH; e += 256) s_a[e] = 0.f;          // padding rows / columns stay zero
    for (int e = tid; e < 4 * TSU * HT + HTAIL; e += 256) s_h[e] = {0.f, 0.f};

    float* const sa = s_a + wv * 2 * AH;
    cx<float>* const shw = s_h + wv * TSU * HT;
    cx<float>* const spw = s_ph + wv * TSU * NPH;

    // records of this lane (lmax <= 3): loaded once
    EntryRec<L> rr[REGREC ? EPL : 1];
    if constexpr (REGREC) {
#pragma unroll
        for (int t = 0; t < EPL; ++t) {
            const int e = lane + 64 * t;
            if (e < EC) load_rec<L>(a.rec + (size_t)e * WXM_REC, rr[t]);
            else rr[t] = EntryRec<L>{};
        }
    }

    // set-up lanes: lane group g = lane / GW serves source t0 + g of a set-up
    // tile; within it, lane gl = lane % GW <= 2L computes Legendre column
    // mu = gl and the phases e^{+-i gl phi}
    const int g = lane / GW, gl = lane % GW;
    float dg = 0.70710678118654752440f;
    for (int v = 1; v <= gl && v <= P2; ++v) dg *= sqrtf((2.f * v + 1.f) / (2.f * v));
    float la[P2 + 1], lb[P2 + 1];
#pragma unroll
    for (int p = 0; p <= P2; ++p) {
        const float pf = (float)p, mf = (float)gl;
        la[p] = p == gl + 1 ? sqrtf(2.f * mf + 3.f)
                            : (p > gl + 1 ? sqrtf((4.f * pf * pf - 1.f) / (pf * pf - mf * mf)) : 0.f);
        lb[p] = p > gl + 1 ? sqrtf((2.f * pf + 1.f) * ((pf - 1.f) * (pf - 1.f) - mf * mf) /
                                   ((2.f * pf - 3.f) * (pf * pf - mf * mf)))
                           : 0.f;
    }

    const double xi = active ? a.px[i] : 0.0;
    const double yi = active ? a.py[i] : 0.0;
    const double zi = active ? a.pz[i] : 0.0;

    v4f acc[2][NMAT * MT][NT];   // [half][operand matrix x row tile][column tile]
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int mt = 0; mt < NMAT * MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[h][mt][nt] = v4f{0.f, 0.f, 0.f, 0.f};

    const int j0 = chunk * a.chunk_len;
    const int j1 = min(a.n, j0 + a.chunk_len);
    // B operands of a staged tile (TS sources, a contiguous run of the
    // prep kernel's operand-ordered records).  For 64-wide blocks they pass
    // through registers: the next tile's are loaded while the current
    // tile's products run (the narrower blocks would lose a wave of
    // occupancy to the registers and copy directly)
    constexpr bool PREFETCH = NT == 4;
    constexpr int XQ = TS * 2 * XH / 4;         // float4 of a full staged tile
    constexpr int QPT = PREFETCH ? (XQ + 255) / 256 : 1;
    static_assert((2 * XH) % 4 == 0, "a source's operands are whole float4");
    float4 pre[QPT];
    if (PREFETCH && j0 < j1) {
        const int nq = min(TS, j1 - j0) * 2 * XH / 4;
        const float4* src = reinterpret_cast<const float4*>(a.xb + ((size_t)blockIdx.z * a.n + j0) * 2 * XH);
#pragma unroll
        for (int q = 0; q < QPT; ++q) pre[q] = tid + 256 * q < nq ? src[tid + 256 * q] : float4{0.f, 0.f, 0.f, 0.f};
    }
    for (int t0 = j0; t0 < j1; t0 += TSU) {
        const int nsu = min(TSU, j1 - t0);
        __syncthreads();
        // centres of the set-up tile
        if (tid < 3 * nsu) {
            const int jj = tid / 3, c = tid % 3;
            s_pos[tid] = (c == 0 ? a.px : c == 1 ? a.py : a.pz)[t0 + jj];
        }
        __syncthreads();
        // ---- set-up of the tile's pairs: geometry, h_p, H_p^mu = h_p P_p^mu, e^{ik phi} ----
        if (active && g < nsu && t0 + g != i && gl <= P2) {
            const double dx = xi - s_pos[3 * g], dy = yi - s_pos[3 * g + 1], dz = zi - s_pos[3 * g + 2];
            const double rho2 = dx * dx + dy * dy;
            const double r = sqrt(rho2 + dz * dz);
            const double inv_r = 1.0 / r;
            const double rho = sqrt(rho2);
            const float ct = (float)(dz * inv_r), st = (float)(rho * inv_r);
            float cph = 1.f, sph = 0.f;
            if (rho > 0.0) {
                const double ir = 1.0 / rho;
                cph = (float)(dx * ir);
                sph = (float)(dy * ir);
            }
            cx<float> hv[P2 + 1];
            pair_hankel<L, HMODE>(r, inv_r, a, hv);
            cx<float>* sh = shw + g * HT;
            float pw = 1.f;
#pragma unroll
            for (int q = 1; q <= P2; ++q) pw = q <= gl ? pw * st : pw;
            float p1 = 0.f, p2 = 0.f;
#pragma unroll
            for (int p = 0; p <= P2; ++p) {
                const float v = p == gl ? dg * pw : la[p] * ct * p1 - lb[p] * p2;
                p2 = p1;
                p1 = v;
                sh[gl * HS + p] = {hv[p].re * v, hv[p].im * v};
            }
            cx<float> ep = {1.f, 0.f};
            const cx<float> e1 = {cph, sph};
#pragma unroll
            for (int q = 1; q <= P2; ++q)
                if (q <= gl) ep = cmul(ep, e1);
            spw[g * NPH + 2 * L + gl] = ep;
            if (gl > 0) spw[g * NPH + 2 * L - gl] = {ep.re, -ep.im};
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
      for (int u0 = 0; u0 < nsu; u0 += TS) {
        const int ntile = min(TS, nsu - u0);
        __syncthreads();
        // B operands of the staged tile (fetched during the previous tile)
        {
            float4* dst = reinterpret_cast<float4*>(s_x);
            const int nq = ntile * 2 * XH / 4;
            if constexpr (PREFETCH) {
#pragma unroll
                for (int q = 0; q < QPT; ++q) {
                    const int idx = tid + 256 * q;
                    if (idx < nq) dst[idx] = pre[q];
                }
            } else {
                const float4* src =
                    reinterpret_cast<const float4*>(a.xb + ((size_t)blockIdx.z * a.n + t0 + u0) * 2 * XH);
                for (int idx = tid; idx < nq; idx += 256) dst[idx] = src[idx];
            }
        }
        __syncthreads();
        if (PREFETCH && t0 + u0 + TS < j1) {
            const int s0 = t0 + u0 + TS;
            const int nq = min(TS, j1 - s0) * 2 * XH / 4;
            const float4* src = reinterpret_cast<const float4*>(a.xb + ((size_t)blockIdx.z * a.n + s0) * 2 * XH);
#pragma unroll
            for (int q = 0; q < QPT; ++q)
                pre[q] = tid + 256 * q < nq ? src[tid + 256 * q] : float4{0.f, 0.f, 0.f, 0.f};
        }
        for (int jj = 0; jj < ntile; ++jj) {
            const int j = t0 + u0 + jj;
            if (!active || j == i) continue;
            const cx<float>* sh = shw + (u0 + jj) * HT;
            const cx<float>* sp = spw + (u0 + jj) * NPH;
            // ---- reduced block entries (record pairs), lane-parallel, into the real-form operands ----
#pragma unroll
            for (int t = 0; t < EPL; ++t) {
                const int e = lane + 64 * t;
                if (t < EPL - 1 || EC % 64 == 0 || e < EC) {
                    if constexpr (REGREC) {
                        build_entry<L>(rr[t], sh, sp, sa, sa + AH);
                    } else {
                        EntryRec<L> rc;
                        load_rec<L>(s_rec + e * WXM_REC, rc);
                        build_entry<L>(rc, sh, sp, sa, sa + AH);
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // ---- block products on the matrix cores: operand matrix mm of
            // the block against operand matrix mm of the source half ----
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if constexpr (S::G3) {
                    // Re P . Re x, Im P . Im x and (Re P + Im P)(Re x + Im x):
                    // the third source matrix is the sum of the two staged ones
                    float af[3][KS];
#pragma unroll
                    for (int mm = 0; mm < 3; ++mm)
#pragma unroll
                        for (int q = 0; q < KQ; ++q) {
                            const float4 v = *(const float4*)(sa + h * AH + mm * S::MSZ + lane * KS + 4 * q);
                            af[mm][4 * q] = v.x;
                            af[mm][4 * q + 1] = v.y;
                            af[mm][4 * q + 2] = v.z;
                            af[mm][4 * q + 3] = v.w;
                        }
                    const float* xb = s_x + (jj * 2 + h) * XH + lane * KS;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        float b0[KS], b1[KS];
#pragma unroll
                        for (int q = 0; q < KQ; ++q) {
                            const float4 u = *(const float4*)(xb + nt * 64 * KS + 4 * q);
                            const float4 v = *(const float4*)(xb + XM + nt * 64 * KS + 4 * q);
                            b0[4 * q] = u.x;
                            b0[4 * q + 1] = u.y;
                            b0[4 * q + 2] = u.z;
                            b0[4 * q + 3] = u.w;
                            b1[4 * q] = v.x;
                            b1[4 * q + 1] = v.y;
                            b1[4 * q + 2] = v.z;
                            b1[4 * q + 3] = v.w;
                        }
#pragma unroll
                        for (int ks = 0; ks < KS; ++ks) {
                            acc[h][0][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[0][ks], b0[ks], acc[h][0][nt], 0, 0, 0);
                            acc[h][1][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[1][ks], b1[ks], acc[h][1][nt], 0, 0, 0);
                            acc[h][2][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[2][ks], b0[ks] + b1[ks],
                                                                                 acc[h][2][nt], 0, 0, 0);
                        }
                    }
                    continue;
                }
#pragma unroll
                for (int mm = 0; mm < NMAT; ++mm) {
                    const float* ab = sa + h * AH + mm * S::MSZ + lane * KS;
                    float af[MT][KS];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int q = 0; q < KQ; ++q) {
                            const float4 v = *(const float4*)(ab + mt * 64 * KS + 4 * q);
                            af[mt][4 * q] = v.x;
                            af[mt][4 * q + 1] = v.y;
                            af[mt][4 * q + 2] = v.z;
                            af[mt][4 * q + 3] = v.w;
                        }
                    const float* xb = s_x + (jj * 2 + h) * XH + mm * XM + lane * KS;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        float bf[KS];
#pragma unroll
                        for (int q = 0; q < KQ; ++q) {
                            const float4 v = *(const float4*)(xb + nt * 64 * KS + 4 * q);
                            bf[4 * q] = v.x;
                            bf[4 * q + 1] = v.y;
                            bf[4 * q + 2] = v.z;
                            bf[4 * q + 3] = v.w;
                        }
#pragma unroll
                        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                            for (int mt = 0; mt < MT; ++mt)
                                acc[h][mm * MT + mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                    af[mt][ks], bf[ks], acc[h][mm * MT + mt][nt], 0, 0, 0);
                    }
                }
            }
        }
      }
    }
    if (!active) return;
    // lane holds C[16 mt + 4 (lane / 16) + t][16 nt + lane % 16]: real-form
    // row -> (half h, entry (l, m), real or imaginary part), column -> RHS
    float* pf = reinterpret_cast<float*>(a.part);
    if constexpr (S::G3) {
        // three-product form: row r = entry (l, m); Re = T1 - T2, Im = T3 - T1 - T2
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int e = 4 * (lane >> 4) + t;
                    if (e < HALF) {
                        const float t1 = acc[h][0][nt][t], t2 = acc[h][1][nt][t], t3 = acc[h][2][nt][t];
                        const int col = 16 * nt + (lane & 15);
                        const size_t o =
                            (((size_t)chunk * a.nrhs + k0 + col) * (2 * HALF) + h * HALF + e) * a.ldp + i;
                        pf[2 * o] = t1 - t2;
                        pf[2 * o + 1] = t3 - t1 - t2;
                    }
                }
        return;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int rr2 = 16 * mt + 4 * (lane >> 4) + t;
                    if (rr2 < 2 * HALF) {
                        const int e = rr2 < HALF ? rr2 : rr2 - HALF;
                        const int col = 16 * nt + (lane & 15);
                        const size_t o =
                            (((size_t)chunk * a.nrhs + k0 + col) * (2 * HALF) + h * HALF + e) * a.ldp + i;
                        pf[2 * o + (rr2 < HALF ? 0 : 1)] = acc[h][mt][nt][t];
                    }
                }
}

// x [K][N][nmax] (tau blocks, complex64) -> xb [K / KN][N][2][NT][64][KS]:
// for right-hand-side block z and source j, the real form of s = x1 + x2
// (h = 0) and d = x1 - x2 (h = 1) as B operands of v_mfma_f32_16x16x4f32:
// real-form row k (Re of entry k < HALF, Im of entry k - HALF below 2 HALF,
// zero padding above) of right-hand side col = 16 nt + c sits at lane
// (k % 4) 16 + c, k-step k / 4
// (three-product form: xb [K / KN][N][2][2][NT][64][KS], operand matrices
// Re and Im of the HALF entries, row k = entry k; the kernel forms Re + Im)
template <int L, int NT>
__global__ void wx_mfma_prep_kernel(const cx<float>* __restrict__ x0, const int* kstep, int kin, int64_t slot_stride,
                                    float* __restrict__ xb, int n, int K) {
    using S = MShape<L>;
    constexpr int HALF = S::HALF, KS = S::KS, KN = 16 * NT, NMX = S::NMX;
    constexpr int XH = NMX * NT * 64 * KS;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)(K / KN) * n * 2 * XH;
    if (t >= total) return;
    const cx<float>* x = x0 + (kstep ? (int64_t)(*kstep + kin) * slot_stride : 0);
    const int ks = (int)(t % KS);
    int64_t r = t / KS;
    const int ln = (int)(r % 64);
    r /= 64;
    const int nt = (int)(r % NT);
    r /= NT;
    const int mm = (int)(r % NMX);
    r /= NMX;
    const int h = (int)(r % 2);
    r /= 2;
    const int j = (int)(r % n);
    const int z = (int)(r / n);
    const int k = 4 * ks + (ln >> 4);
    const int col = z * KN + 16 * nt + (ln & 15);
    float v = 0.f;
    const int e = S::G3 ? k : (k < HALF ? k : k - HALF);
    if (S::G3 ? k < HALF : k < 2 * HALF) {
        const cx<float>* xr = x + ((size_t)col * n + j) * 2 * HALF;
        const cx<float> x1 = xr[e], x2 = xr[HALF + e];
        const cx<float> sd = h == 0 ? cx<float>{x1.re + x2.re, x1.im + x2.im} : cx<float>{x1.re - x2.re, x1.im - x2.im};
        if constexpr (S::G3) v = mm == 0 ? sd.re : sd.im;
        else v = k < HALF ? sd.re : sd.im;
    }
    xb[t] = v;
}

template <int L, int NT>
void launch_nt(const WxMfmaArgs& a, int hmode, int nchunk, hipStream_t s, const hipEvent_t* ev) {
    using S = MShape<L>;
    const int64_t total = (int64_t)(a.nrhs / (16 * NT)) * a.n * 2 * (S::NMX * NT * 64 * S::KS);
    hipLaunchKernelGGL((wx_mfma_prep_kernel<L, NT>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a.x,
                       a.kstep, a.kin, a.slot_stride, a.xb, a.n, a.nrhs);
    dim3 grid((unsigned)((a.n + 3) / 4), (unsigned)nchunk, (unsigned)(a.nrhs / (16 * NT)));
    if (ev) hipEventRecord(ev[0], s);
    if (hmode == 0)
        hipLaunchKernelGGL((wx_mfma_kernel<L, NT, 0>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((wx_mfma_kernel<L, NT, 1>), grid, dim3(256), 0, s, a);
    if (ev) hipEventRecord(ev[1], s);
}

template <int L>
void launch_L(const WxMfmaArgs& a, int width, int hmode, int nchunk, hipStream_t s, const hipEvent_t* ev) {
    if (width == 64) launch_nt<L, 4>(a, hmode, nchunk, s, ev);
    else if (width == 32) launch_nt<L, 2>(a, hmode, nchunk, s, ev);
    else launch_nt<L, 1>(a, hmode, nchunk, s, ev);
}

}  // namespace

size_t wx_mfma_xb_floats(int L, int64_t N, int K) {
    // per right-hand side and source half: R rows (real form) or 2 x 16 (three-product form, lmax 3:
    // Re and Im; the kernel forms Re + Im)
    const int rows = L == 3 ? 2 * 16 : (2 * L * (L + 2) + 15) / 16 * 16;
    return (size_t)2 * K * N * rows;
}

int wx_mfma_block(int L, int K, bool any) {
    if (L < 1 || L > WXM_MAX_L || K <= 0) return 0;
    if (K % 64 == 0) return 64;
    // measured on MI355X: 32-wide blocks beat the VALU kernel only up to
    // lmax 3, 16-wide blocks never (the per-pair block build is amortised
    // over too few right-hand sides)
    if (K % 32 == 0 && (any || L <= 3)) return 32;
    if (K % 16 == 0 && any) return 16;
    return 0;
}

int wx_mfma_launch(const WxMfmaArgs& a, int L, int width, int hmode, int nchunk, hipStream_t s,
                   const hipEvent_t* ev) {
    if (wx_mfma_block(L, a.nrhs, true) == 0 || (width != 16 && width != 32 && width != 64) || a.nrhs % width)
        return -1;
    switch (L) {
        case 1: launch_L<1>(a, width, hmode, nchunk, s, ev); break;
        case 2: launch_L<2>(a, width, hmode, nchunk, s, ev); break;
        case 3: launch_L<3>(a, width, hmode, nchunk, s, ev); break;
        case 4: launch_L<4>(a, width, hmode, nchunk, s, ev); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace celes

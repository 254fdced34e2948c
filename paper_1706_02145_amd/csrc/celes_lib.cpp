// Host side of the library: problem set-up, incident fields, the Krylov
// solvers that drive the device mat-vec, observables and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/celes.h"
#include "device_common.hpp"
#include "host_math.hpp"
#include "farfield.hpp"
#include "nearfield.hpp"
#include "internal.hpp"
#include "precond.hpp"
#include "vec_kernels.hpp"
#include "wx_launch.hpp"
#include "wx_mfma.hpp"
#include "batch_kernels.hpp"

using celes::cplx;
using celes::cx;

namespace {

thread_local std::string g_create_error;
using celes::DevBuf;

}  // namespace

namespace celes {
// Records of the reduced block entries for the matrix-core mat-vec.  Entry
// (n, n'), receiving n = (l, m), source n' = (l', m'), mu = |m' - m|; one
// record per mirror pair {(m, m'), (-m, -m')}, kept for m > 0 or m = 0 <= m':
//   [0]    p_A offset mu (4L+1) + p_A | p_B offset << 10 | (m' - m + 2L) << 20
//          | mirror flag << 30                                  (int bits)
//   [1, 2] LDS offsets of the real-form positions (n, n'), (n+H, n'+H) and
//          (n, n'+H), (n+H, n'), 16 bits each                   (int bits)
//   [3, 4] the same for the mirror entry
//   [5 .. 5+L]      a5(l',m'|l,m|p), p = p_A, p_A + 2, ...  (zero-padded)
//   [6+L .. 5+2L]   b5(l',m'|l,m|p) / i, p = p_B, p_B + 2, ...
// p_A is the least p >= max(|l-l'|, mu) with l+l'+p even and p_B the least
// p >= max(|l-l'|+1, mu) with l+l'+p odd (Appendix A.2 selection rules); an
// empty B sum points at a zero slot.  Operand position (r, c) of the real
// form, R = 2 HALF rounded up to 16, KS = R / 4, sits at
// (r / 16) 64 KS + (r % 16) KS + 16 KS (c % 4) + c / 4.
void wx_mfma_records(int L, std::vector<float>* rec) {
    const int half = L * (L + 2), hs = celes::wxm_h_stride(L), ta = L + 1, tb = L;
    // lmax 3 uses the three-product form: complex order 15 padded to 16, one
    // offset per entry (the same in the Re, Im and Re + Im matrices)
    const bool g3 = L == 3;
    const int R = g3 ? 16 : (2 * half + 15) / 16 * 16, KS = R / 4;
    rec->clear();
    auto F = [&](int r) { return (r / 16) * 64 * KS + (r % 16) * KS; };
    auto G = [&](int c) { return 16 * KS * (c % 4) + c / 4; };
    auto as_float = [](int v) {
        float f;
        std::memcpy(&f, &v, sizeof(float));
        return f;
    };
    auto pos = [&](int n, int np, float* w) {
        if (g3) {
            w[0] = as_float(F(n) + G(np));
            w[1] = as_float(0);
            return;
        }
        w[0] = as_float(F(n) + G(np) | (F(n + half) + G(np + half)) << 16);
        w[1] = as_float(F(n) + G(np + half) | (F(n + half) + G(np)) << 16);
    };
    for (int l = 1; l <= L; ++l)
        for (int m = 0; m <= l; ++m)
            for (int lp = 1; lp <= L; ++lp)
                for (int mp = -lp; mp <= lp; ++mp) {
                    if (m == 0 && mp < 0) continue;
                    float r[WXM_REC] = {};
                    const int mu = std::abs(mp - m);
                    int pa = std::max(std::abs(l - lp), mu);
                    if ((l + lp + pa) & 1) ++pa;
                    int pb = std::max(std::abs(l - lp) + 1, mu);
                    if (!((l + lp + pb) & 1)) ++pb;
                    const int hA = mu * hs + pa;
                    const int hB = pb <= l + lp - 1 ? mu * hs + pb : mu * hs + 2 * L + 1;
                    const bool mirror = !(m == 0 && mp == 0);
                    r[0] = as_float(hA | hB << 10 | (mp - m + 2 * L) << 20 | (mirror ? 1 : 0) << 30);
                    pos(lm_index(l, m), lm_index(lp, mp), r + 1);
                    pos(lm_index(l, -m), lm_index(lp, -mp), r + 3);
                    for (int q = 0; q < ta; ++q) {
                        const int p = pa + 2 * q;
                        r[5 + q] = p <= l + lp ? (float)a5_coef(lp, mp, l, m, p) : 0.f;
                    }
                    for (int q = 0; q < tb; ++q) {
                        const int p = pb + 2 * q;
                        r[5 + ta + q] = p <= l + lp - 1 ? (float)b5im_coef(lp, mp, l, m, p) : 0.f;
                    }
                    rec->insert(rec->end(), r, r + WXM_REC);
                }
}
}  // namespace celes

namespace {

int fail(celes_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    else g_create_error = msg;
    return code;
}

#define HIPCHK(h, expr)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((h), CELES_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// geometry checks
// ---------------------------------------------------------------------------
bool find_overlap(int64_t N, const double* pos, const double* rad, int64_t* a, int64_t* bidx) {
    double rmax = 0;
    double lo[3] = {1e300, 1e300, 1e300};
    for (int64_t i = 0; i < N; ++i) {
        rmax = std::max(rmax, rad[i]);
        for (int c = 0; c < 3; ++c) lo[c] = std::min(lo[c], pos[3 * i + c]);
    }
    const double cell = 2.0 * rmax > 0 ? 2.0 * rmax : 1.0;
    std::map<std::tuple<int64_t, int64_t, int64_t>, std::vector<int64_t>> grid;
    auto key = [&](int64_t i) {
        return std::make_tuple((int64_t)std::floor((pos[3 * i] - lo[0]) / cell),
                               (int64_t)std::floor((pos[3 * i + 1] - lo[1]) / cell),
                               (int64_t)std::floor((pos[3 * i + 2] - lo[2]) / cell));
    };
    for (int64_t i = 0; i < N; ++i) grid[key(i)].push_back(i);
    for (int64_t i = 0; i < N; ++i) {
        auto [cx_, cy, cz] = key(i);
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    auto it = grid.find(std::make_tuple(cx_ + dx, cy + dy, cz + dz));
                    if (it == grid.end()) continue;
                    for (int64_t j : it->second) {
                        if (j <= i) continue;
                        double d2 = 0;
                        for (int c = 0; c < 3; ++c) {
                            double t = pos[3 * i + c] - pos[3 * j + c];
                            d2 += t * t;
                        }
                        double rr = rad[i] + rad[j];
                        if (d2 <= rr * rr) {
                            *a = i;
                            *bidx = j;
                            return true;
                        }
                    }
                }
    }
    return false;
}

// ---------------------------------------------------------------------------
// Hankel lookup table: cubic Hermite per interval for h_0 and h_1, Horner
// coefficients in t, [n_int][2][4]; the kernels build the higher orders
// with the upward recurrence
// ---------------------------------------------------------------------------
void lut_geometry(const celes_handle* h, double dr, double* lo, int64_t* n) {
    double rmin = *std::min_element(h->radius.begin(), h->radius.end());
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < h->N; ++i)
        for (int c = 0; c < 3; ++c) {
            mn[c] = std::min(mn[c], h->pos[3 * i + c]);
            mx[c] = std::max(mx[c], h->pos[3 * i + c]);
        }
    double dmax = std::sqrt((mx[0] - mn[0]) * (mx[0] - mn[0]) + (mx[1] - mn[1]) * (mx[1] - mn[1]) +
                            (mx[2] - mn[2]) * (mx[2] - mn[2]));
    double dlo = std::max(dr, (std::floor(2.0 * rmin / dr) - 1.0) * dr);
    *lo = dlo;
    // a single sphere has no pairs: one interval keeps the table well formed
    *n = std::max<int64_t>(1, (int64_t)std::ceil((dmax - dlo) / dr) + 1);
}

int build_lut(celes_handle* h) {
    const int P = 1;   // highest tabulated order
    lut_geometry(h, h->opt.lut_dr, &h->lut_lo, &h->lut_n);
    h->lut_dr = h->opt.lut_dr;
    const int64_t nn = h->lut_n + 1;
    std::vector<cplx> val((size_t)nn * (P + 1)), der((size_t)nn * (P + 1));
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nn; ++q) {
        double d = h->lut_lo + (double)q * h->lut_dr;
        cplx hv[16], dh[16];
        celes::sph_hankel(P, h->k * d, hv, dh);
        for (int p = 0; p <= P; ++p) {
            val[(size_t)q * (P + 1) + p] = hv[p];
            der[(size_t)q * (P + 1) + p] = h->k * h->lut_dr * dh[p];  // d/dt = dr * d/dd
        }
    }
    std::vector<cx<double>> c64((size_t)h->lut_n * 2 * 4);
    std::vector<cx<float>> c32(c64.size());
    for (int64_t q = 0; q < h->lut_n; ++q)
        for (int p = 0; p <= 1; ++p) {
            cplx h0 = val[(size_t)q * (P + 1) + p], h1 = val[(size_t)(q + 1) * (P + 1) + p];
            cplx g0 = der[(size_t)q * (P + 1) + p], g1 = der[(size_t)(q + 1) * (P + 1) + p];
            cplx c[4] = {h0, g0, 3.0 * (h1 - h0) - 2.0 * g0 - g1, 2.0 * (h0 - h1) + g0 + g1};
            for (int t = 0; t < 4; ++t) {
                size_t o = ((size_t)q * 2 + p) * 4 + t;
                c64[o] = {c[t].real(), c[t].imag()};
                c32[o] = {(float)c[t].real(), (float)c[t].imag()};
            }
        }
    if (!h->d_lut64.ensure(c64.size() * sizeof(cx<double>)) || !h->d_lut32.ensure(c32.size() * sizeof(cx<float>)))
        return fail(h, CELES_E_OOM, "cannot allocate the Hankel lookup table");
    HIPCHK(h, hipMemcpy(h->d_lut64.p, c64.data(), c64.size() * sizeof(cx<double>), hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(h->d_lut32.p, c32.data(), c32.size() * sizeof(cx<float>), hipMemcpyHostToDevice));
    return CELES_OK;
}

// ---------------------------------------------------------------------------
// mat-vec driver
// ---------------------------------------------------------------------------
// right-hand-side block width: largest compiled width that divides K
template <typename T>
int pick_kb(int L, int K) {
    const char* env = std::getenv("CELES_WX_KB");
    int mx = celes::wx_max_kb<T>(L);
    if (env) mx = std::min(mx, std::max(1, std::atoi(env)));
    for (int kb = mx; kb > 1; kb /= 2)
        if (K % kb == 0) return kb;
    return 1;
}


// events for the next coupling-kernel launch when kernel timing is on
static const hipEvent_t* timing_events(celes_handle* h) {
    constexpr size_t kMaxTimed = 4096;   // launches recorded per timing window
    if (!h->time_kernels || h->tev_used >= 2 * kMaxTimed) return nullptr;
    if (h->tev_used + 2 > h->tev.size()) {
        for (int q = 0; q < 2; ++q) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            h->tev.push_back(e);
        }
    }
    const hipEvent_t* ev = h->tev.data() + h->tev_used;
    h->tev_used += 2;
    return ev;
}

// complex64 mat-vec of K = a multiple of 16 right-hand sides on the matrix
// cores (lmax <= 4)
static int matvec_mfma(celes_handle* h, const cx<float>* x, cx<float>* y, int K, int width, int epilogue,
                       hipStream_t s) {
    const int64_t N = h->N;
    const int64_t nbx = (N + 3) / 4 * (K / width);
    const char* env = std::getenv("CELES_WXM_TARGET_BLOCKS");
    // about 20,000 blocks: at 80 KB of LDS two blocks fit a compute unit, so
    // one chunk (N/4 blocks) leaves a partial last round; measured on the
    // 10,000-sphere slab at lmax 3 with 64 right-hand sides, 8 chunks take
    // 224.9 ms against 233.3 ms for one.  Chunks keep at least 64 sources
    // (an explicit target may go down to 2, for tests of the chunk split).
    const int target = env ? std::max(1, std::atoi(env)) : 20000;
    const int64_t max_chunks = env ? (N + 1) / 2 : std::max<int64_t>(1, N / 64);
    int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>((target + nbx - 1) / nbx, max_chunks));
    int64_t chunk_len = (N + nchunk - 1) / nchunk;
    chunk_len += chunk_len & 1;
    const int nchunk_eff = (int)((N + chunk_len - 1) / chunk_len);
    if (!h->d_xsd.ensure(celes::wx_mfma_xb_floats(h->L, N, K) * sizeof(float)) ||
        !h->d_part.ensure((size_t)nchunk_eff * K * h->nmax * N * sizeof(cx<float>)))
        return fail(h, CELES_E_OOM, "cannot allocate mat-vec scratch");
    celes::WxMfmaArgs a;
    a.px = h->d_px.as<double>();
    a.py = h->d_py.as<double>();
    a.pz = h->d_pz.as<double>();
    a.x = x;
    a.kstep = nullptr;
    a.kin = 0;
    a.slot_stride = 0;
    a.active = nullptr;
    a.sys0 = 0;
    a.xb = h->d_xsd.as<float>();
    a.part = h->d_part.as<cx<float>>();
    a.rec = h->d_mrec.as<float>();
    a.lut.coef = h->d_lut32.as<cx<float>>();
    a.lut.d_lo = h->lut_lo;
    a.lut.inv_dr = 1.0 / h->lut_dr;
    a.lut.inv_k = 1.0 / h->k;
    a.lut.n_int = (int)h->lut_n;
    a.k = h->k;
    a.n = (int)N;
    a.chunk_len = (int)chunk_len;
    a.ldp = (int)N;
    a.nrhs = K;
    const int rc = celes::wx_launch_mfma(a, h->L, width, h->opt.hankel == CELES_HANKEL_DIRECT ? 1 : 0, nchunk_eff, x,
                                         h->d_tq32.as<cx<float>>(), y, epilogue, s, timing_events(h));
    if (rc != 0) return fail(h, CELES_E_DEVICE, "matrix-core mat-vec launch failed");
    return CELES_OK;
}

// matrix-core path for K right-hand sides in complex64?  CELES_WXM=0 turns
// it off, CELES_WXM=2 takes it for every applicable width (tests)
static int mfma_width(const celes_handle* h, int K) {
    const char* env = std::getenv("CELES_WXM");
    const int mode = env ? std::atoi(env) : 1;
    if (mode == 0) return 0;
    return celes::wx_mfma_block(h->L, K, mode == 2);
}

// y = W x (epilogue 0) or x - T W x (epilogue 1) for K right-hand sides,
// x, y: [K][N][nmax] device buffers of precision T
template <typename T>
static int matvec_valu(celes_handle* h, const cx<T>* x, cx<T>* y, int K, int epilogue, hipStream_t s, int target,
                       bool timed, void* ext = nullptr, size_t ext_bytes = 0);

// default source-chunk split: about this many blocks (receiver tiles x
// source chunks x passes), so that the last round of resident blocks is a
// small part of a launch.  Measured on the 20,000-sphere slab at lmax 4
// (kernel ms at 4,096 / 32,768 blocks): direct FP64 147.6 / 144.1,
// complex64 77.7 / 75.1; rotation scheme (one wave per block) FP64 78.7 /
// 67.1, complex64 40.0 / 30.4; flat from there to 262,144.
constexpr int kDefaultTargetBlocks = 32768;

// source-chunk split without tuning: the environment (tests), the handle's
// forced value, or kDefaultTargetBlocks
static int matvec_target_fixed(const celes_handle* h) {
    const char* env = std::getenv("CELES_WX_TARGET_BLOCKS");
    if (env) return std::max(1, std::atoi(env));
    return h->target_blocks > 0 ? h->target_blocks : kDefaultTargetBlocks;
}

// source-chunk split of the VALU mat-vec: the environment (tests), the
// handle's forced value, the autotuned value, or kDefaultTargetBlocks.  With
// opt.autotune the first call of each precision times the candidate splits
// on the caller's x and y (each candidate writes y completely) and keeps the
// fastest; not while the stream is being captured.
template <typename T>
static int matvec_target(celes_handle* h, const cx<T>* x, cx<T>* y, int K, int epilogue, hipStream_t s) {
    const char* env = std::getenv("CELES_WX_TARGET_BLOCKS");
    if (env) return std::max(1, std::atoi(env));
    if (h->target_blocks > 0) return h->target_blocks;
    if (h->opt.deterministic) return kDefaultTargetBlocks;
    int& tuned = h->tuned_blocks[sizeof(T) == 8 ? 0 : 1];
    if (tuned > 0 || !h->opt.autotune) return tuned > 0 ? tuned : kDefaultTargetBlocks;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return kDefaultTargetBlocks;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return kDefaultTargetBlocks;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return kDefaultTargetBlocks;
    }
    float best = 1e30f;
    int best_t = kDefaultTargetBlocks;
    for (int t : {4096, 8192, 16384, 32768, 65536, 131072}) {
        if (matvec_valu<T>(h, x, y, K, epilogue, s, t, false) != CELES_OK) continue;   // warm
        hipEventRecord(e0, s);
        const int rc = matvec_valu<T>(h, x, y, K, epilogue, s, t, false);
        hipEventRecord(e1, s);
        float ms = 0;
        if (rc != CELES_OK || hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            continue;
        if (ms < best) {
            best = ms;
            best_t = t;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    tuned = best_t;
    return tuned;
}

template <typename T>
int matvec(celes_handle* h, const cx<T>* x, cx<T>* y, int K, int epilogue, hipStream_t s) {
    if constexpr (sizeof(T) == 4) {
        const int width = mfma_width(h, K);
        if (width > 0) return matvec_mfma(h, x, y, K, width, epilogue, s);
    }
    return matvec_valu<T>(h, x, y, K, epilogue, s, matvec_target<T>(h, x, y, K, epilogue, s), true);
}

// With ext (bytes ext_bytes) the source sums/differences and the chunk
// partial sums live in that caller-given device buffer, with the number of
// source chunks capped so that both fit, and nothing is allocated.
template <typename T>
static int matvec_valu(celes_handle* h, const cx<T>* x, cx<T>* y, int K, int epilogue, hipStream_t s, int target,
                       bool timed, void* ext, size_t ext_bytes) {
    const int64_t N = h->N;
    const bool rot = h->opt.translation == CELES_TRANSLATION_ROTATE;
    const int kb = rot ? 1 : pick_kb<T>(h->L, K);
    int64_t nbx = rot ? (N + celes::WX_RTR_BLOCK_SIZE - 1) / celes::WX_RTR_BLOCK_SIZE * 2 * K
                      : (N + celes::WX_BLOCK_SIZE - 1) / celes::WX_BLOCK_SIZE * celes::wx_num_groups(h->L) * (K / kb);
    int64_t nchunk = (target + nbx - 1) / nbx;
    nchunk = std::max<int64_t>(1, std::min<int64_t>(nchunk, (N + celes::WX_TILE_SIZE - 1) / celes::WX_TILE_SIZE));
    const size_t vec_bytes = (size_t)K * N * h->nmax * sizeof(cx<T>);     // one [K][N][nmax] vector
    const size_t xsd_bytes = (vec_bytes + 255) / 256 * 256;
    // the partial sums hold nchunk vectors: at most 2 GiB of them, but never
    // fewer chunks than a 4,096-block split would take (the partial sums of a
    // split of T blocks come to about T x 256 x nmax x element bytes x (RHS
    // per block) / (pass groups), whatever N and K)
    const int64_t cap = std::max<int64_t>((4096 + nbx - 1) / nbx, (int64_t)(((size_t)2 << 30) / vec_bytes));
    nchunk = std::max<int64_t>(1, std::min(nchunk, cap));
    if (ext) {
        const size_t fit = ext_bytes > xsd_bytes ? (ext_bytes - xsd_bytes) / vec_bytes : 0;
        if (fit < 1)
            return fail(h, CELES_E_ARG, "K N nmax too large for the fixed scratch buffer (needs " +
                                            std::to_string(xsd_bytes + vec_bytes) + " bytes, has " +
                                            std::to_string(ext_bytes) + ")");
        nchunk = std::min<int64_t>(nchunk, (int64_t)fit);
    }
    int64_t chunk_len = (N + nchunk - 1) / nchunk;
    chunk_len = (chunk_len + celes::WX_TILE_SIZE - 1) / celes::WX_TILE_SIZE * celes::WX_TILE_SIZE;
    const int nchunk_eff = (int)((N + chunk_len - 1) / chunk_len);
    if (!ext && (!h->d_xsd.ensure(vec_bytes) || !h->d_part.ensure((size_t)nchunk_eff * vec_bytes)))
        return fail(h, CELES_E_OOM, "cannot allocate mat-vec scratch");
    celes::WxArgs<T> a;
    a.px = h->d_px.as<double>();
    a.py = h->d_py.as<double>();
    a.pz = h->d_pz.as<double>();
    a.xsd = ext ? (cx<T>*)ext : h->d_xsd.as<cx<T>>();
    a.part = ext ? (cx<T>*)((char*)ext + xsd_bytes) : h->d_part.as<cx<T>>();
    a.lut.coef = (sizeof(T) == 8) ? (const cx<T>*)h->d_lut64.p : (const cx<T>*)h->d_lut32.p;
    a.lut.d_lo = h->lut_lo;
    a.lut.inv_dr = 1.0 / h->lut_dr;
    a.lut.inv_k = 1.0 / h->k;
    a.lut.n_int = (int)h->lut_n;
    a.k = h->k;
    a.n = (int)N;
    a.chunk_len = (int)chunk_len;
    a.ldp = (int)N;
    a.nrhs = K;
    a.kb = kb;
    a.active = nullptr;
    a.sys0 = 0;
    const cx<T>* tq = (sizeof(T) == 8) ? (const cx<T>*)h->d_tq64.p : (const cx<T>*)h->d_tq32.p;
    int rc = celes::wx_launch<T>(a, h->L, h->opt.hankel == CELES_HANKEL_DIRECT ? 1 : 0, nchunk_eff, x, tq, y,
                                 epilogue, s, timed ? timing_events(h) : nullptr, rot ? 1 : 0);
    if (rc == -1) return fail(h, CELES_E_UNSUPPORTED, "lmax not compiled");
    if (rc != 0) return fail(h, CELES_E_DEVICE, "mat-vec launch failed");
    return CELES_OK;
}

// ---------------------------------------------------------------------------
// GMRES (right-preconditioned, restarted, classical Gram-Schmidt with one
// re-orthogonalisation) on device vectors of precision T.  Inner products
// accumulate in FP64.  Solves M x = rhs from the initial x.
// ---------------------------------------------------------------------------
struct GmresResult {
    int iterations = 0;
    int restarts = 0;
    int matvecs = 0;
    double est = 0;       // final implicit relative residual estimate
    bool breakdown = false;
    double matvec_seconds = 0;
};

template <typename T>
int gmres_device(celes_handle* h, const cx<T>* rhs, cx<T>* x, double tol, int maxiter, double rhs_norm,
                 GmresResult* out, hipStream_t s, cx<T>* V, cx<T>* w, cx<T>* z) {
    const int64_t n = h->N * h->nmax;
    const int m = std::max(1, h->opt.restart);
    cx<double>* dh = h->d_h.as<cx<double>>();
    cx<double>* dpart = h->d_partial.as<cx<double>>();
    std::vector<cx<double>> hh(m + 2), hh2(m + 2);
    std::vector<cplx> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
    const bool use_pre = (bool)h->pre;
    auto apply_pre = [&](const cx<T>* in, cx<T>* outv) -> int {
        return h->pre->apply<T>(in, outv, s);
    };
    // mat-vec time from events around each mat-vec, read once the stream has
    // reached the next host synchronisation (norm2), never by waiting on them
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    // a failed copy or synchronisation ends the solve with CELES_E_DEVICE
    // (the host would otherwise go on with stale values)
    bool dev_err = false;
    auto dev_ok = [&](hipError_t e) {
        if (e != hipSuccess) dev_err = true;
        return e == hipSuccess;
    };
    bool pending = false;
    auto collect = [&]() {
        if (!pending) return;
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) out->matvec_seconds += ms * 1e-3;
        pending = false;
    };
    auto norm2 = [&](const cx<T>* v) -> double {
        celes::vec_dots<T>(v, 0, 1, v, n, dpart, dh, s);
        cx<double> r;
        if (!dev_ok(hipMemcpyAsync(&r, dh, sizeof(r), hipMemcpyDeviceToHost, s)) || !dev_ok(hipStreamSynchronize(s)))
            return std::numeric_limits<double>::quiet_NaN();
        collect();
        return std::sqrt(std::max(0.0, r.re));
    };
    auto timed_matvec = [&](const cx<T>* in, cx<T>* outv) -> int {
        hipEventRecord(e0, s);
        int rc = matvec<T>(h, in, outv, 1, 1, s);
        hipEventRecord(e1, s);
        pending = true;
        out->matvecs++;
        return rc;
    };
    int rc = CELES_OK;
    while (true) {
        // r = rhs - M x  -> V[0]
        if ((rc = timed_matvec(x, w)) != CELES_OK) break;
        celes::vec_sub<T>(rhs, w, V, n, s);
        double beta = norm2(V);
        out->est = beta / rhs_norm;
        if (dev_err) break;
        if (!std::isfinite(beta)) {
            out->breakdown = true;
            break;
        }
        if (out->est <= tol || out->iterations >= maxiter) break;
        celes::vec_scale<T>(V, 1.0 / beta, V, n, s);
        std::fill(g.begin(), g.end(), cplx(0, 0));
        g[0] = beta;
        int kk = 0, used = 0;
        for (kk = 0; kk < m; ++kk) {
            cx<T>* vk = V + (int64_t)kk * n;
            cx<T>* vk1 = V + (int64_t)(kk + 1) * n;
            const cx<T>* zin = vk;
            if (use_pre) {
                if ((rc = apply_pre(vk, z)) != CELES_OK) break;
                zin = z;
            }
            if ((rc = timed_matvec(zin, vk1)) != CELES_OK) break;
            // CGS2
            celes::vec_dots<T>(V, n, kk + 1, vk1, n, dpart, dh, s);
            celes::vec_gemv_sub<T>(V, n, kk + 1, dh, vk1, n, s);
            dev_ok(hipMemcpyAsync(hh.data(), dh, (kk + 1) * sizeof(cx<double>), hipMemcpyDeviceToHost, s));
            celes::vec_dots<T>(V, n, kk + 1, vk1, n, dpart, dh, s);
            celes::vec_gemv_sub<T>(V, n, kk + 1, dh, vk1, n, s);
            dev_ok(hipMemcpyAsync(hh2.data(), dh, (kk + 1) * sizeof(cx<double>), hipMemcpyDeviceToHost, s));
            double hn = norm2(vk1);
            for (int i = 0; i <= kk; ++i)
                H[(size_t)i * m + kk] = cplx(hh[i].re + hh2[i].re, hh[i].im + hh2[i].im);
            H[(size_t)(kk + 1) * m + kk] = hn;
            if (dev_err) break;
            if (!std::isfinite(hn)) {
                out->breakdown = true;
                break;
            }
            // previous Givens rotations G_i = [[conj(c), conj(s)], [-s, c]]
            for (int i = 0; i < kk; ++i) {
                cplx a = H[(size_t)i * m + kk], bb = H[(size_t)(i + 1) * m + kk];
                H[(size_t)i * m + kk] = std::conj(cs[i]) * a + std::conj(sn[i]) * bb;
                H[(size_t)(i + 1) * m + kk] = -sn[i] * a + cs[i] * bb;
            }
            cplx a = H[(size_t)kk * m + kk], bb = H[(size_t)(kk + 1) * m + kk];
            double den = std::sqrt(std::norm(a) + std::norm(bb));
            cs[kk] = den > 0 ? a / den : cplx(1, 0);
            sn[kk] = den > 0 ? bb / den : cplx(0, 0);
            H[(size_t)kk * m + kk] = den;
            H[(size_t)(kk + 1) * m + kk] = 0;
            g[kk + 1] = -sn[kk] * g[kk];
            g[kk] = std::conj(cs[kk]) * g[kk];
            out->iterations++;
            used = kk + 1;
            if (hn > 0) celes::vec_scale<T>(vk1, 1.0 / hn, vk1, n, s);
            double est = std::abs(g[kk + 1]) / rhs_norm;
            out->est = est;
            if (hn == 0 || est <= tol || out->iterations >= maxiter) break;
        }
        if (rc != CELES_OK || out->breakdown || dev_err) break;
        // y = H^{-1} g (upper triangular), u = V y, x += P^{-1} u
        std::vector<cplx> y(used);
        for (int i = used - 1; i >= 0; --i) {
            cplx t = g[i];
            for (int j = i + 1; j < used; ++j) t -= H[(size_t)i * m + j] * y[j];
            y[i] = t / H[(size_t)i * m + i];
        }
        std::vector<cx<double>> yd(used);
        for (int i = 0; i < used; ++i) yd[i] = {y[i].real(), y[i].imag()};
        dev_ok(hipMemcpyAsync(dh, yd.data(), used * sizeof(cx<double>), hipMemcpyHostToDevice, s));
        if (use_pre) {
            dev_ok(hipMemsetAsync(w, 0, n * sizeof(cx<T>), s));
            celes::vec_gemv_add<T>(V, n, used, dh, w, n, s);
            if ((rc = apply_pre(w, z)) != CELES_OK) break;
            // x += z : reuse gemv_add with a single "basis vector" z and coefficient 1
            cx<double> one = {1.0, 0.0};
            dev_ok(hipMemcpyAsync(dh, &one, sizeof(one), hipMemcpyHostToDevice, s));
            celes::vec_gemv_add<T>(z, n, 1, dh, x, n, s);
        } else {
            celes::vec_gemv_add<T>(V, n, used, dh, x, n, s);
        }
        if (!dev_ok(hipStreamSynchronize(s))) break;
        out->restarts++;
        if (h->opt.verbose)
            std::fprintf(stderr, "gmres (%s) cycle %d: %d iterations, estimate %.3e\n",
                         sizeof(T) == 8 ? "fp64" : "fp32", out->restarts, out->iterations, out->est);
    }
    if (pending && !dev_err) {
        hipEventSynchronize(e1);
        collect();
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (dev_err && rc == CELES_OK)
        rc = fail(h, CELES_E_DEVICE, std::string("device error during GMRES: ") + hipGetErrorString(hipGetLastError()));
    return rc;
}

// ---------------------------------------------------------------------------
// BiCGSTAB (right-preconditioned, the alternative solver of Section 3.2) on
// device vectors of precision T, inner products in FP64.  Solves M x = rhs
// from the initial x.  A run starts from the true residual r = rhs - M x
// with shadow residual r~ = r and ends when the updated residual reaches
// tol * ||rhs|| or on a breakdown (rho = 0, r~^H v = 0, omega = 0); the true
// residual then decides whether a new run starts.  A run that makes no
// iteration ends the solve.  work: 7 vectors of N nmax.
// ---------------------------------------------------------------------------
template <typename T>
int bicgstab_device(celes_handle* h, const cx<T>* rhs, cx<T>* x, double tol, int maxiter, double rhs_norm,
                    GmresResult* out, hipStream_t s, cx<T>* work) {
    const int64_t n = h->N * h->nmax;
    // r (later s) and t are adjacent and r~ sits two vectors after r, so one
    // dots launch over {r, t} or {r, r~} yields two inner products
    cx<T>* r = work;
    cx<T>* t = work + n;
    cx<T>* rt = work + 2 * n;
    cx<T>* p = work + 3 * n;
    cx<T>* v = work + 4 * n;
    cx<T>* ph = work + 5 * n;
    cx<T>* sh = work + 6 * n;
    cx<double>* dh = h->d_h.as<cx<double>>();
    cx<double>* dpart = h->d_partial.as<cx<double>>();
    const bool use_pre = (bool)h->pre;
    cx<double> hv[2];
    // a failed copy or synchronisation ends the solve with CELES_E_DEVICE
    bool dev_err = false;
    // out[c] = V[c]^H w for c < m, V[c] = V0 + c * ldv; copied to hv (NaN
    // after a device error)
    auto dots = [&](const cx<T>* V0, int64_t ldv, int m, const cx<T>* w) {
        celes::vec_dots<T>(V0, ldv, m, w, n, dpart, dh, s);
        if (hipMemcpyAsync(hv, dh, m * sizeof(cx<double>), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            dev_err = true;
            const double nan = std::numeric_limits<double>::quiet_NaN();
            for (int c = 0; c < m; ++c) hv[c] = {nan, nan};
        }
    };
    auto cplx_of = [](cx<double> a) { return cplx(a.re, a.im); };
    auto cxd = [](cplx a) { return cx<double>{a.real(), a.imag()}; };
    const cx<double> one = {1.0, 0.0}, zero = {0.0, 0.0};
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    auto timed_matvec = [&](const cx<T>* in, cx<T>* outv) -> int {
        hipEventRecord(e0, s);
        int rc = matvec<T>(h, in, outv, 1, 1, s);
        hipEventRecord(e1, s);
        hipEventSynchronize(e1);
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        out->matvec_seconds += ms * 1e-3;
        out->matvecs++;
        return rc;
    };
    // returns the vector holding P^{-1} in (in itself without a preconditioner)
    auto precond = [&](const cx<T>* in, cx<T>* buf, int* rc) -> const cx<T>* {
        if (!use_pre) return in;
        *rc = h->pre->apply<T>(in, buf, s);
        return buf;
    };
    int rc = CELES_OK;
    while (true) {
        if ((rc = timed_matvec(x, t)) != CELES_OK) break;
        celes::vec_sub<T>(rhs, t, r, n, s);
        dots(r, 0, 1, r);
        double res = std::sqrt(std::max(0.0, hv[0].re)) / rhs_norm;
        out->est = res;
        if (!std::isfinite(res)) {
            out->breakdown = true;
            break;
        }
        if (res <= tol || out->iterations >= maxiter) break;
        celes::vec_scale<T>(r, 1.0, rt, n, s);
        cplx rho = hv[0].re, rho_old = 1.0, alpha = 1.0, omega = 1.0;
        int run_its = 0;
        while (out->iterations < maxiter) {
            if (rho == cplx(0, 0)) break;
            if (run_its == 0) {
                celes::vec_scale<T>(r, 1.0, p, n, s);
            } else {
                const cplx beta = (rho / rho_old) * (alpha / omega);
                celes::vec_comb3<T>(r, one, p, cxd(beta), v, cxd(-beta * omega), p, n, s);
            }
            const cx<T>* phat = precond(p, ph, &rc);
            if (rc != CELES_OK) break;
            if ((rc = timed_matvec(phat, v)) != CELES_OK) break;
            dots(rt, 0, 1, v);
            const cplx rv = cplx_of(hv[0]);
            if (rv == cplx(0, 0)) break;
            alpha = rho / rv;
            // s = r - alpha v, kept in r
            celes::vec_comb3<T>(r, one, v, cxd(-alpha), nullptr, zero, r, n, s);
            out->iterations++;
            run_its++;
            dots(r, 0, 1, r);
            const double snorm = std::sqrt(std::max(0.0, hv[0].re)) / rhs_norm;
            out->est = snorm;
            if (!std::isfinite(snorm)) {
                out->breakdown = true;
                break;
            }
            if (snorm <= tol) {
                celes::vec_comb3<T>(x, one, phat, cxd(alpha), nullptr, zero, x, n, s);
                break;
            }
            const cx<T>* shat = precond(r, sh, &rc);
            if (rc != CELES_OK) break;
            if ((rc = timed_matvec(shat, t)) != CELES_OK) break;
            dots(r, n, 2, t);  // {s^H t, t^H t}
            const double tt = hv[1].re;
            omega = tt > 0 ? std::conj(cplx_of(hv[0])) / tt : cplx(0, 0);
            celes::vec_comb3<T>(x, one, phat, cxd(alpha), shat, cxd(omega), x, n, s);
            celes::vec_comb3<T>(r, one, t, cxd(-omega), nullptr, zero, r, n, s);
            rho_old = rho;
            dots(r, 2 * n, 2, r);  // {r^H r, r~^H r}
            const double rnorm = std::sqrt(std::max(0.0, hv[0].re)) / rhs_norm;
            rho = cplx_of(hv[1]);
            out->est = rnorm;
            if (!std::isfinite(rnorm)) {
                out->breakdown = true;
                break;
            }
            if (rnorm <= tol || omega == cplx(0, 0)) break;
        }
        if (rc != CELES_OK || out->breakdown) break;
        out->restarts++;
        if (h->opt.verbose)
            std::fprintf(stderr, "bicgstab (%s) run %d: %d iterations, updated residual %.3e\n",
                         sizeof(T) == 8 ? "fp64" : "fp32", out->restarts, out->iterations, out->est);
        if (run_its == 0) break;
    }
    if (hipStreamSynchronize(s) != hipSuccess) dev_err = true;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (dev_err && rc == CELES_OK)
        rc = fail(h, CELES_E_DEVICE, std::string("device error during BiCGSTAB: ") + hipGetErrorString(hipGetLastError()));
    return rc;
}

int ensure_solver_buffers(celes_handle* h, bool mixed) {
    const int64_t n = h->N * h->nmax;
    const int m = std::max(1, h->opt.restart);
    bool ok = h->d_h.ensure((m + 2) * sizeof(cx<double>)) &&
              h->d_partial.ensure((size_t)celes::VEC_PARTIAL_BLOCKS * (m + 2) * sizeof(cx<double>)) &&
              h->d_w.ensure(n * sizeof(cx<double>)) && h->d_z.ensure(n * sizeof(cx<double>)) &&
              h->d_r.ensure(n * sizeof(cx<double>)) && h->d_x.ensure(n * sizeof(cx<double>)) &&
              h->d_rhs.ensure(n * sizeof(cx<double>));
    // Krylov basis (GMRES) or the seven work vectors (BiCGSTAB)
    const size_t nv = h->opt.solver == CELES_SOLVER_BICGSTAB ? 7 : (size_t)(m + 1);
    if (mixed)
        ok = ok && h->d_V32.ensure(nv * n * sizeof(cx<float>)) &&
             h->d_w32.ensure(n * sizeof(cx<float>)) && h->d_z32.ensure(n * sizeof(cx<float>)) &&
             h->d_r32.ensure(n * sizeof(cx<float>)) && h->d_x32.ensure(n * sizeof(cx<float>));
    else
        ok = ok && h->d_V.ensure(nv * n * sizeof(cx<double>));
    return ok ? CELES_OK : fail(h, CELES_E_OOM, "cannot allocate solver buffers");
}

double host_norm(const std::vector<cplx>& v, size_t off, size_t n) {
    double s = 0;
    for (size_t i = 0; i < n; ++i) s += std::norm(v[off + i]);
    return std::sqrt(s);
}

// FP64 residual r = rhs - M x on the device; returns ||r||
double residual64(celes_handle* h, const cx<double>* rhs, const cx<double>* x, cx<double>* r, hipStream_t s,
                  int* rc, double* mv_sec) {
    const int64_t n = h->N * h->nmax;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    hipEventRecord(e0, s);
    *rc = matvec<double>(h, x, h->d_w.as<cx<double>>(), 1, 1, s);
    hipEventRecord(e1, s);
    celes::vec_sub<double>(rhs, h->d_w.as<cx<double>>(), r, n, s);
    celes::vec_dots<double>(r, 0, 1, r, n, h->d_partial.as<cx<double>>(), h->d_h.as<cx<double>>(), s);
    cx<double> v;
    if (hipMemcpyAsync(&v, h->d_h.p, sizeof(v), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        if (*rc == CELES_OK)
            *rc = fail(h, CELES_E_DEVICE, std::string("device error in the FP64 residual: ") +
                                              hipGetErrorString(hipGetLastError()));
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        return std::numeric_limits<double>::quiet_NaN();
    }
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    *mv_sec += ms * 1e-3;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return std::sqrt(std::max(0.0, v.re));
}

}  // namespace

int matvec_on_scratch(celes_handle* h, int precision, int K, const void* x, void* y, hipStream_t s, void* scratch,
                      size_t scratch_bytes) {
    if (precision == CELES_FP64)
        return matvec_valu<double>(h, (const cx<double>*)x, (cx<double>*)y, K, 0, s, matvec_target_fixed(h), false,
                                   scratch, scratch_bytes);
    if (precision == CELES_MIXED)
        return matvec_valu<float>(h, (const cx<float>*)x, (cx<float>*)y, K, 0, s, matvec_target_fixed(h), false,
                                  scratch, scratch_bytes);
    return fail(h, CELES_E_ARG, "unknown precision");
}


// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void celes_default_options(celes_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = CELES_FP64;
    opt->hankel = CELES_HANKEL_LUT;
    opt->lut_dr = 1.0;
    opt->tol = 1e-8;
    opt->inner_tol = 1e-4;
    opt->restart = 100;
    opt->maxiter = 2000;
    opt->max_refinements = 30;
    opt->cuboid_edge = 0.0;
    opt->device = 0;
    opt->verbose = 0;
    opt->solver = CELES_SOLVER_GMRES;
    opt->target_Nj = 100.0;
    opt->mem_cap_bytes = 0.0;
    opt->autotune = 0;
}

int celes_version(void) { return CELES_VERSION; }

const char* celes_last_error(const celes_handle* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

static int celes_build_preconditioner_impl(celes_handle* h, double cuboid_edge);

static int celes_create_impl(celes_handle** out, int64_t N, const double* pos, const double* radius, const double* n_sphere,
                 double n0, double wavelength, int lmax, const celes_options* opt) {
    if (!out) return fail(nullptr, CELES_E_ARG, "null handle pointer");
    *out = nullptr;
    if (N < 1 || !pos || !radius || !n_sphere) return fail(nullptr, CELES_E_ARG, "N < 1 or null input array");
    if (lmax < 1) return fail(nullptr, CELES_E_ARG, "lmax < 1");
    if (lmax > CELES_MAX_LMAX) return fail(nullptr, CELES_E_UNSUPPORTED, "lmax above CELES_MAX_LMAX");
    if (!(n0 > 0) || !(wavelength > 0) || !std::isfinite(n0) || !std::isfinite(wavelength))
        return fail(nullptr, CELES_E_ARG, "n0 and wavelength must be positive and finite");
    if (N > (int64_t)std::numeric_limits<int>::max() / 64)
        return fail(nullptr, CELES_E_ARG, "N too large");
    for (int64_t i = 0; i < N; ++i) {
        for (int c = 0; c < 3; ++c)
            if (!std::isfinite(pos[3 * i + c])) return fail(nullptr, CELES_E_NONFINITE, "non-finite position");
        if (!std::isfinite(radius[i]) || !(radius[i] > 0))
            return fail(nullptr, CELES_E_NONFINITE, "radius must be positive and finite");
        if (!std::isfinite(n_sphere[2 * i]) || !std::isfinite(n_sphere[2 * i + 1]))
            return fail(nullptr, CELES_E_NONFINITE, "non-finite refractive index");
    }
    int64_t oa, ob;
    if (find_overlap(N, pos, radius, &oa, &ob))
        return fail(nullptr, CELES_E_OVERLAP,
                    "spheres " + std::to_string(oa) + " and " + std::to_string(ob) + " overlap");
    std::unique_ptr<celes_handle> h(new celes_handle());
    if (opt) h->opt = *opt;
    else celes_default_options(&h->opt);
    if (!(h->opt.lut_dr > 0)) return fail(nullptr, CELES_E_ARG, "lut_dr must be positive");
    if (h->opt.restart < 1) h->opt.restart = 1;
    if (h->opt.solver != CELES_SOLVER_GMRES && h->opt.solver != CELES_SOLVER_BICGSTAB)
        return fail(nullptr, CELES_E_ARG, "unknown solver");
    if (h->opt.translation != CELES_TRANSLATION_DIRECT && h->opt.translation != CELES_TRANSLATION_ROTATE)
        return fail(nullptr, CELES_E_ARG, "unknown translation scheme");
    if (hipSetDevice(h->opt.device) != hipSuccess) return fail(nullptr, CELES_E_DEVICE, "hipSetDevice failed");
    h->N = N;
    h->L = lmax;
    h->nmax = celes::nmax_of(lmax);
    h->half = celes::half_of(lmax);
    h->n0 = n0;
    h->wavelength = wavelength;
    h->k = 2.0 * M_PI * n0 / wavelength;
    h->pos.assign(pos, pos + 3 * N);
    h->radius.assign(radius, radius + N);
    h->nsph.resize(N);
    for (int64_t i = 0; i < N; ++i) h->nsph[i] = cplx(n_sphere[2 * i], n_sphere[2 * i + 1]);
    // Mie coefficients (Appendix B), relative index n_i / n0
    h->tq.resize((size_t)N * 2 * lmax);
    {
        std::map<std::pair<double, std::pair<double, double>>, std::vector<cplx>> cache;
        std::vector<cplx> q1(lmax), q2(lmax);
        for (int64_t i = 0; i < N; ++i) {
            auto key = std::make_pair(radius[i], std::make_pair(h->nsph[i].real(), h->nsph[i].imag()));
            auto it = cache.find(key);
            if (it == cache.end()) {
                celes::mie_Q(lmax, h->k * radius[i], h->nsph[i] / n0, q1.data(), q2.data());
                std::vector<cplx> v(2 * lmax);
                for (int l = 0; l < lmax; ++l) {
                    v[l] = q1[l];
                    v[lmax + l] = q2[l];
                }
                it = cache.emplace(key, v).first;
            }
            std::copy(it->second.begin(), it->second.end(), h->tq.begin() + (size_t)i * 2 * lmax);
        }
    }
    // device geometry and T
    std::vector<double> px(N), py(N), pz(N);
    for (int64_t i = 0; i < N; ++i) {
        px[i] = pos[3 * i];
        py[i] = pos[3 * i + 1];
        pz[i] = pos[3 * i + 2];
    }
    std::vector<cx<double>> t64(h->tq.size());
    std::vector<cx<float>> t32(h->tq.size());
    for (size_t i = 0; i < h->tq.size(); ++i) {
        t64[i] = {h->tq[i].real(), h->tq[i].imag()};
        t32[i] = {(float)h->tq[i].real(), (float)h->tq[i].imag()};
    }
    celes_handle* hp = h.get();
    if (!h->d_px.ensure(N * 8) || !h->d_py.ensure(N * 8) || !h->d_pz.ensure(N * 8) ||
        !h->d_tq64.ensure(t64.size() * sizeof(cx<double>)) || !h->d_tq32.ensure(t32.size() * sizeof(cx<float>)))
        return fail(nullptr, CELES_E_OOM, "device allocation failed");
    if (hipMemcpy(h->d_px.p, px.data(), N * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_py.p, py.data(), N * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_pz.p, pz.data(), N * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_tq64.p, t64.data(), t64.size() * sizeof(cx<double>), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_tq32.p, t32.data(), t32.size() * sizeof(cx<float>), hipMemcpyHostToDevice) != hipSuccess)
        return fail(nullptr, CELES_E_DEVICE, "host-to-device copy failed");
    int rc = build_lut(hp);
    if (rc != CELES_OK) {
        g_create_error = hp->err;
        return rc;
    }
    if (lmax <= celes::WXM_MAX_L) {
        std::vector<float> rec;
        celes::wx_mfma_records(lmax, &rec);
        if (!hp->d_mrec.ensure(rec.size() * sizeof(float)) ||
            hipMemcpy(hp->d_mrec.p, rec.data(), rec.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
            return fail(nullptr, CELES_E_DEVICE, "cannot upload the block-entry records");
    }
    if (hp->opt.cuboid_edge != 0 && (rc = celes_build_preconditioner_impl(hp, hp->opt.cuboid_edge)) != CELES_OK) {
        g_create_error = hp->err;
        return rc;
    }
    *out = h.release();
    return CELES_OK;
}
int celes_create(celes_handle** out, int64_t N, const double* pos, const double* radius, const double* n_sphere,
                 double n0, double wavelength, int lmax, const celes_options* opt) {
    return celes_guard([&] { return celes_create_impl(out, N, pos, radius, n_sphere, n0, wavelength, lmax, opt); });
}


void celes_destroy(celes_handle* h) { delete h; }

int celes_set_solve_options(celes_handle* h, const celes_options* opt) {
    if (!h || !opt) return CELES_E_ARG;
    if (opt->solver != CELES_SOLVER_GMRES && opt->solver != CELES_SOLVER_BICGSTAB)
        return fail(h, CELES_E_ARG, "unknown solver");
    if (opt->precision != CELES_FP64 && opt->precision != CELES_MIXED) return fail(h, CELES_E_ARG, "unknown precision");
    if (opt->translation != CELES_TRANSLATION_DIRECT && opt->translation != CELES_TRANSLATION_ROTATE)
        return fail(h, CELES_E_ARG, "unknown translation scheme");
    celes_options& o = h->opt;
    o.precision = opt->precision;
    o.tol = opt->tol;
    o.inner_tol = opt->inner_tol;
    o.restart = std::max(1, opt->restart);
    o.maxiter = opt->maxiter;
    o.max_refinements = opt->max_refinements;
    o.verbose = opt->verbose;
    o.solver = opt->solver;
    o.target_Nj = opt->target_Nj;
    o.mem_cap_bytes = opt->mem_cap_bytes;
    o.autotune = opt->autotune;
    o.deterministic = opt->deterministic;
    if (o.translation != opt->translation) {
        o.translation = opt->translation;
        h->tuned_blocks[0] = h->tuned_blocks[1] = 0;     // a tuned split belongs to one scheme
    }
    return CELES_OK;
}

int celes_dims(const celes_handle* h, int64_t* N, int* lmax, int* nmax) {
    if (!h) return CELES_E_ARG;
    if (N) *N = h->N;
    if (lmax) *lmax = h->L;
    if (nmax) *nmax = h->nmax;
    return CELES_OK;
}

int celes_lut_info(const celes_handle* h, double* d_lo, double* dr, int64_t* n_int) {
    if (!h) return CELES_E_ARG;
    if (d_lo) *d_lo = h->lut_lo;
    if (dr) *dr = h->lut_dr;
    if (n_int) *n_int = h->lut_n;
    return CELES_OK;
}

int celes_num_rhs(const celes_handle* h) { return h ? h->K : 0; }

static int celes_set_plane_waves_impl(celes_handle* h, int K, const double* beta, const double* alpha, const int* pol,
                          const double* E0) {
    if (!h) return CELES_E_ARG;
    if (K < 1 || !beta || !alpha || !pol) return fail(h, CELES_E_ARG, "K < 1 or null array");
    for (int kk = 0; kk < K; ++kk)
        if (pol[kk] != 1 && pol[kk] != 2) return fail(h, CELES_E_ARG, "pol must be 1 or 2");
    const int64_t N = h->N;
    const int nm = h->nmax, L = h->L;
    h->a_in.assign((size_t)K * N * nm, cplx(0, 0));
    for (int kk = 0; kk < K; ++kk) {
        const double b = beta[kk], al = alpha[kk];
        const cplx e0 = E0 ? cplx(E0[2 * kk], E0[2 * kk + 1]) : cplx(1, 0);
        // a_{in,n}^i = 4 E0 e^{i k.r_i} e^{-i m alpha} B^dagger_{nj}(beta)
        std::vector<cplx> base(nm);
        for (int tau = 1; tau <= 2; ++tau)
            for (int l = 1; l <= L; ++l)
                for (int m = -l; m <= l; ++m)
                    base[(tau - 1) * h->half + celes::lm_index(l, m)] =
                        4.0 * e0 * std::exp(cplx(0, -m * al)) * celes::b_dagger(tau, l, m, pol[kk], b);
        const double kx = h->k * std::sin(b) * std::cos(al), ky = h->k * std::sin(b) * std::sin(al),
                     kz = h->k * std::cos(b);
        for (int64_t i = 0; i < N; ++i) {
            cplx ph = std::exp(cplx(0, kx * h->pos[3 * i] + ky * h->pos[3 * i + 1] + kz * h->pos[3 * i + 2]));
            cplx* dst = &h->a_in[((size_t)kk * N + i) * nm];
            for (int c = 0; c < nm; ++c) dst[c] = ph * base[c];
        }
    }
    h->K = K;
    h->have_solution = false;
    h->gaussian = false;
    h->pw_beta.assign(beta, beta + K);
    h->pw_alpha.assign(alpha, alpha + K);
    h->pw_pol.assign(pol, pol + K);
    h->pw_E0.resize(K);
    for (int kk = 0; kk < K; ++kk) h->pw_E0[kk] = E0 ? cplx(E0[2 * kk], E0[2 * kk + 1]) : cplx(1, 0);
    return CELES_OK;
}
int celes_set_plane_waves(celes_handle* h, int K, const double* beta, const double* alpha, const int* pol,
                          const double* E0) {
    return celes_guard([&] { return celes_set_plane_waves_impl(h, K, beta, alpha, pol, E0); });
}


static int celes_set_gaussian_beam_impl(celes_handle* h, double waist, const double* focus, double alpha_G, double E0_re,
                            double E0_im, int n_beta) {
    if (!h) return CELES_E_ARG;
    if (!(waist > 0) || !focus) return fail(h, CELES_E_ARG, "waist must be positive and focus non-null");
    if (n_beta <= 0) n_beta = 512;
    const int64_t N = h->N;
    const int nm = h->nmax, L = h->L;
    const double k = h->k;
    std::vector<double> xg(n_beta), wg(n_beta);
    celes::gauss_legendre(n_beta, xg.data(), wg.data());
    // beta nodes on [0, pi/2]; weight factor sin cos exp(-w^2 k^2 sin^2 / 4)
    std::vector<double> bet(n_beta), wb(n_beta);
    for (int q = 0; q < n_beta; ++q) {
        bet[q] = 0.25 * M_PI * (xg[q] + 1.0);
        double sb = std::sin(bet[q]), cb = std::cos(bet[q]);
        wb[q] = 0.25 * M_PI * wg[q] * sb * cb * std::exp(-waist * waist * k * k * sb * sb / 4.0);
    }
    // B^dagger table [q][n][j]
    std::vector<cplx> Bd((size_t)n_beta * nm * 2);
    for (int q = 0; q < n_beta; ++q)
        for (int tau = 1; tau <= 2; ++tau)
            for (int l = 1; l <= L; ++l)
                for (int m = -l; m <= l; ++m)
                    for (int j = 1; j <= 2; ++j)
                        Bd[((size_t)q * nm + (tau - 1) * h->half + celes::lm_index(l, m)) * 2 + (j - 1)] =
                            celes::b_dagger(tau, l, m, j, bet[q]);
    const cplx E0(E0_re, E0_im);
    const cplx pref = E0 * k * k * waist * waist / M_PI;
    h->a_in.assign((size_t)N * nm, cplx(0, 0));
    const cplx I(0, 1);
    auto ipow = [](int e) -> cplx {
        switch (((e % 4) + 4) % 4) {
            case 0: return {1, 0};
            case 1: return {0, 1};
            case 2: return {-1, 0};
            default: return {0, -1};
        }
    };
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        const double rx = h->pos[3 * i] - focus[0], ry = h->pos[3 * i + 1] - focus[1],
                     rz = h->pos[3 * i + 2] - focus[2];
        const double rho = std::hypot(rx, ry), phG = std::atan2(ry, rx);
        std::vector<cplx> acc(nm, cplx(0, 0));
        std::vector<double> J(L + 3);
        for (int q = 0; q < n_beta; ++q) {
            const double sb = std::sin(bet[q]), cb = std::cos(bet[q]);
            const double x = k * rho * sb;
            // J_0..J_{L+1}(x): downward recurrence from two library values
            if (x == 0.0) {
                std::fill(J.begin(), J.end(), 0.0);
                J[0] = 1.0;
            } else {
                J[L + 1] = std::cyl_bessel_j((double)(L + 1), x);
                J[L] = std::cyl_bessel_j((double)L, x);
                for (int nn = L; nn >= 1; --nn) J[nn - 1] = 2.0 * nn / x * J[nn] - J[nn + 1];
            }
            const cplx ax = std::exp(I * (k * rz * cb)) * wb[q];
            for (int l = 1; l <= L; ++l)
                for (int m = -l; m <= l; ++m) {
                    // I_{jn} / (2 pi), for j = 1, 2
                    const cplx t1 = std::exp(-I * alpha_G) * ipow(std::abs(m - 1)) *
                                    std::exp(-I * ((double)(m - 1) * phG)) * J[std::abs(m - 1)];
                    const cplx t2 = std::exp(I * alpha_G) * ipow(std::abs(m + 1)) *
                                    std::exp(-I * ((double)(m + 1) * phG)) * J[std::abs(m + 1)];
                    const cplx Ij1 = 2.0 * M_PI * 0.5 * (t1 + t2);
                    const cplx Ij2 = 2.0 * M_PI * 0.5 * (-I * t1 + I * t2);
                    for (int tau = 1; tau <= 2; ++tau) {
                        const int c = (tau - 1) * h->half + celes::lm_index(l, m);
                        const cplx* bd = &Bd[((size_t)q * nm + c) * 2];
                        acc[c] += ax * (bd[0] * Ij1 + bd[1] * Ij2);
                    }
                }
        }
        for (int c = 0; c < nm; ++c) h->a_in[(size_t)i * nm + c] = pref * acc[c];
    }
    h->K = 1;
    h->have_solution = false;
    h->gaussian = true;
    h->g_waist = waist;
    for (int c = 0; c < 3; ++c) h->g_focus[c] = focus[c];
    h->g_alpha = alpha_G;
    h->g_E0 = E0;
    return CELES_OK;
}
int celes_set_gaussian_beam(celes_handle* h, double waist, const double* focus, double alpha_G, double E0_re,
                            double E0_im, int n_beta) {
    return celes_guard([&] { return celes_set_gaussian_beam_impl(h, waist, focus, alpha_G, E0_re, E0_im, n_beta); });
}


static int celes_get_incident_impl(const celes_handle* h, double* a_out) {
    if (!h || !a_out) return CELES_E_ARG;
    if (h->K < 1) return CELES_E_STATE;
    std::memcpy(a_out, h->a_in.data(), h->a_in.size() * sizeof(cplx));
    return CELES_OK;
}
int celes_get_incident(const celes_handle* h, double* a_out) {
    return celes_guard([&] { return celes_get_incident_impl(h, a_out); });
}


static int celes_apply_W_impl(celes_handle* h, int precision, int K, const void* x_dev, void* y_dev, void* stream) {
    if (!h) return CELES_E_ARG;
    if (K < 1 || !x_dev || !y_dev) return fail(h, CELES_E_ARG, "K < 1 or null device pointer");
    hipStream_t s = (hipStream_t)stream;
    if (precision == CELES_FP64) return matvec<double>(h, (const cx<double>*)x_dev, (cx<double>*)y_dev, K, 0, s);
    if (precision == CELES_MIXED) return matvec<float>(h, (const cx<float>*)x_dev, (cx<float>*)y_dev, K, 0, s);
    return fail(h, CELES_E_ARG, "unknown precision");
}
int celes_apply_W(celes_handle* h, int precision, int K, const void* x_dev, void* y_dev, void* stream) {
    return celes_guard([&] { return celes_apply_W_impl(h, precision, K, x_dev, y_dev, stream); });
}


static int celes_apply_M_impl(celes_handle* h, int precision, int K, const void* x_dev, void* y_dev, void* stream) {
    if (!h) return CELES_E_ARG;
    if (K < 1 || !x_dev || !y_dev) return fail(h, CELES_E_ARG, "K < 1 or null device pointer");
    hipStream_t s = (hipStream_t)stream;
    if (precision == CELES_FP64) return matvec<double>(h, (const cx<double>*)x_dev, (cx<double>*)y_dev, K, 1, s);
    if (precision == CELES_MIXED) return matvec<float>(h, (const cx<float>*)x_dev, (cx<float>*)y_dev, K, 1, s);
    return fail(h, CELES_E_ARG, "unknown precision");
}
int celes_apply_M(celes_handle* h, int precision, int K, const void* x_dev, void* y_dev, void* stream) {
    return celes_guard([&] { return celes_apply_M_impl(h, precision, K, x_dev, y_dev, stream); });
}


static int celes_apply_preconditioner_impl(celes_handle* h, int precision, int K, const void* x_dev, void* y_dev,
                                           void* stream) {
    if (!h) return CELES_E_ARG;
    if (K < 1 || !x_dev || !y_dev || x_dev == y_dev) return fail(h, CELES_E_ARG, "K < 1, null or aliasing pointer");
    if (!h->pre) return fail(h, CELES_E_STATE, "no preconditioner built");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = h->N * h->nmax;
    int rc;
    if (precision == CELES_FP64)
        rc = K == 1 ? h->pre->apply<double>((const cx<double>*)x_dev, (cx<double>*)y_dev, s)
                    : h->pre->apply_multi<double>((const cx<double>*)x_dev, (cx<double>*)y_dev, K, n, nullptr, 0, s);
    else if (precision == CELES_MIXED)
        rc = K == 1 ? h->pre->apply<float>((const cx<float>*)x_dev, (cx<float>*)y_dev, s)
                    : h->pre->apply_multi<float>((const cx<float>*)x_dev, (cx<float>*)y_dev, K, n, nullptr, 0, s);
    else return fail(h, CELES_E_ARG, "unknown precision");
    return rc == CELES_OK ? CELES_OK : fail(h, rc, "preconditioner apply failed");
}
int celes_apply_preconditioner(celes_handle* h, int precision, int K, const void* x_dev, void* y_dev, void* stream) {
    return celes_guard([&] { return celes_apply_preconditioner_impl(h, precision, K, x_dev, y_dev, stream); });
}

static int celes_build_preconditioner_impl(celes_handle* h, double cuboid_edge) {
    if (!h) return CELES_E_ARG;
    h->pre.reset();
    ++h->pre_gen;
    if (cuboid_edge == 0) return CELES_OK;
    if (!std::isfinite(cuboid_edge)) return fail(h, CELES_E_ARG, "cuboid edge must be finite");
    // memory budget (Section 3.2.1: the LU storage grows as sum_j N_j^2),
    // checked before anything is allocated or launched
    double cap = h->opt.mem_cap_bytes;
    if (!(cap > 0)) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail(h, CELES_E_DEVICE, "hipMemGetInfo failed");
        cap = 0.9 * (double)free_b;
    }
    std::string msg;
    std::vector<int64_t> perm, offsets;
    if (cuboid_edge < 0) {
        if (celes::plan_cuboid_edge(h->N, h->pos.data(), h->L, h->opt.target_Nj, cap, &cuboid_edge, &offsets, &msg) != 0)
            return fail(h, CELES_E_OOM, msg);
    } else {
        celes::partition_cuboids(h->N, h->pos.data(), cuboid_edge, &perm, &offsets);
    }
    const double need = celes::BlockPrecond::precond_bytes(h->N, h->L, offsets);
    if (need > cap)
        return fail(h, CELES_E_OOM, "preconditioner needs " + std::to_string((long long)(need / (1 << 20))) +
                                        " MiB, above the cap of " + std::to_string((long long)(cap / (1 << 20))) + " MiB");
    auto p = std::make_unique<celes::BlockPrecond>();
    int rc = p->build(h->N, h->L, h->pos.data(), h->k, h->tq.data(), cuboid_edge,
                      h->opt.hankel == CELES_HANKEL_DIRECT ? 1 : 0, h->d_lut64.p, h->lut_lo, h->lut_dr,
                      (int)h->lut_n, &msg);
    if (rc != CELES_OK) return fail(h, rc, msg);
    h->pre = std::move(p);
    return CELES_OK;
}
int celes_build_preconditioner(celes_handle* h, double cuboid_edge) {
    return celes_guard([&] { return celes_build_preconditioner_impl(h, cuboid_edge); });
}

int celes_plan_preconditioner(int64_t N, const double* pos, int lmax, double target_Nj, double mem_cap_bytes,
                              double* edge_out, int64_t* nblocks_out, double* bytes_out, int64_t* max_Nj_out) {
    return celes_guard([&] {
        if (N < 1 || !pos || lmax < 1) return fail(nullptr, CELES_E_ARG, "N < 1, lmax < 1 or null positions");
        for (int64_t i = 0; i < 3 * N; ++i)
            if (!std::isfinite(pos[i])) return fail(nullptr, CELES_E_NONFINITE, "non-finite position");
        double edge = 0;
        std::vector<int64_t> offsets;
        std::string msg;
        if (celes::plan_cuboid_edge(N, pos, lmax, target_Nj, mem_cap_bytes, &edge, &offsets, &msg) != 0)
            return fail(nullptr, CELES_E_OOM, msg);
        int64_t mx = 0;
        for (size_t j = 0; j + 1 < offsets.size(); ++j) mx = std::max<int64_t>(mx, offsets[j + 1] - offsets[j]);
        if (edge_out) *edge_out = edge;
        if (nblocks_out) *nblocks_out = (int64_t)offsets.size() - 1;
        if (bytes_out) *bytes_out = celes::BlockPrecond::precond_bytes(N, lmax, offsets);
        if (max_Nj_out) *max_Nj_out = mx;
        return CELES_OK;
    });
}

int celes_preconditioner_info(const celes_handle* h, double* edge, int64_t* nblocks, double* bytes) {
    if (!h) return CELES_E_ARG;
    if (edge) *edge = h->pre ? h->pre->edge() : 0.0;
    if (nblocks) *nblocks = h->pre ? h->pre->num_blocks() : 0;
    if (bytes) *bytes = h->pre ? h->pre->bytes() : 0.0;
    return CELES_OK;
}


static int celes_solve_impl(celes_handle* h, const double* x0, double* b_out, celes_solve_info* info) {
    if (!h) return CELES_E_ARG;
    if (h->K < 1) return fail(h, CELES_E_STATE, "no incident field set");
    const bool mixed = h->opt.precision == CELES_MIXED;
    const bool bicg = h->opt.solver == CELES_SOLVER_BICGSTAB;
    int rc = ensure_solver_buffers(h, mixed);
    if (rc != CELES_OK) return rc;
    hipStream_t s = nullptr;
    const int64_t N = h->N, nm = h->nmax, n = N * nm;
    celes_solve_info inf{};
    h->b.assign((size_t)h->K * n, cplx(0, 0));
    auto t0 = std::chrono::steady_clock::now();
    int status = CELES_OK;
    double worst = 0;
    for (int kk = 0; kk < h->K; ++kk) {
        // rhs = T a_in
        std::vector<cx<double>> rhs(n), x(n);
        for (int64_t i = 0; i < N; ++i)
            for (int tau = 0; tau < 2; ++tau)
                for (int c = 0; c < h->half; ++c) {
                    int l = (int)std::floor(std::sqrt((double)(c + 1)));
                    while (l * (l + 2) < c + 1) ++l;
                    while ((l - 1) * (l + 1) >= c + 1) --l;
                    cplx q = h->tq[((size_t)i * 2 + tau) * h->L + (l - 1)];
                    cplx v = q * h->a_in[((size_t)kk * N + i) * nm + tau * h->half + c];
                    rhs[i * nm + tau * h->half + c] = {v.real(), v.imag()};
                }
        for (int64_t c = 0; c < n; ++c) {
            if (x0) {
                x[c] = {x0[2 * ((size_t)kk * n + c)], x0[2 * ((size_t)kk * n + c) + 1]};
                if (!std::isfinite(x[c].re) || !std::isfinite(x[c].im)) return fail(h, CELES_E_NONFINITE, "non-finite x0");
            } else {
                x[c] = {0, 0};
            }
        }
        double rn = 0;
        for (auto& v : rhs) rn += v.re * v.re + v.im * v.im;
        rn = std::sqrt(rn);
        cx<double>* drhs = h->d_rhs.as<cx<double>>();
        cx<double>* dx = h->d_x.as<cx<double>>();
        HIPCHK(h, hipMemcpy(drhs, rhs.data(), n * sizeof(cx<double>), hipMemcpyHostToDevice));
        HIPCHK(h, hipMemcpy(dx, x.data(), n * sizeof(cx<double>), hipMemcpyHostToDevice));
        double final_res = 0;
        double x0_res = 1.0;
        if (x0 && rn > 0) {
            // The initial guess enters with the complex weight alpha that
            // minimises ||rhs - alpha M x0|| (one FP64 mat-vec): alpha =
            // (M x0)^H rhs / ||M x0||^2, residual^2 = ||rhs||^2 - |(M x0)^H
            // rhs|^2 / ||M x0||^2 <= ||rhs||^2.  It is used if that beats
            // x0 = 0; alpha = 1 for a guess that is already the solution.
            double mv = 0;
            int rc0 = CELES_OK;
            (void)residual64(h, drhs, dx, h->d_r.as<cx<double>>(), s, &rc0, &mv);   // d_w = M x0
            inf.matvecs++;
            if (rc0 != CELES_OK) return rc0;
            cx<double> d1, d2;
            const cx<double>* mx = h->d_w.as<cx<double>>();
            celes::vec_dots<double>(mx, 0, 1, drhs, n, h->d_partial.as<cx<double>>(), h->d_h.as<cx<double>>(), s);
            HIPCHK(h, hipMemcpyAsync(&d1, h->d_h.p, sizeof(d1), hipMemcpyDeviceToHost, s));
            celes::vec_dots<double>(mx, 0, 1, mx, n, h->d_partial.as<cx<double>>(), h->d_h.as<cx<double>>(), s);
            HIPCHK(h, hipMemcpyAsync(&d2, h->d_h.p, sizeof(d2), hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            const double proj = d2.re > 0 ? (d1.re * d1.re + d1.im * d1.im) / d2.re : 0.0;
            if (std::isfinite(proj) && proj > 0) {
                const cplx alpha = cplx(d1.re, d1.im) / d2.re;
                for (auto& v : x) {
                    const cplx z = alpha * cplx(v.re, v.im);
                    v = {z.real(), z.imag()};
                }
                HIPCHK(h, hipMemcpy(dx, x.data(), n * sizeof(cx<double>), hipMemcpyHostToDevice));
                inf.x0_used = 1;
                x0_res = std::sqrt(std::max(0.0, rn * rn - proj)) / rn;
            } else {
                HIPCHK(h, hipMemset(dx, 0, n * sizeof(cx<double>)));
            }
        }
        inf.x0_residual = std::max(inf.x0_residual, x0_res);
        if (rn == 0) {
            HIPCHK(h, hipMemset(dx, 0, n * sizeof(cx<double>)));
        } else if (!mixed) {
            GmresResult gr;
            if (bicg)
                rc = bicgstab_device<double>(h, drhs, dx, h->opt.tol, h->opt.maxiter, rn, &gr, s,
                                             h->d_V.as<cx<double>>());
            else
                rc = gmres_device<double>(h, drhs, dx, h->opt.tol, h->opt.maxiter, rn, &gr, s,
                                          h->d_V.as<cx<double>>(), h->d_w.as<cx<double>>(), h->d_z.as<cx<double>>());
            if (rc != CELES_OK) return rc;
            inf.iterations += gr.iterations;
            inf.refinements += gr.restarts;
            inf.matvecs += gr.matvecs;
            inf.matvec_seconds += gr.matvec_seconds;
            double mv = 0;
            double r = residual64(h, drhs, dx, h->d_r.as<cx<double>>(), s, &rc, &mv) / rn;
            if (rc != CELES_OK) return rc;
            inf.matvecs++;
            inf.matvec_seconds += mv;
            final_res = r;
            if (gr.breakdown || !std::isfinite(r)) status = CELES_E_BREAKDOWN;
            else if (r > h->opt.tol && status == CELES_OK) status = CELES_E_NOCONV;
        } else {
            // iterative refinement: FP64 residual, complex64 GMRES correction
            int inner_left = h->opt.maxiter;
            double mv = 0;
            double r = residual64(h, drhs, dx, h->d_r.as<cx<double>>(), s, &rc, &mv) / rn;
            if (rc != CELES_OK) return rc;
            inf.matvecs++;
            for (int it = 0; it < h->opt.max_refinements && r > h->opt.tol && inner_left > 0; ++it) {
                // correction problem M d = r in complex64, from d = 0
                celes::vec_to32(h->d_r.as<cx<double>>(), h->d_r32.as<cx<float>>(), n, s);
                HIPCHK(h, hipMemsetAsync(h->d_x32.p, 0, n * sizeof(cx<float>), s));
                GmresResult gr;
                double rnorm = r * rn;
                double inner = std::max(h->opt.inner_tol, 0.5 * h->opt.tol / r);
                if (bicg)
                    rc = bicgstab_device<float>(h, h->d_r32.as<cx<float>>(), h->d_x32.as<cx<float>>(), inner,
                                                inner_left, rnorm, &gr, s, h->d_V32.as<cx<float>>());
                else
                    rc = gmres_device<float>(h, h->d_r32.as<cx<float>>(), h->d_x32.as<cx<float>>(), inner,
                                             inner_left, rnorm, &gr, s, h->d_V32.as<cx<float>>(),
                                             h->d_w32.as<cx<float>>(), h->d_z32.as<cx<float>>());
                if (rc != CELES_OK) return rc;
                inf.iterations += gr.iterations;
                inf.matvecs += gr.matvecs;
                inf.matvec_seconds += gr.matvec_seconds;
                inner_left -= std::max(1, gr.iterations);
                celes::vec_acc32(h->d_x32.as<cx<float>>(), dx, n, s);
                double rnew = residual64(h, drhs, dx, h->d_r.as<cx<double>>(), s, &rc, &mv) / rn;
                if (rc != CELES_OK) return rc;
                inf.matvecs++;
                inf.refinements++;
                if (h->opt.verbose) std::fprintf(stderr, "refinement %d: residual %.3e (inner its %d)\n", it, rnew, gr.iterations);
                if (!(rnew < r) && gr.breakdown) break;
                r = rnew;
            }
            inf.matvec_seconds += mv;
            final_res = r;
            if (!std::isfinite(r)) status = CELES_E_BREAKDOWN;
            else if (r > h->opt.tol && status == CELES_OK) status = CELES_E_NOCONV;
        }
        worst = std::max(worst, final_res);
        HIPCHK(h, hipMemcpy(x.data(), dx, n * sizeof(cx<double>), hipMemcpyDeviceToHost));
        for (int64_t c = 0; c < n; ++c) h->b[(size_t)kk * n + c] = cplx(x[c].re, x[c].im);
    }
    auto t1 = std::chrono::steady_clock::now();
    inf.seconds = std::chrono::duration<double>(t1 - t0).count();
    inf.rel_residual = worst;
    inf.status = status;
    h->have_solution = true;
    if (b_out) std::memcpy(b_out, h->b.data(), h->b.size() * sizeof(cplx));
    if (info) *info = inf;
    const char* name = bicg ? "BiCGSTAB" : "GMRES";
    if (status == CELES_E_NOCONV) h->err = std::string(name) + " did not reach the tolerance";
    if (status == CELES_E_BREAKDOWN) h->err = std::string(name) + " breakdown (non-finite iterate)";
    return status;
}
int celes_solve(celes_handle* h, const double* x0, double* b_out, celes_solve_info* info) {
    return celes_guard([&] { return celes_solve_impl(h, x0, b_out, info); });
}

// Sub-ensemble initial guess (Section 4.2): a problem of the spheres idx
// alone, with their rows of the incident coefficients, solved with this
// problem's options; its solution is scattered into x0 (zero elsewhere).
static int celes_subsystem_guess_impl(celes_handle* h, int64_t n_sub, const int64_t* idx, double cuboid_edge,
                                      double* x0_out, celes_solve_info* info) {
    if (!h) return CELES_E_ARG;
    if (n_sub < 1 || n_sub > h->N || !idx || !x0_out) return fail(h, CELES_E_ARG, "n_sub out of range or null array");
    if (h->K < 1) return fail(h, CELES_E_STATE, "no incident field set");
    std::vector<char> seen(h->N, 0);
    for (int64_t j = 0; j < n_sub; ++j) {
        if (idx[j] < 0 || idx[j] >= h->N) return fail(h, CELES_E_ARG, "sphere index out of range");
        if (seen[idx[j]]) return fail(h, CELES_E_ARG, "repeated sphere index");
        seen[idx[j]] = 1;
    }
    const int nm = h->nmax;
    std::vector<double> pos(3 * n_sub), rad(n_sub), ns(2 * n_sub);
    for (int64_t j = 0; j < n_sub; ++j) {
        const int64_t i = idx[j];
        for (int c = 0; c < 3; ++c) pos[3 * j + c] = h->pos[3 * i + c];
        rad[j] = h->radius[i];
        ns[2 * j] = h->nsph[i].real();
        ns[2 * j + 1] = h->nsph[i].imag();
    }
    celes_options o = h->opt;
    o.cuboid_edge = 0.0;
    celes_handle* raw = nullptr;
    int rc = celes_create_impl(&raw, n_sub, pos.data(), rad.data(), ns.data(), h->n0, h->wavelength, h->L, &o);
    if (rc != CELES_OK) return fail(h, rc, "sub-ensemble: " + g_create_error);
    std::unique_ptr<celes_handle> sub(raw);
    // a sphere's incident coefficients depend on its own position only
    sub->K = h->K;
    sub->a_in.assign((size_t)h->K * n_sub * nm, cplx(0, 0));
    for (int kk = 0; kk < h->K; ++kk)
        for (int64_t j = 0; j < n_sub; ++j)
            std::copy_n(&h->a_in[((size_t)kk * h->N + idx[j]) * nm], nm, &sub->a_in[((size_t)kk * n_sub + j) * nm]);
    if (cuboid_edge > 0 && (rc = celes_build_preconditioner_impl(sub.get(), cuboid_edge)) != CELES_OK)
        return fail(h, rc, "sub-ensemble preconditioner: " + sub->err);
    std::vector<double> bs((size_t)h->K * n_sub * nm * 2);
    celes_solve_info si{};
    rc = celes_solve_impl(sub.get(), nullptr, bs.data(), &si);
    if (info) *info = si;
    if (rc != CELES_OK && rc != CELES_E_NOCONV) return fail(h, rc, "sub-ensemble solve: " + sub->err);
    std::fill(x0_out, x0_out + (size_t)h->K * h->N * nm * 2, 0.0);
    for (int kk = 0; kk < h->K; ++kk)
        for (int64_t j = 0; j < n_sub; ++j)
            std::copy_n(&bs[((size_t)kk * n_sub + j) * nm * 2], 2 * nm, &x0_out[((size_t)kk * h->N + idx[j]) * nm * 2]);
    if (rc == CELES_E_NOCONV) h->err = "sub-ensemble solve: " + sub->err;
    return rc;
}
int celes_subsystem_guess(celes_handle* h, int64_t n_sub, const int64_t* idx, double cuboid_edge, double* x0_out,
                          celes_solve_info* info) {
    return celes_guard([&] { return celes_subsystem_guess_impl(h, n_sub, idx, cuboid_edge, x0_out, info); });
}


static int celes_mie_coefficients_impl(int lmax, double kR, double m_re, double m_im, double* Q_out) {
    if (lmax < 1 || !(kR > 0) || !Q_out) return CELES_E_ARG;
    std::vector<cplx> q1(lmax), q2(lmax);
    celes::mie_Q(lmax, kR, cplx(m_re, m_im), q1.data(), q2.data());
    for (int l = 0; l < lmax; ++l) {
        Q_out[2 * l] = q1[l].real();
        Q_out[2 * l + 1] = q1[l].imag();
        Q_out[2 * (lmax + l)] = q2[l].real();
        Q_out[2 * (lmax + l) + 1] = q2[l].imag();
    }
    return CELES_OK;
}
int celes_mie_coefficients(int lmax, double kR, double m_re, double m_im, double* Q_out) {
    return celes_guard([&] { return celes_mie_coefficients_impl(lmax, kR, m_re, m_im, Q_out); });
}


static int celes_translation_tables_impl(int lmax, double* a5_out, double* b5im_out) {
    if (lmax < 1 || lmax > CELES_MAX_LMAX || !a5_out || !b5im_out) return CELES_E_ARG;
    const int W = 2 * lmax + 1;
    for (int l = 1; l <= lmax; ++l)
        for (int m = -lmax; m <= lmax; ++m)
            for (int lp = 1; lp <= lmax; ++lp)
                for (int mp = -lmax; mp <= lmax; ++mp)
                    for (int p = 0; p <= 2 * lmax; ++p) {
                        size_t o = ((((size_t)(l - 1) * W + (m + lmax)) * lmax + (lp - 1)) * W + (mp + lmax)) * W + p;
                        bool ok = std::abs(m) <= l && std::abs(mp) <= lp;
                        a5_out[o] = ok ? celes::a5_coef(l, m, lp, mp, p) : 0.0;
                        b5im_out[o] = ok ? celes::b5im_coef(l, m, lp, mp, p) : 0.0;
                    }
    return CELES_OK;
}
int celes_translation_tables(int lmax, double* a5_out, double* b5im_out) {
    return celes_guard([&] { return celes_translation_tables_impl(lmax, a5_out, b5im_out); });
}


// ---------------------------------------------------------------------------
// observables (Appendix D and the SVWF definitions of Appendix A.1)
// ---------------------------------------------------------------------------
// F(theta, phi) from the sphere sums c_n = sum_i e^{-ik rhat.r_i} b^i_n
// (Appendix D): f_{1lm} = (-i)^{l+1} e (i m pi e_theta - tau e_phi),
// f_{2lm} = (-i)^l e (tau e_theta + i m pi e_phi), e = e^{i m phi}/sqrt(2l(l+1))
static void far_field_from_sums(const celes_handle* h, double th, double ph, const cx<double>* c, cplx F[3]) {
    const int L = h->L;
    const double st = std::sin(th), ct = std::cos(th), sp = std::sin(ph), cp = std::cos(ph);
    const double et[3] = {ct * cp, ct * sp, -st};
    const double ep[3] = {-sp, cp, 0.0};
    F[0] = F[1] = F[2] = 0;
    const cplx I(0, 1);
    for (int l = 1; l <= L; ++l) {
        const cplx mi_l = std::pow(cplx(0, -1), l);
        for (int m = -l; m <= l; ++m) {
            double pi, tau;
            celes::pi_tau(l, std::abs(m), th, &pi, &tau);
            const cplx e = std::exp(cplx(0, m * ph)) / std::sqrt(2.0 * l * (l + 1));
            const int c1 = celes::lm_index(l, m), c2 = h->half + c1;
            const cplx a1 = cplx(c[c1].re, c[c1].im) * mi_l * cplx(0, -1) * e, a2 = cplx(c[c2].re, c[c2].im) * mi_l * e;
            const cplx ut = a1 * (I * (double)m * pi) + a2 * tau;
            const cplx up = -a1 * tau + a2 * (I * (double)m * pi);
            for (int q = 0; q < 3; ++q) F[q] += ut * et[q] + up * ep[q];
        }
    }
}

// Far field of right-hand side kk at nd directions (theta, phi): the sphere
// sums on the device (ff_sums_launch) in chunks of directions, the angular
// functions on the host.  F: [nd][3].
static int far_field_batch(celes_handle* h, int kk, int64_t nd, const double* theta, const double* phi,
                           std::vector<std::array<cplx, 3>>* F) {
    const int64_t N = h->N;
    const int nm = h->nmax;
    F->assign(nd, {cplx(0, 0), cplx(0, 0), cplx(0, 0)});
    if (nd == 0) return CELES_OK;
    const int64_t chunk = std::min<int64_t>(nd, 1 << 17);
    if (!h->d_ffb.ensure((size_t)N * nm * sizeof(cx<double>)) || !h->d_ffdir.ensure((size_t)chunk * 3 * sizeof(double)) ||
        !h->d_ffc.ensure((size_t)chunk * nm * sizeof(cx<double>)))
        return fail(h, CELES_E_OOM, "cannot allocate far-field buffers");
    HIPCHK(h, hipMemcpy(h->d_ffb.p, &h->b[(size_t)kk * N * nm], (size_t)N * nm * sizeof(cx<double>),
                        hipMemcpyHostToDevice));
    std::vector<double> dirs((size_t)chunk * 3);
    std::vector<cx<double>> c((size_t)chunk * nm);
    for (int64_t d0 = 0; d0 < nd; d0 += chunk) {
        const int64_t nc = std::min(chunk, nd - d0);
        for (int64_t d = 0; d < nc; ++d) {
            const double st = std::sin(theta[d0 + d]), ct = std::cos(theta[d0 + d]);
            dirs[3 * d] = st * std::cos(phi[d0 + d]);
            dirs[3 * d + 1] = st * std::sin(phi[d0 + d]);
            dirs[3 * d + 2] = ct;
        }
        HIPCHK(h, hipMemcpy(h->d_ffdir.p, dirs.data(), (size_t)nc * 3 * sizeof(double), hipMemcpyHostToDevice));
        if (celes::ff_sums_launch(h->d_px.as<double>(), h->d_py.as<double>(), h->d_pz.as<double>(),
                                  h->d_ffb.as<cx<double>>(), N, nm, h->d_ffdir.as<double>(), nc, h->k,
                                  h->d_ffc.as<cx<double>>(), nullptr) != 0)
            return fail(h, CELES_E_DEVICE, "far-field launch failed");
        HIPCHK(h, hipMemcpy(c.data(), h->d_ffc.p, (size_t)nc * nm * sizeof(cx<double>), hipMemcpyDeviceToHost));
#pragma omp parallel for schedule(static)
        for (int64_t d = 0; d < nc; ++d)
            far_field_from_sums(h, theta[d0 + d], phi[d0 + d], &c[(size_t)d * nm], (*F)[d0 + d].data());
    }
    return CELES_OK;
}


static int celes_far_field_impl(celes_handle* h, int64_t ndir, const double* theta, const double* phi, double* F_out) {
    if (!h) return CELES_E_ARG;
    if (!h->have_solution) return fail(h, CELES_E_STATE, "no solution");
    if (ndir < 0 || (ndir > 0 && (!theta || !phi || !F_out))) return fail(h, CELES_E_ARG, "bad direction arrays");
    std::vector<std::array<cplx, 3>> F;
    for (int kk = 0; kk < h->K; ++kk) {
        int rc = far_field_batch(h, kk, ndir, theta, phi, &F);
        if (rc != CELES_OK) return rc;
        for (int64_t d = 0; d < ndir; ++d)
            for (int q = 0; q < 3; ++q) {
                F_out[(((size_t)kk * ndir + d) * 3 + q) * 2] = F[d][q].real();
                F_out[(((size_t)kk * ndir + d) * 3 + q) * 2 + 1] = F[d][q].imag();
            }
    }
    return CELES_OK;
}
int celes_far_field(celes_handle* h, int64_t ndir, const double* theta, const double* phi, double* F_out) {
    return celes_guard([&] { return celes_far_field_impl(h, ndir, theta, phi, F_out); });
}

// S11 as the paper's validation obtains it: |F|^2 averaged over the solved
// right-hand sides of several problems (e.g. TE and TM runs) and over n_phi
// equally spaced azimuths
static int celes_s11_impl(celes_handle* const* hs, int nh, int64_t n_theta, const double* theta, int n_phi,
                          double* out) {
    if (nh < 1 || !hs || n_theta < 0 || n_phi < 1 || (n_theta > 0 && (!theta || !out))) return CELES_E_ARG;
    int runs = 0;
    for (int j = 0; j < nh; ++j) {
        celes_handle* h = hs[j];
        if (!h) return CELES_E_ARG;
        if (!h->have_solution) return fail(h, CELES_E_STATE, "no solution");
        if (h->k != hs[0]->k) return fail(h, CELES_E_ARG, "problems of different wavenumbers");
        runs += h->K;
    }
    const int64_t nd = n_theta * n_phi;
    std::vector<double> th(nd), ph(nd);
    for (int64_t t = 0; t < n_theta; ++t)
        for (int q = 0; q < n_phi; ++q) {
            th[t * n_phi + q] = theta[t];
            ph[t * n_phi + q] = 2.0 * M_PI * q / n_phi;
        }
    std::vector<double> acc(n_theta, 0.0);
    std::vector<std::array<cplx, 3>> F;
    for (int j = 0; j < nh; ++j)
        for (int kk = 0; kk < hs[j]->K; ++kk) {
            int rc = far_field_batch(hs[j], kk, nd, th.data(), ph.data(), &F);
            if (rc != CELES_OK) return rc;
            for (int64_t d = 0; d < nd; ++d) acc[d / n_phi] += std::norm(F[d][0]) + std::norm(F[d][1]) + std::norm(F[d][2]);
        }
    for (int64_t t = 0; t < n_theta; ++t) out[t] = acc[t] / ((double)runs * n_phi);
    return CELES_OK;
}
int celes_s11(celes_handle* const* hs, int nh, int64_t n_theta, const double* theta, int n_phi, double* out) {
    return celes_guard([&] { return celes_s11_impl(hs, nh, n_theta, theta, n_phi, out); });
}


static int celes_cross_sections_impl(celes_handle* h, double* C_ext, double* C_sca, double* C_abs) {
    if (!h) return CELES_E_ARG;
    if (!h->have_solution) return fail(h, CELES_E_STATE, "no solution");
    const int64_t N = h->N;
    const int nm = h->nmax, L = h->L;
    const double k = h->k;
    // quadrature sized from the band limit L + k D (D: cluster diameter)
    double cen[3] = {0, 0, 0};
    for (int64_t i = 0; i < N; ++i)
        for (int c = 0; c < 3; ++c) cen[c] += h->pos[3 * i + c] / N;
    double D = 0;
    for (int64_t i = 0; i < N; ++i) {
        double t = 0;
        for (int c = 0; c < 3; ++c) t += (h->pos[3 * i + c] - cen[c]) * (h->pos[3 * i + c] - cen[c]);
        D = std::max(D, 2.0 * std::sqrt(t));
    }
    const int band = (int)(L + k * D) + 10;
    const int nt = band + 1, nph = 2 * band + 2;
    std::vector<double> xg(nt), wg(nt);
    celes::gauss_legendre(nt, xg.data(), wg.data());
    for (int kk = 0; kk < h->K; ++kk) {
        double ext = 0, ab = 0;
        for (int64_t i = 0; i < N; ++i)
            for (int tau = 0; tau < 2; ++tau)
                for (int c = 0; c < h->half; ++c) {
                    const size_t o = ((size_t)kk * N + i) * nm + tau * h->half + c;
                    ext += std::real(std::conj(h->a_in[o]) * h->b[o]);
                    int l = (int)std::floor(std::sqrt((double)(c + 1)));
                    while (l * (l + 2) < c + 1) ++l;
                    while ((l - 1) * (l + 1) >= c + 1) --l;
                    const cplx q = h->tq[((size_t)i * 2 + tau) * L + (l - 1)];
                    if (std::abs(q) > 0) ab += std::norm(h->b[o]) * (std::real(1.0 / q) + 1.0);
                }
        if (C_ext) C_ext[kk] = -M_PI / (k * k) * ext;
        if (C_abs) C_abs[kk] = -M_PI / (k * k) * ab;
        if (C_sca) {
            const int64_t nd = (int64_t)nt * nph;
            std::vector<double> th(nd), ph(nd);
            for (int a = 0; a < nt; ++a)
                for (int bq = 0; bq < nph; ++bq) {
                    th[(int64_t)a * nph + bq] = std::acos(xg[a]);
                    ph[(int64_t)a * nph + bq] = 2.0 * M_PI * bq / nph;
                }
            std::vector<std::array<cplx, 3>> F;
            int rc = far_field_batch(h, kk, nd, th.data(), ph.data(), &F);
            if (rc != CELES_OK) return rc;
            double sum = 0;
            for (int64_t d = 0; d < nd; ++d)
                sum += wg[d / nph] * (2.0 * M_PI / nph) * (std::norm(F[d][0]) + std::norm(F[d][1]) + std::norm(F[d][2]));
            C_sca[kk] = sum / (k * k);
        }
    }
    return CELES_OK;
}
int celes_cross_sections(celes_handle* h, double* C_ext, double* C_sca, double* C_abs) {
    return celes_guard([&] { return celes_cross_sections_impl(h, C_ext, C_sca, C_abs); });
}


// Power flux of a Gaussian beam (Appendix D): the transmitted power is the
// flux of g_in + g_sca through the upper hemisphere at infinity, the reflected
// power that of g_sca through the lower one, with g_sca = (i / 2 pi) F the
// stationary-phase pattern of E_sca -> e^{ikr}/(kr) F; absorbed power from
// the Mie coefficients.  Quadrature: Gauss-Legendre in the polar angle (a
// dense set inside the beam's cone sin(beta) < 8/(k w), band-limited sets
// elsewhere), uniform in the azimuth.
static int celes_power_flux_impl(celes_handle* h, int n_beta, int n_alpha, double* out) {
    if (!h || !out) return CELES_E_ARG;
    if (!h->have_solution) return fail(h, CELES_E_STATE, "no solution");
    if (!h->gaussian) return fail(h, CELES_E_STATE, "power flux needs a Gaussian beam (finite incident power)");
    const int64_t N = h->N;
    const int nm = h->nmax, L = h->L;
    const double k = h->k, w = h->g_waist;
    double D = 0;
    for (int64_t i = 0; i < N; ++i) {
        const double* r = &h->pos[3 * i];
        D = std::max(D, 2.0 * std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]));
    }
    const int band = (int)(L + k * D) + 10;
    const int nb = n_beta > 0 ? n_beta : band + 1;
    const int na = n_alpha > 0 ? n_alpha : 2 * band + 2;
    const int nbeam = 64;
    const double b1 = std::min(M_PI / 2, std::asin(std::min(1.0, 8.0 / (k * w))));
    // polar nodes and weights (sin(beta) included): forward, backward
    std::vector<double> fb, fw, bb, bw;
    auto gl = [&](double a, double c, int n, std::vector<double>* xs, std::vector<double>* ws) {
        std::vector<double> x(n), wt(n);
        celes::gauss_legendre(n, x.data(), wt.data());
        for (int q = 0; q < n; ++q) {
            const double t = 0.5 * (c - a) * (x[q] + 1.0) + a;
            xs->push_back(t);
            ws->push_back(0.5 * (c - a) * wt[q] * std::sin(t));
        }
    };
    gl(0.0, b1, nbeam, &fb, &fw);
    if (b1 < M_PI / 2) gl(b1, M_PI / 2, nb, &fb, &fw);
    gl(M_PI / 2, M_PI, nb, &bb, &bw);
    const double wa = 2.0 * M_PI / na;
    const cplx I(0, 1);
    const cplx gs = I / (2.0 * M_PI);
    for (int kk = 0; kk < h->K; ++kk) {
        double P0 = 0, Tn = 0, Rn = 0;
        std::vector<std::array<cplx, 3>> FF, FB;
        {
            const int64_t nf = (int64_t)fb.size() * na, nbk = (int64_t)bb.size() * na;
            std::vector<double> th(std::max(nf, nbk)), ph(std::max(nf, nbk));
            for (int64_t d = 0; d < nf; ++d) {
                th[d] = fb[d / na];
                ph[d] = wa * (d % na);
            }
            int rc = far_field_batch(h, kk, nf, th.data(), ph.data(), &FF);
            if (rc != CELES_OK) return rc;
            for (int64_t d = 0; d < nbk; ++d) {
                th[d] = bb[d / na];
                ph[d] = wa * (d % na);
            }
            rc = far_field_batch(h, kk, nbk, th.data(), ph.data(), &FB);
            if (rc != CELES_OK) return rc;
        }
#pragma omp parallel for reduction(+ : P0, Tn) collapse(2) schedule(static)
        for (int q = 0; q < (int)fb.size(); ++q)
            for (int a = 0; a < na; ++a) {
                const double be = fb[q], al = wa * a;
                const cplx* F = FF[(size_t)q * na + a].data();
                const double sa = std::sin(al), ca = std::cos(al), sbt = std::sin(be), cbt = std::cos(be);
                const cplx Fa = F[0] * -sa + F[1] * ca;
                const cplx Fb = F[0] * (cbt * ca) + F[1] * (cbt * sa) - F[2] * sbt;
                const double g = k * k * w * w / (4.0 * M_PI) * cbt * std::exp(-(w * k * sbt) * (w * k * sbt) / 4.0);
                const double kr = k * (sbt * ca * h->g_focus[0] + sbt * sa * h->g_focus[1] + cbt * h->g_focus[2]);
                const cplx ph = h->g_E0 * std::exp(cplx(0, -kr));
                const cplx ga = g * std::cos(al - h->g_alpha) * ph, gb = g * std::sin(al - h->g_alpha) * ph;
                P0 += fw[q] * wa * (std::norm(ga) + std::norm(gb));
                Tn += fw[q] * wa * (std::norm(ga + gs * Fa) + std::norm(gb + gs * Fb));
            }
#pragma omp parallel for reduction(+ : Rn) collapse(2) schedule(static)
        for (int q = 0; q < (int)bb.size(); ++q)
            for (int a = 0; a < na; ++a) {
                const cplx* F = FB[(size_t)q * na + a].data();
                Rn += bw[q] * wa * (std::norm(F[0]) + std::norm(F[1]) + std::norm(F[2])) / (4.0 * M_PI * M_PI);
            }
        double ab = 0;
        for (int64_t i = 0; i < N; ++i)
            for (int tau = 0; tau < 2; ++tau)
                for (int c = 0; c < h->half; ++c) {
                    const size_t o = ((size_t)kk * N + i) * nm + tau * h->half + c;
                    int l = (int)std::floor(std::sqrt((double)(c + 1)));
                    while (l * (l + 2) < c + 1) ++l;
                    while ((l - 1) * (l + 1) >= c + 1) --l;
                    const cplx qv = h->tq[((size_t)i * 2 + tau) * L + (l - 1)];
                    if (std::abs(qv) > 0) ab += std::norm(h->b[o]) * (std::real(1.0 / qv) + 1.0);
                }
        out[4 * kk + 0] = 4.0 * M_PI * M_PI / (k * k) * P0;
        out[4 * kk + 1] = Rn / P0;
        out[4 * kk + 2] = Tn / P0;
        out[4 * kk + 3] = -ab / (4.0 * M_PI) / P0;
    }
    return CELES_OK;
}

int celes_power_flux(celes_handle* h, int n_beta, int n_alpha, double* out) {
    return celes_guard([&] { return celes_power_flux_impl(h, n_beta, n_alpha, out); });
}

static int celes_near_field_impl(celes_handle* h, int64_t npt, const double* pts, int add_incident, double* E_out) {
    if (!h) return CELES_E_ARG;
    if (!h->have_solution) return fail(h, CELES_E_STATE, "no solution");
    if (npt < 0 || (npt > 0 && (!pts || !E_out))) return fail(h, CELES_E_ARG, "bad point arrays");
    if (npt == 0) return CELES_OK;
    const int64_t N = h->N;
    const int nm = h->nmax;
    const double k = h->k;
    celes::DevBuf d_pts, d_E, d_kv, d_amp;
    if (!d_pts.ensure((size_t)npt * 3 * sizeof(double)) || !d_E.ensure((size_t)npt * 3 * sizeof(cx<double>)) ||
        !h->d_ffb.ensure((size_t)N * nm * sizeof(cx<double>)))
        return fail(h, CELES_E_OOM, "cannot allocate near-field buffers");
    HIPCHK(h, hipMemcpy(d_pts.p, pts, (size_t)npt * 3 * sizeof(double), hipMemcpyHostToDevice));
    // incident field as a plane-wave superposition: one wave, or the angular
    // spectrum of the Gaussian beam (Appendix C, small-beta polarisation form)
    std::vector<double> kv;
    std::vector<cx<double>> amp;
    for (int kk = 0; kk < h->K; ++kk) {
        HIPCHK(h, hipMemcpy(h->d_ffb.p, &h->b[(size_t)kk * N * nm], (size_t)N * nm * sizeof(cx<double>),
                            hipMemcpyHostToDevice));
        if (celes::nf_scattered_launch(h->d_px.as<double>(), h->d_py.as<double>(), h->d_pz.as<double>(),
                                       h->d_ffb.as<cx<double>>(), N, h->L, d_pts.as<double>(), npt, k,
                                       d_E.as<cx<double>>(), nullptr) != 0)
            return fail(h, CELES_E_DEVICE, "near-field launch failed");
        if (add_incident) {
            kv.clear();
            amp.clear();
            double origin[3] = {0, 0, 0};
            if (!h->gaussian) {
                const double be = h->pw_beta[kk], al = h->pw_alpha[kk];
                kv = {k * std::sin(be) * std::cos(al), k * std::sin(be) * std::sin(al), k * std::cos(be)};
                double e[3];
                if (h->pw_pol[kk] == 1) { e[0] = -std::sin(al); e[1] = std::cos(al); e[2] = 0; }
                else { e[0] = std::cos(be) * std::cos(al); e[1] = std::cos(be) * std::sin(al); e[2] = -std::sin(be); }
                for (int c = 0; c < 3; ++c) {
                    const cplx v = h->pw_E0[kk] * e[c];
                    amp.push_back({v.real(), v.imag()});
                }
            } else {
                const int nb = 256, na = 256;
                std::vector<double> xg(nb), wg(nb);
                celes::gauss_legendre(nb, xg.data(), wg.data());
                const double w = h->g_waist;
                for (int c = 0; c < 3; ++c) origin[c] = h->g_focus[c];
                for (int bq = 0; bq < nb; ++bq) {
                    const double be = 0.25 * M_PI * (xg[bq] + 1.0), wb = 0.25 * M_PI * wg[bq];
                    const double sb = std::sin(be), cb = std::cos(be);
                    const double gq = k * k * w * w / (4 * M_PI) * sb * cb * std::exp(-(w * k * sb) * (w * k * sb) / 4);
                    for (int aq = 0; aq < na; ++aq) {
                        const double al = 2 * M_PI * aq / na;
                        const double ca = std::cos(al), sa = std::sin(al);
                        const double pa = std::cos(al - h->g_alpha), qa = std::sin(al - h->g_alpha);
                        const double pol[3] = {pa * (-sa) + qa * cb * ca, pa * ca + qa * cb * sa, -qa * sb};
                        const cplx f = h->g_E0 * (wb * 2 * M_PI / na * gq);
                        kv.push_back(k * sb * ca);
                        kv.push_back(k * sb * sa);
                        kv.push_back(k * cb);
                        for (int c = 0; c < 3; ++c) amp.push_back({(f * pol[c]).real(), (f * pol[c]).imag()});
                    }
                }
            }
            const int64_t nn = (int64_t)kv.size() / 3;
            if (!d_kv.ensure(kv.size() * sizeof(double)) || !d_amp.ensure(amp.size() * sizeof(cx<double>)))
                return fail(h, CELES_E_OOM, "cannot allocate incident-field nodes");
            HIPCHK(h, hipMemcpy(d_kv.p, kv.data(), kv.size() * sizeof(double), hipMemcpyHostToDevice));
            HIPCHK(h, hipMemcpy(d_amp.p, amp.data(), amp.size() * sizeof(cx<double>), hipMemcpyHostToDevice));
            if (celes::nf_planewaves_launch(d_kv.as<double>(), d_amp.as<cx<double>>(), nn, origin[0], origin[1],
                                            origin[2], d_pts.as<double>(), npt, d_E.as<cx<double>>(), nullptr) != 0)
                return fail(h, CELES_E_DEVICE, "incident near-field launch failed");
        }
        HIPCHK(h, hipMemcpy(E_out + (size_t)kk * npt * 3 * 2, d_E.p, (size_t)npt * 3 * sizeof(cx<double>),
                            hipMemcpyDeviceToHost));
    }
    return CELES_OK;
}
int celes_near_field(celes_handle* h, int64_t npt, const double* pts, int add_incident, double* E_out) {
    return celes_guard([&] { return celes_near_field_impl(h, npt, pts, add_incident, E_out); });
}


}  // extern "C"


// ===========================================================================
// batched solver: many problems and right-hand sides in one flat vector
// ===========================================================================
struct celes_batch {
    std::vector<celes_handle*> probs;
    celes_options opt;
    int L = 0, nmax = 0, half = 0, nprob = 0, nsys = 0, m = 0;
    int64_t total = 0;
    std::vector<int64_t> elem_off;   // [nprob+1]
    std::vector<int> sys0;           // [nprob+1]
    std::vector<int> sys_prob;       // [nsys]
    // mat-vec configuration (set by celes_batch_autotune or defaults)
    // (persistent blocks of 256 threads; the rotation scheme launches twice
    // as many blocks of 64)
    int chunk_len = 256, kb32 = 1, kb64 = 1, persist_blocks = 2048;
    // complex64 mat-vec of problems whose right-hand sides fill matrix-core blocks
    std::vector<int> mf_prob, mf_width, mf_nch;
    std::vector<celes::WxMfmaArgs> mf_args;
    DevBuf d_xb;
    // device buffers
    DevBuf d_elem_off, d_half_off, d_n, d_nrhs, d_nchunk, d_part_off, d_tq32, d_tq64;
    DevBuf d_args32, d_args64, d_item_off, d_nbx, d_nch, d_counter;
    DevBuf d_xsd, d_part;
    DevBuf d_bseg, d_blo, d_bhi, d_sblk;
    DevBuf d_rhs64, d_x64, d_r64, d_t64, d_V, d_d32, d_rhs32, d_t32, d_partial;
    DevBuf st_H, st_cs, st_sn, st_g, st_y, st_h1, st_h2, st_hn, st_bn, st_est, st_sc, st_act, st_en, st_used, st_it, d_k;
    celes::SegInfo si{};
    celes::GmresState st{};
    int nseg_blocks = 0;
    int64_t part_elems = 0;
    hipStream_t stream = nullptr;
    hipGraphExec_t graph32 = nullptr, graph64 = nullptr;
    void* graph_V = nullptr;          // basis the captured graphs point to
    std::vector<uint64_t> graph_pre;  // preconditioner generations the captured graphs use
    bool any_pre = false;             // some problem has a block-diagonal preconditioner
    DevBuf d_pz, d_pw;                // preconditioned Arnoldi step: gathered and preconditioned vectors
    std::string err;
    ~celes_batch() {
        if (graph32) hipGraphExecDestroy(graph32);
        if (graph64) hipGraphExecDestroy(graph64);
        if (stream) hipStreamDestroy(stream);
    }
};

namespace {

int bfail(celes_batch* b, int code, const std::string& msg) {
    if (b) b->err = msg;
    else g_create_error = msg;
    return code;
}

template <typename T>
bool upload(DevBuf& d, const std::vector<T>& v) {
    if (!d.ensure(std::max<size_t>(1, v.size()) * sizeof(T))) return false;
    return v.empty() || hipMemcpy(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
}

// (re)build the work items and WxArgs of both precisions for the current
// chunk length / right-hand-side blocks
int batch_configure(celes_batch* b) {
    const int G = celes::wx_num_groups(b->L);
    const bool rot = b->opt.translation == CELES_TRANSLATION_ROTATE;
    const int rblock = rot ? celes::WX_RTR_BLOCK_SIZE : celes::WX_BLOCK_SIZE;
    std::vector<int> nbx(b->nprob), nch(b->nprob), item32(b->nprob + 1, 0), item64(b->nprob + 1, 0);
    std::vector<int64_t> part_off(b->nprob);
    std::vector<celes::WxArgs<float>> a32(b->nprob);
    std::vector<celes::WxArgs<double>> a64(b->nprob);
    int64_t poff = 0;
    for (int p = 0; p < b->nprob; ++p) {
        celes_handle* h = b->probs[p];
        const int K = b->sys0[p + 1] - b->sys0[p];
        const int64_t N = h->N;
        nbx[p] = (int)((N + rblock - 1) / rblock);
        int64_t cl = std::max<int64_t>(celes::WX_TILE_SIZE, (int64_t)b->chunk_len);
        cl = (cl + celes::WX_TILE_SIZE - 1) / celes::WX_TILE_SIZE * celes::WX_TILE_SIZE;
        nch[p] = (int)((N + cl - 1) / cl);
        part_off[p] = poff;
        poff += (int64_t)nch[p] * K * b->nmax * N;
        const int mw = mfma_width(h, K);
        // per (receiver tile, chunk): pass groups x right-hand-side blocks
        // (direct) or the two polarisation passes x right-hand sides (rotation)
        const int z32 = rot ? 2 * K : G * (K / b->kb32), z64 = rot ? 2 * K : G * (K / b->kb64);
        item32[p + 1] = item32[p] + (mw > 0 ? 0 : nbx[p] * nch[p] * z32);
        item64[p + 1] = item64[p] + nbx[p] * nch[p] * z64;
        auto fill = [&](auto& a) {
            a.px = h->d_px.as<double>();
            a.py = h->d_py.as<double>();
            a.pz = h->d_pz.as<double>();
            a.lut.d_lo = h->lut_lo;
            a.lut.inv_dr = 1.0 / h->lut_dr;
            a.lut.inv_k = 1.0 / h->k;
            a.lut.n_int = (int)h->lut_n;
            a.k = h->k;
            a.n = (int)N;
            a.chunk_len = (int)cl;
            a.ldp = (int)N;
            a.nrhs = K;
            a.sys0 = b->sys0[p];
            a.active = b->st_act.as<int>();
        };
        fill(a32[p]);
        fill(a64[p]);
        a32[p].lut.coef = h->d_lut32.as<cx<float>>();
        a64[p].lut.coef = h->d_lut64.as<cx<double>>();
        a32[p].kb = b->kb32;
        a64[p].kb = b->kb64;
    }
    b->part_elems = poff;
    // scratch: xsd sized for FP64 (also serves FP32), partial sums likewise
    if (!b->d_xsd.ensure((size_t)b->total * sizeof(cx<double>)) ||
        !b->d_part.ensure((size_t)std::max<int64_t>(1, poff) * sizeof(cx<double>)))
        return bfail(b, CELES_E_OOM, "cannot allocate batch mat-vec scratch");
    // matrix-core problems: same source chunks as the VALU path (the finish
    // kernel reduces nch[p] partial sums), operand-ordered sources in d_xb
    b->mf_prob.clear();
    b->mf_width.clear();
    b->mf_nch.clear();
    b->mf_args.clear();
    size_t xb_floats = 0;
    std::vector<size_t> xb_off;
    for (int p = 0; p < b->nprob; ++p) {
        celes_handle* h = b->probs[p];
        const int K = b->sys0[p + 1] - b->sys0[p];
        const int mw = mfma_width(h, K);
        if (mw == 0) continue;
        b->mf_prob.push_back(p);
        b->mf_width.push_back(mw);
        b->mf_nch.push_back(nch[p]);
        xb_off.push_back(xb_floats);
        xb_floats += celes::wx_mfma_xb_floats(b->L, h->N, K);
    }
    if (!b->mf_prob.empty() && !b->d_xb.ensure(xb_floats * sizeof(float)))
        return bfail(b, CELES_E_OOM, "cannot allocate batch matrix-core scratch");
    for (size_t q = 0; q < b->mf_prob.size(); ++q) {
        const int p = b->mf_prob[q];
        celes_handle* h = b->probs[p];
        celes::WxMfmaArgs m{};
        m.px = h->d_px.as<double>();
        m.py = h->d_py.as<double>();
        m.pz = h->d_pz.as<double>();
        m.xb = b->d_xb.as<float>() + xb_off[q];
        m.part = (cx<float>*)b->d_part.p + part_off[p];
        m.rec = h->d_mrec.as<float>();
        m.lut.coef = h->d_lut32.as<cx<float>>();
        m.lut.d_lo = h->lut_lo;
        m.lut.inv_dr = 1.0 / h->lut_dr;
        m.lut.inv_k = 1.0 / h->k;
        m.lut.n_int = (int)h->lut_n;
        m.k = h->k;
        m.n = (int)h->N;
        m.chunk_len = a32[p].chunk_len;
        m.ldp = (int)h->N;
        m.nrhs = b->sys0[p + 1] - b->sys0[p];
        m.slot_stride = b->total;
        m.active = b->st_act.as<int>();
        m.sys0 = b->sys0[p];
        b->mf_args.push_back(m);
    }
    for (int p = 0; p < b->nprob; ++p) {
        a32[p].xsd = (const cx<float>*)b->d_xsd.p + b->elem_off[p];
        a64[p].xsd = (const cx<double>*)b->d_xsd.p + b->elem_off[p];
        a32[p].part = (cx<float>*)b->d_part.p + part_off[p];
        a64[p].part = (cx<double>*)b->d_part.p + part_off[p];
    }
    bool ok = upload(b->d_args32, a32) && upload(b->d_args64, a64) && upload(b->d_nbx, nbx) &&
              upload(b->d_nch, nch) && upload(b->d_part_off, part_off) && b->d_item_off.ensure(2 * (b->nprob + 1) * 4);
    if (!ok) return bfail(b, CELES_E_OOM, "batch upload failed");
    hipMemcpy(b->d_item_off.p, item32.data(), (b->nprob + 1) * 4, hipMemcpyHostToDevice);
    hipMemcpy((int*)b->d_item_off.p + (b->nprob + 1), item64.data(), (b->nprob + 1) * 4, hipMemcpyHostToDevice);
    return CELES_OK;
}

celes::BatchGeom batch_geom(const celes_batch* b, bool fp64) {
    celes::BatchGeom g;
    g.elem_off = b->d_elem_off.as<int64_t>();
    g.half_off = b->d_half_off.as<int64_t>();
    g.n = b->d_n.as<int>();
    g.nrhs = b->d_nrhs.as<int>();
    g.nchunk = b->d_nch.as<int>();
    g.part_off = b->d_part_off.as<int64_t>();
    g.tq = (const void* const*)(fp64 ? b->d_tq64.p : b->d_tq32.p);
    g.nprob = b->nprob;
    g.half = b->half;
    g.L = b->L;
    g.host_elems = b->total;
    return g;
}

// y = M x (epilogue) for every system; x = V + slot, y = Y + slot' (slots
// from *kstep when kstep is given)
template <typename T>
int batch_matvec(celes_batch* b, const cx<T>* V, const int* kstep, int kin, cx<T>* Y, int kout, int epilogue,
                 hipStream_t s) {
    const bool f64 = sizeof(T) == 8;
    celes::BatchGeom g = batch_geom(b, f64);
    // partial-sum offsets are element offsets of cx<double>; the FP32 kernel uses the same element offsets
    celes::bk_zero_int(b->d_counter.as<int>(), 1, s);
    celes::bk_prep<T>(g, V, b->total, kstep, kin, (cx<T>*)b->d_xsd.p, s);
    const int* item_off = (const int*)b->d_item_off.p + (f64 ? b->nprob + 1 : 0);
    const celes::WxArgs<T>* args = (const celes::WxArgs<T>*)(f64 ? b->d_args64.p : b->d_args32.p);
    const int hmode = b->opt.hankel == CELES_HANKEL_DIRECT ? 1 : 0;
    int rc = b->opt.translation == CELES_TRANSLATION_ROTATE
                 ? celes::wx_rtr_batch_run<T>(b->L, args, item_off, b->d_nbx.as<int>(), b->d_nch.as<int>(), b->nprob,
                                              b->d_counter.as<int>(), 2 * b->persist_blocks, hmode, s)
                 : celes::wx_batch_run<T>(b->L, args, item_off, b->d_nbx.as<int>(), b->d_nch.as<int>(), b->nprob,
                                          b->d_counter.as<int>(), b->persist_blocks, f64 ? b->kb64 : b->kb32, hmode,
                                          s);
    if (rc != 0) return bfail(b, CELES_E_DEVICE, "batch mat-vec launch failed");
    if constexpr (sizeof(T) == 4) {
        for (size_t q = 0; q < b->mf_prob.size(); ++q) {
            celes::WxMfmaArgs m = b->mf_args[q];
            m.x = (const cx<float>*)V + b->elem_off[b->mf_prob[q]];
            m.kstep = kstep;
            m.kin = kin;
            if (celes::wx_mfma_launch(m, b->L, b->mf_width[q], b->opt.hankel == CELES_HANKEL_DIRECT ? 1 : 0,
                                      b->mf_nch[q], s) != 0)
                return bfail(b, CELES_E_DEVICE, "batch matrix-core mat-vec launch failed");
        }
    }
    celes::bk_finish<T>(g, (const cx<T>*)b->d_part.p, V, b->total, kstep, kin, kout, Y, epilogue, s);
    return CELES_OK;
}

// out = P^{-1} in, system by system: a problem's block-diagonal
// preconditioner on each of its right-hand sides, the identity for problems
// without one (flat layout, in and out must not alias)
template <typename T>
int batch_precond_apply(celes_batch* b, const cx<T>* in, cx<T>* out, hipStream_t s, bool skip_inactive) {
    // one pass over a problem's inverses per group of eight of its systems;
    // inside an Arnoldi step groups of converged systems are skipped (their
    // slots are not read); the cycle-end update applies every system, since
    // one that converged during the cycle still needs its last correction
    for (int p = 0; p < b->nprob; ++p) {
        celes_handle* h = b->probs[p];
        const int64_t n = h->N * h->nmax, off = b->elem_off[p];
        if (h->pre) {
            if (h->pre->apply_multi<T>(in + off, out + off, h->K, n, skip_inactive ? b->st.active : nullptr,
                                       b->sys0[p], s) != 0)
                return bfail(b, CELES_E_DEVICE, "batch preconditioner apply failed");
        } else {
            celes::vec_scale<T>(in + off, 1.0, out + off, (int64_t)h->K * n, s);
        }
    }
    return CELES_OK;
}

template <typename T>
void record_arnoldi_step(celes_batch* b, cx<T>* V, double tol, hipStream_t s) {
    const int* k = b->d_k.as<int>();
    const int ld = b->m + 1;
    if (b->any_pre) {
        // right preconditioning: V_{k+1} = M P^{-1} V_k, through two flat
        // buffers because the apply takes plain pointers and the step index
        // lives on the device
        celes::bk_slot_copy<T>(V, k, 0, b->d_pz.as<cx<T>>(), nullptr, 0, b->total, s);
        batch_precond_apply<T>(b, b->d_pz.as<cx<T>>(), b->d_pw.as<cx<T>>(), s, true);
        celes::bk_slot_copy<T>(b->d_pw.as<cx<T>>(), nullptr, 0, V, k, 1, b->total, s);
        batch_matvec<T>(b, V, k, 1, V, 1, 1, s);                              // in place on slot k+1
    } else {
        batch_matvec<T>(b, V, k, 0, V, 1, 1, s);                              // V_{k+1} = M V_k
    }
    celes::bk_dots<T>(b->si, V, b->total, V, k, 1, 1, 0, b->st.active, b->d_partial.as<cx<double>>(), ld,
                      b->st.h1, ld, s);                                       // h1 = V^H V_{k+1}
    celes::bk_gemv<T>(b->si, V, b->total, b->st.h1, ld, k, 1, nullptr, b->st.active, V, 1, -1.0, s);
    celes::bk_dots<T>(b->si, V, b->total, V, k, 1, 1, 0, b->st.active, b->d_partial.as<cx<double>>(), ld,
                      b->st.h2, ld, s);                                       // second pass
    celes::bk_gemv<T>(b->si, V, b->total, b->st.h2, ld, k, 1, nullptr, b->st.active, V, 1, -1.0, s);
    celes::bk_dots<T>(b->si, V, b->total, V, k, 0, 1, 1, b->st.active, b->d_partial.as<cx<double>>(), ld,
                      b->st.hn, ld, s);                                       // ||V_{k+1}||^2
    celes::bk_givens(b->st, k, tol, s);
    celes::bk_scale<T>(b->si, V, b->total, k, 1, b->st.scale, s);
    celes::bk_incr(b->d_k.as<int>(), s);
}

// GMRES(m) cycles on M d = rhs (precision T) for the enabled systems, from
// d = 0, to relative tolerance tol (relative to each system's ||rhs||, taken
// from st.bnorm).  Returns the number of cycles.
template <typename T>
int batch_gmres(celes_batch* b, const cx<T>* rhs, cx<T>* d, cx<T>* tmp, double tol, int max_cycles, bool use_graph,
                int* rc_out) {
    hipStream_t s = b->stream;
    cx<T>* V = (cx<T>*)b->d_V.p;
    hipGraphExec_t& graph = sizeof(T) == 8 ? b->graph64 : b->graph32;
    const int nsys = b->nsys, m = b->m;
    *rc_out = CELES_OK;
    // the captured step holds the preconditioners' device pointers: re-capture
    // when any problem's preconditioner was rebuilt or removed
    std::vector<uint64_t> gens(b->nprob);
    bool any_pre = false;
    for (int p = 0; p < b->nprob; ++p) {
        gens[p] = b->probs[p]->pre ? b->probs[p]->pre_gen : 0;
        any_pre = any_pre || b->probs[p]->pre;
    }
    if (gens != b->graph_pre) {
        if (b->graph32) { hipGraphExecDestroy(b->graph32); b->graph32 = nullptr; }
        if (b->graph64) { hipGraphExecDestroy(b->graph64); b->graph64 = nullptr; }
        b->graph_pre = gens;
    }
    b->any_pre = any_pre;
    if (any_pre && (!b->d_pz.ensure((size_t)b->total * sizeof(cx<T>)) || !b->d_pw.ensure((size_t)b->total * sizeof(cx<T>)))) {
        *rc_out = bfail(b, CELES_E_OOM, "cannot allocate preconditioner buffers");
        return 0;
    }
    celes::bk_zero<T>(d, b->total, s);
    int cycle = 0;
    std::vector<int> act(nsys);
    for (; cycle < max_cycles; ++cycle) {
        // V_0 = rhs - M d  (d = 0 on the first cycle), beta = ||V_0||, V_0 /= beta
        if (cycle == 0) {
            celes::bk_copy_scaled<T>(b->si, rhs, V, nullptr, s);
        } else {
            // every system is inactive at the end of a cycle: re-enable the
            // participating ones so that the mat-vec computes their residuals
            celes::bk_copy_int(b->st.enabled, b->st.active, nsys, s);
            if ((*rc_out = batch_matvec<T>(b, d, nullptr, 0, tmp, 0, 1, s)) != CELES_OK) return cycle;
            celes::bk_sub<T>(rhs, tmp, V, b->total, s);
        }
        celes::bk_dots<T>(b->si, nullptr, b->total, V, nullptr, 0, 0, 1, nullptr, b->d_partial.as<cx<double>>(),
                          m + 1, b->st.hn, m + 1, s);
        celes::bk_cycle_start(b->st, tol, s);
        celes::bk_copy_scaled<T>(b->si, V, V, b->st.scale, s);
        celes::bk_zero_int(b->d_k.as<int>(), 1, s);
        for (int k = 0; k < m; ++k) {
            if (use_graph) {
                if (!graph) {
                    hipGraph_t gr;
                    hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
                    record_arnoldi_step<T>(b, V, tol, s);
                    hipStreamEndCapture(s, &gr);
                    if (hipGraphInstantiate(&graph, gr, nullptr, nullptr, 0) != hipSuccess) {
                        graph = nullptr;
                        use_graph = false;
                    }
                    hipGraphDestroy(gr);
                }
                if (graph) hipGraphLaunch(graph, s);
                else record_arnoldi_step<T>(b, V, tol, s);
            } else {
                record_arnoldi_step<T>(b, V, tol, s);
            }
            if ((k & 7) == 7 || k == m - 1) {
                hipMemcpyAsync(act.data(), b->st.active, nsys * sizeof(int), hipMemcpyDeviceToHost, s);
                hipStreamSynchronize(s);
                bool any = false;
                for (int v : act) any = any || v;
                if (!any) break;
            }
        }
        // d += V y over each system's used steps (d += P^{-1} V y when preconditioned)
        celes::bk_backsolve(b->st, s);
        if (any_pre) {
            celes::bk_zero<T>(b->d_pz.as<cx<T>>(), b->total, s);
            celes::bk_gemv<T>(b->si, V, b->total, b->st.y, m + 1, nullptr, 0, b->st.used, nullptr,
                              b->d_pz.as<cx<T>>(), 0, 1.0, s);
            if ((*rc_out = batch_precond_apply<T>(b, b->d_pz.as<cx<T>>(), b->d_pw.as<cx<T>>(), s, false)) != CELES_OK)
                return cycle;
            celes::bk_add<T>(d, b->d_pw.as<cx<T>>(), d, b->total, s);
        } else {
            celes::bk_gemv<T>(b->si, V, b->total, b->st.y, m + 1, nullptr, 0, b->st.used, nullptr, d, 0, 1.0, s);
        }
        std::vector<double> est(nsys);
        std::vector<int> en(nsys);
        hipMemcpyAsync(est.data(), b->st.est, nsys * 8, hipMemcpyDeviceToHost, s);
        hipMemcpyAsync(en.data(), b->st.enabled, nsys * 4, hipMemcpyDeviceToHost, s);
        hipStreamSynchronize(s);
        double worst = 0;
        for (int i = 0; i < nsys; ++i)
            if (en[i]) worst = std::max(worst, est[i]);
        if (b->opt.verbose) std::fprintf(stderr, "batch cycle %d: worst inner estimate %.3e\n", cycle, worst);
        if (!(worst > tol)) {
            ++cycle;
            break;
        }
    }
    return cycle;
}

}  // namespace

extern "C" {

static int celes_batch_create_impl(celes_batch** out, int nprob, celes_handle* const* probs, const celes_options* opt) {
    if (!out) return bfail(nullptr, CELES_E_ARG, "null batch pointer");
    *out = nullptr;
    if (nprob < 1 || !probs) return bfail(nullptr, CELES_E_ARG, "empty batch");
    std::unique_ptr<celes_batch> b(new celes_batch());
    if (opt) b->opt = *opt;
    else celes_default_options(&b->opt);
    b->nprob = nprob;
    b->probs.assign(probs, probs + nprob);
    b->L = probs[0]->L;
    if (b->L > 4) return bfail(nullptr, CELES_E_UNSUPPORTED, "batches are compiled for lmax <= 4");
    if (b->opt.solver != CELES_SOLVER_GMRES) return bfail(nullptr, CELES_E_UNSUPPORTED, "batches run GMRES only");
    if (b->opt.translation != CELES_TRANSLATION_DIRECT && b->opt.translation != CELES_TRANSLATION_ROTATE)
        return bfail(nullptr, CELES_E_ARG, "unknown translation scheme");
    b->nmax = probs[0]->nmax;
    b->half = probs[0]->half;
    b->m = std::max(1, b->opt.restart);
    b->elem_off.assign(nprob + 1, 0);
    b->sys0.assign(nprob + 1, 0);
    for (int p = 0; p < nprob; ++p) {
        celes_handle* h = probs[p];
        if (!h || h->L != b->L) return bfail(nullptr, CELES_E_ARG, "all problems of a batch need the same lmax");
        if (h->K < 1) return bfail(nullptr, CELES_E_STATE, "problem without incident field");
        b->elem_off[p + 1] = b->elem_off[p] + (int64_t)h->K * h->N * h->nmax;
        b->sys0[p + 1] = b->sys0[p] + h->K;
        for (int k = 0; k < h->K; ++k) b->sys_prob.push_back(p);
    }
    b->nsys = b->sys0[nprob];
    b->total = b->elem_off[nprob];
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
        return bfail(nullptr, CELES_E_DEVICE, "stream creation failed");
    // per-problem descriptors
    std::vector<int64_t> half_off(nprob + 1);
    std::vector<int> n(nprob), nrhs(nprob);
    std::vector<const void*> tq32(nprob), tq64(nprob);
    for (int p = 0; p <= nprob; ++p) half_off[p] = b->elem_off[p] / 2;
    for (int p = 0; p < nprob; ++p) {
        n[p] = (int)probs[p]->N;
        nrhs[p] = probs[p]->K;
        tq32[p] = probs[p]->d_tq32.p;
        tq64[p] = probs[p]->d_tq64.p;
    }
    // right-hand-side blocks that divide every problem's K
    auto kb_for = [&](int mx) {
        for (int kb = mx; kb > 1; kb /= 2) {
            bool ok = true;
            for (int p = 0; p < nprob; ++p) ok = ok && (nrhs[p] % kb == 0);
            if (ok) return kb;
        }
        return 1;
    };
    b->kb32 = kb_for(celes::wx_max_kb<float>(b->L));
    b->kb64 = kb_for(celes::wx_max_kb<double>(b->L));
    // segmented-reduction blocks: slices of at most 8192 elements per system
    const int64_t SLICE = 8192;
    std::vector<int> bseg, sblk(b->nsys + 1, 0);
    std::vector<int64_t> blo, bhi;
    int64_t maxblk = 0;
    for (int sy = 0; sy < b->nsys; ++sy) {
        const int p = b->sys_prob[sy];
        const int64_t len = probs[p]->N * b->nmax;
        const int64_t base = b->elem_off[p] + (int64_t)(sy - b->sys0[p]) * len;
        sblk[sy] = (int)bseg.size();
        for (int64_t o = 0; o < len; o += SLICE) {
            bseg.push_back(sy);
            blo.push_back(base + o);
            bhi.push_back(base + std::min(len, o + SLICE));
            maxblk = std::max(maxblk, std::min(len, o + SLICE) - o);
        }
    }
    sblk[b->nsys] = (int)bseg.size();
    const int nsys = b->nsys, m = b->m;
    const size_t tot = (size_t)b->total;
    bool ok = upload(b->d_elem_off, b->elem_off) && upload(b->d_half_off, half_off) && upload(b->d_n, n) &&
              upload(b->d_nrhs, nrhs) && upload(b->d_tq32, tq32) && upload(b->d_tq64, tq64) &&
              upload(b->d_bseg, bseg) && upload(b->d_blo, blo) && upload(b->d_bhi, bhi) && upload(b->d_sblk, sblk) &&
              b->d_counter.ensure(64) && b->d_k.ensure(64) &&
              b->d_rhs64.ensure(tot * 16) && b->d_x64.ensure(tot * 16) && b->d_r64.ensure(tot * 16) &&
              b->d_t64.ensure(tot * 16) &&
              b->d_partial.ensure((size_t)bseg.size() * (m + 1) * sizeof(cx<double>)) &&
              b->st_H.ensure((size_t)nsys * (m + 1) * m * 16) && b->st_cs.ensure((size_t)nsys * m * 16) &&
              b->st_sn.ensure((size_t)nsys * m * 16) && b->st_g.ensure((size_t)nsys * (m + 1) * 16) &&
              b->st_y.ensure((size_t)nsys * (m + 1) * 16) && b->st_h1.ensure((size_t)nsys * (m + 1) * 16) &&
              b->st_h2.ensure((size_t)nsys * (m + 1) * 16) && b->st_hn.ensure((size_t)nsys * (m + 1) * 16) &&
              b->st_bn.ensure(nsys * 8) && b->st_est.ensure(nsys * 8) && b->st_sc.ensure(nsys * 8) &&
              b->st_act.ensure(nsys * 4) && b->st_en.ensure(nsys * 4) && b->st_used.ensure(nsys * 4) &&
              b->st_it.ensure(nsys * 4);
    if (!ok) return bfail(nullptr, CELES_E_OOM, "batch allocation failed");
    b->si = {nsys, (int)bseg.size(), maxblk, b->d_bseg.as<int>(), b->d_blo.as<int64_t>(), b->d_bhi.as<int64_t>(),
             b->d_sblk.as<int>()};
    b->st = {nsys, m, b->st_H.as<cx<double>>(), b->st_cs.as<cx<double>>(), b->st_sn.as<cx<double>>(),
             b->st_g.as<cx<double>>(), b->st_y.as<cx<double>>(), b->st_h1.as<cx<double>>(),
             b->st_h2.as<cx<double>>(), b->st_hn.as<cx<double>>(), b->st_bn.as<double>(), b->st_est.as<double>(),
             b->st_sc.as<double>(), b->st_act.as<int>(), b->st_en.as<int>(), b->st_used.as<int>(),
             b->st_it.as<int>()};
    std::vector<int> ones(nsys, 1);
    upload(b->st_act, ones);
    int rc = batch_configure(b.get());
    if (rc != CELES_OK) {
        g_create_error = b->err;
        return rc;
    }
    *out = b.release();
    return CELES_OK;
}
int celes_batch_create(celes_batch** out, int nprob, celes_handle* const* probs, const celes_options* opt) {
    return celes_guard([&] { return celes_batch_create_impl(out, nprob, probs, opt); });
}


void celes_batch_destroy(celes_batch* b) { delete b; }

int celes_batch_num_systems(const celes_batch* b) { return b ? b->nsys : 0; }

const char* celes_batch_last_error(const celes_batch* b) { return b ? b->err.c_str() : g_create_error.c_str(); }

static int celes_batch_apply_M_impl(celes_batch* b, int precision, const void* x_dev, void* y_dev, void* stream) {
    if (!b || !x_dev || !y_dev) return bfail(b, CELES_E_ARG, "null argument");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int> ones(b->nsys, 1);
    upload(b->st_act, ones);
    if (precision == CELES_FP64) return batch_matvec<double>(b, (const cx<double>*)x_dev, nullptr, 0, (cx<double>*)y_dev, 0, 1, s);
    if (precision == CELES_MIXED) return batch_matvec<float>(b, (const cx<float>*)x_dev, nullptr, 0, (cx<float>*)y_dev, 0, 1, s);
    return bfail(b, CELES_E_ARG, "unknown precision");
}
int celes_batch_apply_M(celes_batch* b, int precision, const void* x_dev, void* y_dev, void* stream) {
    return celes_guard([&] { return celes_batch_apply_M_impl(b, precision, x_dev, y_dev, stream); });
}


static int celes_batch_autotune_impl(celes_batch* b, int precision, double* best_ms, int* best_chunk, int* best_kb) {
    if (!b) return CELES_E_ARG;
    if (b->opt.deterministic) return bfail(b, CELES_E_STATE, "the batch was created deterministic: no timing-based split");
    const bool f64 = precision == CELES_FP64;
    const int mxkb = f64 ? celes::wx_max_kb<double>(b->L) : celes::wx_max_kb<float>(b->L);
    hipStream_t s = b->stream;
    std::vector<int> ones(b->nsys, 1);
    upload(b->st_act, ones);
    double best = 1e300;
    int bc = b->chunk_len, bk = f64 ? b->kb64 : b->kb32;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    const int chunks[] = {128, 256, 512, 1024};
    // the rotation scheme takes one right-hand side per work item
    const int kb_max = b->opt.translation == CELES_TRANSLATION_ROTATE ? 1 : mxkb;
    for (int kb = 1; kb <= kb_max; kb *= 2) {
        bool divides = true;
        for (int p = 0; p < b->nprob; ++p) divides = divides && ((b->sys0[p + 1] - b->sys0[p]) % kb == 0);
        if (!divides) continue;
        for (int cl : chunks) {
            b->chunk_len = cl;
            if (f64) b->kb64 = kb;
            else b->kb32 = kb;
            if (batch_configure(b) != CELES_OK) continue;
            auto run = [&]() {
                if (f64) batch_matvec<double>(b, b->d_x64.as<cx<double>>(), nullptr, 0, b->d_t64.as<cx<double>>(), 0, 1, s);
                else batch_matvec<float>(b, (cx<float>*)b->d_x64.p, nullptr, 0, (cx<float>*)b->d_t64.p, 0, 1, s);
            };
            run();
            hipEventRecord(e0, s);
            run();
            run();
            hipEventRecord(e1, s);
            hipEventSynchronize(e1);
            float ms = 0;
            hipEventElapsedTime(&ms, e0, e1);
            ms *= 0.5f;
            if (ms < best) {
                best = ms;
                bc = cl;
                bk = kb;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    b->chunk_len = bc;
    if (f64) b->kb64 = bk;
    else b->kb32 = bk;
    if (b->graph32) { hipGraphExecDestroy(b->graph32); b->graph32 = nullptr; }
    if (b->graph64) { hipGraphExecDestroy(b->graph64); b->graph64 = nullptr; }
    int rc = batch_configure(b);
    if (best_ms) *best_ms = best;
    if (best_chunk) *best_chunk = bc;
    if (best_kb) *best_kb = bk;
    return rc;
}
int celes_batch_autotune(celes_batch* b, int precision, double* best_ms, int* best_chunk, int* best_kb) {
    return celes_guard([&] { return celes_batch_autotune_impl(b, precision, best_ms, best_chunk, best_kb); });
}


static int celes_batch_solve_impl(celes_batch* b, celes_solve_info* infos, celes_solve_info* summary) {
    if (!b) return CELES_E_ARG;
    hipStream_t s = b->stream;
    const int nsys = b->nsys;
    const int64_t tot = b->total;
    auto t0 = std::chrono::steady_clock::now();
    // rhs = T a_in and x0 = 0, system by system in the flat layout
    std::vector<cx<double>> rhs(tot);
    std::vector<double> bn(nsys, 0.0);
    for (int p = 0; p < b->nprob; ++p) {
        celes_handle* h = b->probs[p];
        const int64_t n = h->N * h->nmax;
        for (int k = 0; k < h->K; ++k) {
            double acc = 0;
            for (int64_t i = 0; i < h->N; ++i)
                for (int tau = 0; tau < 2; ++tau)
                    for (int c = 0; c < h->half; ++c) {
                        int l = (int)std::floor(std::sqrt((double)(c + 1)));
                        while (l * (l + 2) < c + 1) ++l;
                        while ((l - 1) * (l + 1) >= c + 1) --l;
                        const cplx q = h->tq[((size_t)i * 2 + tau) * h->L + (l - 1)];
                        const cplx v = q * h->a_in[((size_t)k * h->N + i) * h->nmax + tau * h->half + c];
                        rhs[b->elem_off[p] + k * n + i * h->nmax + tau * h->half + c] = {v.real(), v.imag()};
                        acc += std::norm(v);
                    }
            bn[b->sys0[p] + k] = std::sqrt(acc);
        }
    }
    if (hipMemcpy(b->d_rhs64.p, rhs.data(), tot * 16, hipMemcpyHostToDevice) != hipSuccess)
        return bfail(b, CELES_E_DEVICE, "copy failed");
    const bool mixed = b->opt.precision == CELES_MIXED;
    const size_t vbytes = (size_t)(b->m + 1) * tot * (mixed ? 8 : 16);
    if (!b->d_V.ensure(vbytes) || !b->d_d32.ensure(tot * 16) || !b->d_rhs32.ensure(tot * 16) ||
        !b->d_t32.ensure(tot * 16))
        return bfail(b, CELES_E_OOM, "cannot allocate the Krylov basis");
    if (b->graph_V != b->d_V.p) {
        if (b->graph32) { hipGraphExecDestroy(b->graph32); b->graph32 = nullptr; }
        if (b->graph64) { hipGraphExecDestroy(b->graph64); b->graph64 = nullptr; }
        b->graph_V = b->d_V.p;
    }
    celes::bk_zero<double>(b->d_x64.as<cx<double>>(), tot, s);
    celes::bk_zero_int(b->st.iters, nsys, s);
    std::vector<int> iters_total(nsys, 0);
    std::vector<double> res(nsys, 1.0);
    int refinements = 0, status = CELES_OK, matvecs = 0;
    const double tol = b->opt.tol;
    const bool use_graph = std::getenv("CELES_NO_GRAPH") == nullptr;
    for (int it = 0; it <= b->opt.max_refinements; ++it) {
        // FP64 residual r = rhs - M x, per-system norms
        std::vector<int> ones(nsys, 1);
        upload(b->st_act, ones);
        int rc = batch_matvec<double>(b, b->d_x64.as<cx<double>>(), nullptr, 0, b->d_t64.as<cx<double>>(), 0, 1, s);
        if (rc != CELES_OK) return rc;
        ++matvecs;
        celes::bk_sub<double>(b->d_rhs64.as<cx<double>>(), b->d_t64.as<cx<double>>(), b->d_r64.as<cx<double>>(), tot, s);
        celes::bk_dots<double>(b->si, nullptr, tot, b->d_r64.as<cx<double>>(), nullptr, 0, 0, 1, nullptr,
                               b->d_partial.as<cx<double>>(), b->m + 1, b->st.hn, b->m + 1, s);
        std::vector<cx<double>> hn((size_t)nsys * (b->m + 1));
        hipMemcpyAsync(hn.data(), b->st.hn, hn.size() * 16, hipMemcpyDeviceToHost, s);
        hipStreamSynchronize(s);
        std::vector<int> en(nsys);
        std::vector<double> rn(nsys);
        bool any = false;
        double worst = 0;
        for (int sy = 0; sy < nsys; ++sy) {
            rn[sy] = std::sqrt(std::max(0.0, hn[(size_t)sy * (b->m + 1)].re));
            res[sy] = bn[sy] > 0 ? rn[sy] / bn[sy] : 0.0;
            en[sy] = res[sy] > tol ? 1 : 0;
            any = any || en[sy];
            worst = std::max(worst, res[sy]);
        }
        if (!any || it == b->opt.max_refinements) break;
        upload(b->st_en, en);
        upload(b->st_bn, rn);
        // inner solve on M d = r, relative tolerance against ||r||
        double inner = mixed ? std::max(b->opt.inner_tol, 0.5 * tol / worst) : 0.5 * tol / worst;
        int cycles_left = std::max(1, b->opt.maxiter / b->m);
        int cyc;
        if (mixed) {
            celes::bk_to32(b->d_r64.as<cx<double>>(), b->d_rhs32.as<cx<float>>(), tot, s);
            cyc = batch_gmres<float>(b, b->d_rhs32.as<cx<float>>(), b->d_d32.as<cx<float>>(),
                                     b->d_t32.as<cx<float>>(), inner, cycles_left, use_graph, &rc);
            if (rc != CELES_OK) return rc;
            celes::bk_acc32(b->d_d32.as<cx<float>>(), b->d_x64.as<cx<double>>(), tot, s);
        } else {
            cyc = batch_gmres<double>(b, b->d_r64.as<cx<double>>(), b->d_d32.as<cx<double>>(),
                                      b->d_t32.as<cx<double>>(), inner, cycles_left, use_graph, &rc);
            if (rc != CELES_OK) return rc;
            celes::bk_add<double>(b->d_x64.as<cx<double>>(), b->d_d32.as<cx<double>>(), b->d_x64.as<cx<double>>(), tot, s);
        }
        (void)cyc;
        ++refinements;
        if (b->opt.verbose) std::fprintf(stderr, "batch refinement %d: worst residual %.3e\n", it, worst);
    }
    hipStreamSynchronize(s);
    std::vector<int> its(nsys);
    hipMemcpy(its.data(), b->st.iters, nsys * 4, hipMemcpyDeviceToHost);
    // solutions back into the handles
    std::vector<cx<double>> x(tot);
    hipMemcpy(x.data(), b->d_x64.p, tot * 16, hipMemcpyDeviceToHost);
    double worst = 0;
    for (int p = 0; p < b->nprob; ++p) {
        celes_handle* h = b->probs[p];
        const int64_t n = (int64_t)h->K * h->N * h->nmax;
        h->b.resize(n);
        for (int64_t i = 0; i < n; ++i) h->b[i] = cplx(x[b->elem_off[p] + i].re, x[b->elem_off[p] + i].im);
        h->have_solution = true;
    }
    auto t1 = std::chrono::steady_clock::now();
    int total_its = 0;
    for (int sy = 0; sy < nsys; ++sy) {
        worst = std::max(worst, res[sy]);
        total_its += its[sy];
        if (!std::isfinite(res[sy])) status = CELES_E_BREAKDOWN;
        else if (res[sy] > tol && status == CELES_OK) status = CELES_E_NOCONV;
        if (infos) {
            infos[sy] = celes_solve_info{};
            infos[sy].status = std::isfinite(res[sy]) ? (res[sy] <= tol ? CELES_OK : CELES_E_NOCONV) : CELES_E_BREAKDOWN;
            infos[sy].iterations = its[sy];
            infos[sy].refinements = refinements;
            infos[sy].rel_residual = res[sy];
            infos[sy].x0_residual = 1.0;        // batches start from zero
        }
    }
    if (summary) {
        *summary = celes_solve_info{};
        summary->status = status;
        summary->iterations = total_its;
        summary->refinements = refinements;
        summary->matvecs = matvecs;
        summary->rel_residual = worst;
        summary->x0_residual = 1.0;
        summary->seconds = std::chrono::duration<double>(t1 - t0).count();
    }
    if (status == CELES_E_NOCONV) b->err = "batched solve did not reach the tolerance";
    return status;
}
int celes_batch_solve(celes_batch* b, celes_solve_info* infos, celes_solve_info* summary) {
    return celes_guard([&] { return celes_batch_solve_impl(b, infos, summary); });
}


int celes_kernel_timing(celes_handle* h, int enable, double* avg_ms, int* count) {
    if (!h) return CELES_E_ARG;
    if (enable) {
        h->time_kernels = true;
        h->tev_used = 0;
        return CELES_OK;
    }
    double sum = 0;
    const int n = (int)(h->tev_used / 2);
    for (int q = 0; q < n; ++q) {
        float ms = 0;
        if (hipEventSynchronize(h->tev[2 * q + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms, h->tev[2 * q], h->tev[2 * q + 1]) != hipSuccess)
            return fail(h, CELES_E_DEVICE, "kernel timing events failed");
        sum += ms;
    }
    h->time_kernels = false;
    h->tev_used = 0;
    if (avg_ms) *avg_ms = n ? sum / n : 0.0;
    if (count) *count = n;
    return CELES_OK;
}

static int celes_get_solution_impl(const celes_handle* h, double* b_out) {
    if (!h || !b_out) return CELES_E_ARG;
    if (!h->have_solution) return CELES_E_STATE;
    std::memcpy(b_out, h->b.data(), h->b.size() * sizeof(cplx));
    return CELES_OK;
}
int celes_get_solution(const celes_handle* h, double* b_out) {
    return celes_guard([&] { return celes_get_solution_impl(h, b_out); });
}


}  // extern "C"

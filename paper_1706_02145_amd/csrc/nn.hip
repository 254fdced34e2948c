// Learned initial guess for the iterative solve (the paper's custom initial
// condition hook, Section 4.2, filled by a small network).
//
// For every sphere i the network sees its own radius and incident
// coefficients and those of its 16 nearest neighbours (relative positions),
// all expressed in sphere i's incident-phase frame and scaled by
// ||a_in^i||, and predicts sphere i's scattered coefficients in the same
// frame.  Architecture: in_pad -> 128 -> 128 -> 128 -> out_pad, SiLU between
// layers, bf16 weights and activations, FP32 accumulation (MFMA
// 16x16x16 bf16), FP32 master weights updated by Adam.  Bf16 rounding
// points: inputs, weights, hidden activations, and the layer gradients dZ
// that enter the backward products; everything else is FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/celes.h"
#include "device_common.hpp"
#include "internal.hpp"

namespace {

using celes::cmul;
using celes::cmulc;
using celes::cx;

constexpr int NN_K = 16;       // neighbours
constexpr int NN_H = 128;      // hidden width
constexpr int NN_LAYERS = 4;   // linear layers (3 hidden)
constexpr int TM = 64, TN = 64, TK = 16;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline unsigned short f2bf(float f) {
    // round to nearest even
    unsigned int u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);  // NaN
    const unsigned int lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (unsigned short)(u >> 16);
}
__host__ __device__ inline float bf2f(unsigned short h) {
    unsigned int u = (unsigned int)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

int round_up(int a, int b) { return (a + b - 1) / b * b; }

// ---------------------------------------------------------------------------
// C[m][n] (+)= sum_k A(m,k) B(k,n); A(m,k) = A[m*sam + k*sak], B(k,n) =
// B[k*sbk + n*sbn] (bf16); C row-major fp32 (ldc).  M, N multiples of 64,
// K multiple of 16.  256 threads: 4 waves, each a 32x32 sub-tile of 2x2
// MFMA 16x16x16 tiles.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) gemm_bf16(const unsigned short* __restrict__ A, int64_t sam, int64_t sak,
                                                 const unsigned short* __restrict__ B, int64_t sbk, int64_t sbn,
                                                 float* __restrict__ C, int64_t ldc, int K, int accumulate) {
    __shared__ unsigned short As[TM][TK + 4];
    __shared__ unsigned short Bs[TK][TN + 4];
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int wm = (wave / 2) * 32, wn = (wave % 2) * 32;
    f32x4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += TK) {
        __syncthreads();
        for (int e = threadIdx.x; e < TM * TK; e += 256) {
            const int r = e / TK, c = e % TK;
            As[r][c] = A[(int64_t)(m0 + r) * sam + (int64_t)(k0 + c) * sak];
        }
        for (int e = threadIdx.x; e < TK * TN; e += 256) {
            const int r = e / TN, c = e % TN;
            Bs[r][c] = B[(int64_t)(k0 + r) * sbk + (int64_t)(n0 + c) * sbn];
        }
        __syncthreads();
        const int kq = 4 * (lane / 16), rc = lane % 16;
        bf16x4 av[2], bv[2];
        for (int a = 0; a < 2; ++a)
            for (int t = 0; t < 4; ++t) av[a][t] = (short)As[wm + 16 * a + rc][kq + t];
        for (int b = 0; b < 2; ++b)
            for (int t = 0; t < 4; ++t) bv[b][t] = (short)Bs[kq + t][wn + 16 * b + rc];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    const int rq = 4 * (lane / 16), cc = lane % 16;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int t = 0; t < 4; ++t) {
                float* dst = C + (int64_t)(m0 + wm + 16 * a + rq + t) * ldc + (n0 + wn + 16 * b + cc);
                *dst = accumulate ? *dst + acc[a][b][t] : acc[a][b][t];
            }
}

__device__ inline float silu(float z) { return z / (1.f + __expf(-z)); }
__device__ inline float dsilu(float z) {
    const float s = 1.f / (1.f + __expf(-z));
    return s * (1.f + z * (1.f - s));
}

// Z = C + b; A = bf16(silu(Z)) for hidden layers (act = 1) or A unused
__global__ void bias_act(float* __restrict__ Z, const float* __restrict__ b, unsigned short* __restrict__ Aout,
                         int64_t M, int N, int act) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= M * N) return;
    const int n = (int)(t % N);
    const float z = Z[t] + b[n];
    Z[t] = z;
    if (act) Aout[t] = f2bf(silu(z));
}

// MSE loss on valid rows (< Mvalid) and columns (< Nvalid); dZ = 2 (Z - Y) / (Mvalid Nvalid)
__global__ void mse_grad(const float* __restrict__ Z, const float* __restrict__ Y, float* __restrict__ dZ,
                         unsigned short* __restrict__ dZb, double* __restrict__ partial, int64_t M, int N,
                         int64_t Mvalid, int Nvalid) {
    __shared__ double red[256];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double l = 0;
    if (t < M * N) {
        const int64_t m = t / N;
        const int n = (int)(t % N);
        float g = 0.f;
        if (m < Mvalid && n < Nvalid) {
            const float d = Z[t] - Y[m * N + n];
            l = (double)d * d;
            g = 2.f * d / (float)((double)Mvalid * Nvalid);
        }
        dZ[t] = g;
        dZb[t] = f2bf(g);
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// dZ = dA * silu'(Z) (dA fp32 from the previous backward product), bf16 copy
__global__ void act_back(const float* __restrict__ dA, const float* __restrict__ Z, float* __restrict__ dZ,
                         unsigned short* __restrict__ dZb, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    const float g = dA[t] * dsilu(Z[t]);
    dZ[t] = g;
    dZb[t] = f2bf(g);
}

// db[n] = sum_m dZ[m][n] (one block per column, fixed order)
__global__ void col_sum(const float* __restrict__ dZ, float* __restrict__ db, int64_t M, int N) {
    __shared__ float red[256];
    const int n = blockIdx.x;
    float s = 0.f;
    for (int64_t m = threadIdx.x; m < M; m += 256) s += dZ[m * N + n];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[n] = red[0];
}

__global__ void to_bf16(const float* __restrict__ x, unsigned short* __restrict__ y, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n) y[t] = f2bf(x[t]);
}

__global__ void adam_step(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, unsigned short* __restrict__ wb, int64_t n, float lr, float b1,
                          float b2, float eps, float c1, float c2) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    const float wt = w[t] - lr * (mt / c1) / (sqrtf(vt / c2) + eps);
    w[t] = wt;
    wb[t] = f2bf(wt);
}

// ---------------------------------------------------------------------------
// neighbours and features
// ---------------------------------------------------------------------------
// 16 nearest neighbours of every sphere (brute force over LDS tiles of the
// centres, sorted by distance, ties by index)
__global__ void __launch_bounds__(256) knn16(const double* __restrict__ px, const double* __restrict__ py,
                                             const double* __restrict__ pz, int n, int* __restrict__ nbr) {
    __shared__ double tx[256], ty[256], tz[256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool act = i < n;
    const double xi = act ? px[i] : 0, yi = act ? py[i] : 0, zi = act ? pz[i] : 0;
    double bd[NN_K];
    int bi[NN_K];
    for (int q = 0; q < NN_K; ++q) {
        bd[q] = 1e300;
        bi[q] = -1;
    }
    for (int t0 = 0; t0 < n; t0 += 256) {
        __syncthreads();
        if (t0 + threadIdx.x < n) {
            tx[threadIdx.x] = px[t0 + threadIdx.x];
            ty[threadIdx.x] = py[t0 + threadIdx.x];
            tz[threadIdx.x] = pz[t0 + threadIdx.x];
        }
        __syncthreads();
        const int nt = min(256, n - t0);
        for (int jj = 0; jj < nt; ++jj) {
            const int j = t0 + jj;
            if (j == i) continue;
            const double dx = tx[jj] - xi, dy = ty[jj] - yi, dz = tz[jj] - zi;
            double d = dx * dx + dy * dy + dz * dz;
            if (d >= bd[NN_K - 1]) continue;
            int jd = j;
#pragma unroll
            for (int q = 0; q < NN_K; ++q) {
                if (d < bd[q]) {
                    const double td = bd[q];
                    const int ti = bi[q];
                    bd[q] = d;
                    bi[q] = jd;
                    d = td;
                    jd = ti;
                }
            }
        }
    }
    if (act)
        for (int q = 0; q < NN_K; ++q) nbr[(int64_t)i * NN_K + q] = bi[q];
}

struct FeatArgs {
    const double* px;
    const double* py;
    const double* pz;
    const double* rad;
    const cx<double>* ain;    // [N][nmax] first right-hand side
    const cx<double>* b;      // [N][nmax] solution (targets) or null
    const int* nbr;           // [N][16]
    int n, nmax, nref, in_dim, in_pad, out_pad;
    double inv_lambda;
    unsigned short* X;        // [rows][in_pad] bf16
    float* Y;                 // [rows][out_pad] fp32 (targets) or null
    cx<double>* frame;        // [N] c_i * ||a_in^i|| (to map predictions back)
};

// one thread per (sphere, feature column)
__global__ void build_features(FeatArgs f) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)f.n * f.in_pad) return;
    const int i = (int)(t / f.in_pad), col = (int)(t % f.in_pad);
    const cx<double>* ai = f.ain + (int64_t)i * f.nmax;
    double nrm = 0;
    for (int c = 0; c < f.nmax; ++c) nrm += ai[c].re * ai[c].re + ai[c].im * ai[c].im;
    nrm = sqrt(nrm);
    cx<double> ref = ai[f.nref];
    const double ra = sqrt(ref.re * ref.re + ref.im * ref.im);
    ref = ra > 0 ? cx<double>{ref.re / ra, ref.im / ra} : cx<double>{1.0, 0.0};
    const double s = nrm > 0 ? 1.0 / nrm : 0.0;
    // value of a_in^j in sphere i's frame, component c (re / im by parity)
    auto framed = [&](const cx<double>* a, int c, int part) {
        const cx<double> v = cmulc(a[c], ref);   // a * conj(ref)
        return (part == 0 ? v.re : v.im) * s;
    };
    double val = 0;
    const int self = 1 + 2 * f.nmax, per = 4 + 2 * f.nmax;
    if (col == 0) {
        val = f.rad[i] * f.inv_lambda;
    } else if (col < self) {
        const int c = (col - 1) / 2;
        val = framed(ai, c, (col - 1) % 2);
    } else if (col < f.in_dim) {
        const int q = (col - self) / per, r = (col - self) % per;
        const int j = f.nbr[(int64_t)i * NN_K + q];
        if (j >= 0) {
            if (r == 0) val = (f.px[j] - f.px[i]) * f.inv_lambda;
            else if (r == 1) val = (f.py[j] - f.py[i]) * f.inv_lambda;
            else if (r == 2) val = (f.pz[j] - f.pz[i]) * f.inv_lambda;
            else if (r == 3) val = f.rad[j] * f.inv_lambda;
            else {
                const int c = (r - 4) / 2;
                val = framed(f.ain + (int64_t)j * f.nmax, c, (r - 4) % 2);
            }
        }
    }
    f.X[t] = f2bf((float)val);
    if (col < f.out_pad && f.Y) {
        double y = 0;
        if (col < 2 * f.nmax && f.b) y = framed(f.b + (int64_t)i * f.nmax, col / 2, col % 2);
        f.Y[(int64_t)i * f.out_pad + col] = (float)y;
    }
    if (col == 0) f.frame[i] = {ref.re * nrm, ref.im * nrm};
}

__global__ void unframe(const float* __restrict__ Z, int out_pad, const cx<double>* __restrict__ frame, int n,
                        int nmax, cx<double>* __restrict__ x0) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)n * nmax) return;
    const int i = (int)(t / nmax), c = (int)(t % nmax);
    const cx<double> y = {(double)Z[(int64_t)i * out_pad + 2 * c], (double)Z[(int64_t)i * out_pad + 2 * c + 1]};
    x0[t] = cmul(y, frame[i]);
}

// dst row r = src row idx[r] (zero when idx[r] < 0), bf16 features and fp32 targets
__global__ void gather_rows(const unsigned short* __restrict__ X, const float* __restrict__ Y,
                            const int64_t* __restrict__ idx, int64_t rows, int in_pad, int out_pad,
                            unsigned short* __restrict__ bx, float* __restrict__ by) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t w = in_pad + out_pad;
    if (t >= rows * w) return;
    const int64_t r = t / w;
    const int c = (int)(t % w);
    const int64_t src = idx[r];
    if (c < in_pad) bx[r * in_pad + c] = src >= 0 ? X[src * in_pad + c] : (unsigned short)0;
    else by[r * out_pad + (c - in_pad)] = src >= 0 ? Y[src * out_pad + (c - in_pad)] : 0.f;
}

inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

// SplitMix64 (Steele, Lea, Flood 2014): counter-based 64-bit generator
uint64_t splitmix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ULL;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
    return x ^ (x >> 31);
}

}  // namespace

struct celes_nn {
    int L = 0, nmax = 0, in_dim = 0, in_pad = 0, out_dim = 0, out_pad = 0;
    int dims[NN_LAYERS + 1];
    std::vector<int64_t> woff, boff;   // offsets in the flat parameter vector
    int64_t nparam = 0;
    celes::DevBuf w32, wbf, grad, am, av;   // master weights, bf16 copy, gradient, Adam moments
    // training set
    std::vector<unsigned short> hX;
    std::vector<float> hY;
    int64_t rows = 0;
    celes::DevBuf dX, dY;
    // work space for a batch of M rows
    celes::DevBuf Z[NN_LAYERS], Ab[NN_LAYERS], dZ, dZb, dA, partial;
    int64_t work_rows = 0;
    int64_t adam_t = 0;
    std::string err;
};

namespace {

int nn_fail(celes_nn* n, int code, const std::string& m) {
    if (n) n->err = m;
    return code;
}

bool nn_work(celes_nn* n, int64_t M) {
    if (M <= n->work_rows) return true;
    for (int l = 0; l < NN_LAYERS; ++l)
        if (!n->Z[l].ensure(M * n->dims[l + 1] * 4) || !n->Ab[l].ensure(M * n->dims[l + 1] * 2)) return false;
    const int mx = std::max(n->in_pad, NN_H) > n->out_pad ? std::max(n->in_pad, NN_H) : n->out_pad;
    if (!n->dZ.ensure(M * mx * 4) || !n->dZb.ensure(M * mx * 2) || !n->dA.ensure(M * mx * 4) ||
        !n->partial.ensure((M * mx / 256 + 2) * 8))
        return false;
    n->work_rows = M;
    return true;
}

// forward on X [M][in_pad] (bf16, device); output Z[3] [M][out_pad] fp32
void nn_forward(celes_nn* n, const unsigned short* X, int64_t M, hipStream_t s) {
    const unsigned short* Wb = n->wbf.as<unsigned short>();
    const float* W = n->w32.as<float>();
    const unsigned short* in = X;
    for (int l = 0; l < NN_LAYERS; ++l) {
        const int K = n->dims[l], N = n->dims[l + 1];
        dim3 grid(N / TN, (unsigned)(M / TM));
        hipLaunchKernelGGL(gemm_bf16, grid, dim3(256), 0, s, in, (int64_t)K, (int64_t)1, Wb + n->woff[l], (int64_t)N,
                           (int64_t)1, n->Z[l].as<float>(), (int64_t)N, K, 0);
        hipLaunchKernelGGL(bias_act, dim3(nb(M * N)), dim3(256), 0, s, n->Z[l].as<float>(), W + n->boff[l],
                           n->Ab[l].as<unsigned short>(), M, N, l < NN_LAYERS - 1 ? 1 : 0);
        in = n->Ab[l].as<unsigned short>();
    }
}

// loss and gradient (into n->grad) of a batch X [M][in_pad], Y [M][out_pad]
// with Mvalid real rows; returns the loss
double nn_backward(celes_nn* n, const unsigned short* X, const float* Y, int64_t M, int64_t Mvalid, hipStream_t s) {
    nn_forward(n, X, M, s);
    const int last = NN_LAYERS - 1;
    const int64_t nblk = nb(M * n->out_pad);
    hipLaunchKernelGGL(mse_grad, dim3((unsigned)nblk), dim3(256), 0, s, n->Z[last].as<float>(), Y, n->dZ.as<float>(),
                       n->dZb.as<unsigned short>(), n->partial.as<double>(), M, n->out_pad, Mvalid, n->out_dim);
    float* G = n->grad.as<float>();
    const unsigned short* Wb = n->wbf.as<unsigned short>();
    for (int l = last; l >= 0; --l) {
        const int K = n->dims[l], N = n->dims[l + 1];
        const unsigned short* in = l > 0 ? n->Ab[l - 1].as<unsigned short>() : X;
        // dW_l = in^T dZ_l  (K x N) ; db_l = colsum dZ_l
        dim3 gw(N / TN, K / TM);
        hipLaunchKernelGGL(gemm_bf16, gw, dim3(256), 0, s, in, (int64_t)1, (int64_t)K, n->dZb.as<unsigned short>(),
                           (int64_t)N, (int64_t)1, G + n->woff[l], (int64_t)N, (int)M, 0);
        hipLaunchKernelGGL(col_sum, dim3(N), dim3(256), 0, s, n->dZ.as<float>(), G + n->boff[l], M, N);
        if (l > 0) {
            // dA_{l-1} = dZ_l W_l^T (M x K), then dZ_{l-1} = dA * silu'(Z_{l-1})
            dim3 ga(K / TN, (unsigned)(M / TM));
            hipLaunchKernelGGL(gemm_bf16, ga, dim3(256), 0, s, n->dZb.as<unsigned short>(), (int64_t)N, (int64_t)1,
                               Wb + n->woff[l], (int64_t)1, (int64_t)N, n->dA.as<float>(), (int64_t)K, N, 0);
            hipLaunchKernelGGL(act_back, dim3(nb(M * K)), dim3(256), 0, s, n->dA.as<float>(),
                               n->Z[l - 1].as<float>(), n->dZ.as<float>(), n->dZb.as<unsigned short>(), M * K);
        }
    }
    std::vector<double> part(nblk);
    hipMemcpyAsync(part.data(), n->partial.p, nblk * 8, hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    double loss = 0;
    for (double v : part) loss += v;
    return loss / ((double)Mvalid * n->out_dim);
}

// (T a_in)[e] of the first right-hand side: Mie coefficient Q_{tau l} of the
// sphere times the incident coefficient, entry e = i nmax + tau half + c
static celes::cplx single_scattering(const celes_handle* h, int64_t e) {
    const int64_t i = e / h->nmax;
    const int r = (int)(e % h->nmax), tau = r / h->half, c = r % h->half;
    int l = 1;
    while (l * (l + 2) < c + 1) ++l;
    return h->tq[((size_t)i * 2 + tau) * h->L + (l - 1)] * h->a_in[e];
}

int nn_features(celes_nn* n, celes_handle* h, int64_t row0, unsigned short* X, float* Y, celes::DevBuf& frame,
                celes::DevBuf& nbr, bool with_targets) {
    if (h->K < 1) return nn_fail(n, CELES_E_STATE, "problem without incident field");
    if (with_targets && !h->have_solution) return nn_fail(n, CELES_E_STATE, "problem not solved");
    const int64_t N = h->N;
    celes::DevBuf dain, db, drad;
    std::vector<cx<double>> a(N * h->nmax), bb;
    for (int64_t i = 0; i < N * h->nmax; ++i) a[i] = {h->a_in[i].real(), h->a_in[i].imag()};
    // reference component: the dipole term (tau, l = 1, m = +-1) with the largest total weight
    int nref = 0;
    double best = -1;
    for (int tau = 0; tau < 2; ++tau)
        for (int m = -1; m <= 1; m += 2) {
            const int c = tau * h->half + celes::lm_index(1, m);
            double s = 0;
            for (int64_t i = 0; i < N; ++i) s += std::norm(h->a_in[i * h->nmax + c]);
            if (s > best) {
                best = s;
                nref = c;
            }
        }
    if (!dain.ensure(a.size() * 16) || !drad.ensure(N * 8) || !nbr.ensure(N * NN_K * 4) || !frame.ensure(N * 16))
        return nn_fail(n, CELES_E_OOM, "feature buffers");
    hipMemcpy(dain.p, a.data(), a.size() * 16, hipMemcpyHostToDevice);
    hipMemcpy(drad.p, h->radius.data(), N * 8, hipMemcpyHostToDevice);
    if (with_targets) {
        // the network learns the multiple-scattering correction b - T a_in
        // to the single-scattering response (celes_nn_predict adds T a_in back)
        bb.resize(N * h->nmax);
        for (int64_t i = 0; i < N * h->nmax; ++i) {
            const celes::cplx v = h->b[i] - single_scattering(h, i);
            bb[i] = {v.real(), v.imag()};
        }
        if (!db.ensure(bb.size() * 16)) return nn_fail(n, CELES_E_OOM, "feature buffers");
        hipMemcpy(db.p, bb.data(), bb.size() * 16, hipMemcpyHostToDevice);
    }
    hipLaunchKernelGGL(knn16, dim3(nb(N)), dim3(256), 0, 0, h->d_px.as<double>(), h->d_py.as<double>(),
                       h->d_pz.as<double>(), (int)N, nbr.as<int>());
    FeatArgs f;
    f.px = h->d_px.as<double>();
    f.py = h->d_py.as<double>();
    f.pz = h->d_pz.as<double>();
    f.rad = drad.as<double>();
    f.ain = dain.as<cx<double>>();
    f.b = with_targets ? db.as<cx<double>>() : nullptr;
    f.nbr = nbr.as<int>();
    f.n = (int)N;
    f.nmax = h->nmax;
    f.nref = nref;
    f.in_dim = n->in_dim;
    f.in_pad = n->in_pad;
    f.out_pad = n->out_pad;
    f.inv_lambda = n->L > 0 ? h->n0 / h->wavelength : 0.0;
    f.X = X + row0 * n->in_pad;
    f.Y = Y ? Y + row0 * n->out_pad : nullptr;
    f.frame = frame.as<cx<double>>();
    hipLaunchKernelGGL(build_features, dim3(nb(N * n->in_pad)), dim3(256), 0, 0, f);
    hipDeviceSynchronize();
    return hipGetLastError() == hipSuccess ? CELES_OK : nn_fail(n, CELES_E_DEVICE, "feature kernels failed");
}

}  // namespace

extern "C" {

static int celes_nn_create_impl(celes_nn** out, int lmax, uint64_t seed) {
    if (!out || lmax < 1 || lmax > CELES_MAX_LMAX) return CELES_E_ARG;
    std::unique_ptr<celes_nn> n(new celes_nn());
    n->L = lmax;
    n->nmax = 2 * lmax * (lmax + 2);
    n->in_dim = 1 + 2 * n->nmax + NN_K * (4 + 2 * n->nmax);
    n->in_pad = round_up(n->in_dim, TM);
    n->out_dim = 2 * n->nmax;
    n->out_pad = round_up(n->out_dim, TN);
    n->dims[0] = n->in_pad;
    n->dims[1] = n->dims[2] = n->dims[3] = NN_H;
    n->dims[4] = n->out_pad;
    int64_t off = 0;
    for (int l = 0; l < NN_LAYERS; ++l) {
        n->woff.push_back(off);
        off += (int64_t)n->dims[l] * n->dims[l + 1];
        n->boff.push_back(off);
        off += n->dims[l + 1];
    }
    n->nparam = off;
    // initial weights: uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) from SplitMix64
    // counters; padded input rows / output columns and biases start at zero
    std::vector<float> p(off, 0.f);
    const int real_in[NN_LAYERS] = {n->in_dim, NN_H, NN_H, NN_H};
    const int real_out[NN_LAYERS] = {NN_H, NN_H, NN_H, n->out_dim};
    for (int l = 0; l < NN_LAYERS; ++l) {
        const double bound = 1.0 / std::sqrt((double)real_in[l]);
        for (int r = 0; r < real_in[l]; ++r)
            for (int c = 0; c < real_out[l]; ++c) {
                const int64_t idx = n->woff[l] + (int64_t)r * n->dims[l + 1] + c;
                const uint64_t u = splitmix64(seed * 0x100000001b3ULL + (uint64_t)idx);
                const double x = (double)(u >> 11) * (1.0 / 9007199254740992.0);
                p[idx] = (float)((2.0 * x - 1.0) * bound);
            }
    }
    if (!n->w32.ensure(off * 4) || !n->wbf.ensure(off * 2) || !n->grad.ensure(off * 4) || !n->am.ensure(off * 4) ||
        !n->av.ensure(off * 4))
        return CELES_E_OOM;
    hipMemcpy(n->w32.p, p.data(), off * 4, hipMemcpyHostToDevice);
    hipLaunchKernelGGL(to_bf16, dim3(nb(off)), dim3(256), 0, 0, n->w32.as<float>(), n->wbf.as<unsigned short>(), off);
    hipMemset(n->am.p, 0, off * 4);
    hipMemset(n->av.p, 0, off * 4);
    hipDeviceSynchronize();
    *out = n.release();
    return CELES_OK;
}
int celes_nn_create(celes_nn** out, int lmax, uint64_t seed) {
    return celes_guard([&] { return celes_nn_create_impl(out, lmax, seed); });
}


void celes_nn_destroy(celes_nn* n) { delete n; }

const char* celes_nn_last_error(const celes_nn* n) { return n ? n->err.c_str() : ""; }

int celes_nn_dims(const celes_nn* n, int* in_dim, int* in_pad, int* hidden, int* out_dim, int* out_pad,
                  int64_t* nparam) {
    if (!n) return CELES_E_ARG;
    if (in_dim) *in_dim = n->in_dim;
    if (in_pad) *in_pad = n->in_pad;
    if (hidden) *hidden = NN_H;
    if (out_dim) *out_dim = n->out_dim;
    if (out_pad) *out_pad = n->out_pad;
    if (nparam) *nparam = n->nparam;
    return CELES_OK;
}

static int celes_nn_get_params_impl(const celes_nn* n, float* p) {
    if (!n || !p) return CELES_E_ARG;
    return hipMemcpy(p, n->w32.p, n->nparam * 4, hipMemcpyDeviceToHost) == hipSuccess ? CELES_OK : CELES_E_DEVICE;
}
int celes_nn_get_params(const celes_nn* n, float* p) {
    return celes_guard([&] { return celes_nn_get_params_impl(n, p); });
}


static int celes_nn_set_params_impl(celes_nn* n, const float* p) {
    if (!n || !p) return CELES_E_ARG;
    if (hipMemcpy(n->w32.p, p, n->nparam * 4, hipMemcpyHostToDevice) != hipSuccess) return CELES_E_DEVICE;
    hipLaunchKernelGGL(to_bf16, dim3(nb(n->nparam)), dim3(256), 0, 0, n->w32.as<float>(), n->wbf.as<unsigned short>(),
                       n->nparam);
    hipMemset(n->am.p, 0, n->nparam * 4);
    hipMemset(n->av.p, 0, n->nparam * 4);
    n->adam_t = 0;
    return hipDeviceSynchronize() == hipSuccess ? CELES_OK : CELES_E_DEVICE;
}
int celes_nn_set_params(celes_nn* n, const float* p) {
    return celes_guard([&] { return celes_nn_set_params_impl(n, p); });
}


static int celes_nn_loss_grad_impl(celes_nn* n, int64_t M, const float* X, const float* Y, double* loss, float* grad) {
    if (!n || M < 1 || !X || !Y) return CELES_E_ARG;
    const int64_t Mp = round_up((int)M, TM);
    std::vector<unsigned short> xb(Mp * n->in_pad, 0);
    std::vector<float> yp(Mp * n->out_pad, 0.f);
    for (int64_t r = 0; r < M; ++r) {
        for (int c = 0; c < n->in_pad; ++c) xb[r * n->in_pad + c] = f2bf(X[r * n->in_pad + c]);
        for (int c = 0; c < n->out_pad; ++c) yp[r * n->out_pad + c] = Y[r * n->out_pad + c];
    }
    celes::DevBuf dx, dy;
    if (!dx.ensure(xb.size() * 2) || !dy.ensure(yp.size() * 4) || !nn_work(n, Mp)) return CELES_E_OOM;
    hipMemcpy(dx.p, xb.data(), xb.size() * 2, hipMemcpyHostToDevice);
    hipMemcpy(dy.p, yp.data(), yp.size() * 4, hipMemcpyHostToDevice);
    const double l = nn_backward(n, dx.as<unsigned short>(), dy.as<float>(), Mp, M, 0);
    if (loss) *loss = l;
    if (grad) hipMemcpy(grad, n->grad.p, n->nparam * 4, hipMemcpyDeviceToHost);
    return hipGetLastError() == hipSuccess ? CELES_OK : CELES_E_DEVICE;
}
int celes_nn_loss_grad(celes_nn* n, int64_t M, const float* X, const float* Y, double* loss, float* grad) {
    return celes_guard([&] { return celes_nn_loss_grad_impl(n, M, X, Y, loss, grad); });
}


static int celes_nn_forward_impl(celes_nn* n, int64_t M, const float* X, float* Z_out) {
    if (!n || M < 1 || !X || !Z_out) return CELES_E_ARG;
    const int64_t Mp = round_up((int)M, TM);
    std::vector<unsigned short> xb(Mp * n->in_pad, 0);
    for (int64_t r = 0; r < M; ++r)
        for (int c = 0; c < n->in_pad; ++c) xb[r * n->in_pad + c] = f2bf(X[r * n->in_pad + c]);
    celes::DevBuf dx;
    if (!dx.ensure(xb.size() * 2) || !nn_work(n, Mp)) return CELES_E_OOM;
    hipMemcpy(dx.p, xb.data(), xb.size() * 2, hipMemcpyHostToDevice);
    nn_forward(n, dx.as<unsigned short>(), Mp, 0);
    std::vector<float> z(Mp * n->out_pad);
    hipMemcpy(z.data(), n->Z[NN_LAYERS - 1].p, z.size() * 4, hipMemcpyDeviceToHost);
    std::memcpy(Z_out, z.data(), M * n->out_pad * 4);
    return CELES_OK;
}
int celes_nn_forward(celes_nn* n, int64_t M, const float* X, float* Z_out) {
    return celes_guard([&] { return celes_nn_forward_impl(n, M, X, Z_out); });
}


static int celes_nn_features_impl(celes_nn* n, celes_handle* h, float* X_out, float* Y_out) {
    if (!n || !h || h->L != n->L) return CELES_E_ARG;
    celes::DevBuf dx, dy, fr, nbr;
    const int64_t N = h->N;
    if (!dx.ensure(N * n->in_pad * 2) || !dy.ensure(N * n->out_pad * 4)) return CELES_E_OOM;
    int rc = nn_features(n, h, 0, dx.as<unsigned short>(), dy.as<float>(), fr, nbr, h->have_solution);
    if (rc != CELES_OK) return rc;
    if (X_out) {
        std::vector<unsigned short> xb(N * n->in_pad);
        hipMemcpy(xb.data(), dx.p, xb.size() * 2, hipMemcpyDeviceToHost);
        for (size_t i = 0; i < xb.size(); ++i) X_out[i] = bf2f(xb[i]);
    }
    if (Y_out && h->have_solution) hipMemcpy(Y_out, dy.p, N * n->out_pad * 4, hipMemcpyDeviceToHost);
    return CELES_OK;
}
int celes_nn_features(celes_nn* n, celes_handle* h, float* X_out, float* Y_out) {
    return celes_guard([&] { return celes_nn_features_impl(n, h, X_out, Y_out); });
}


static int celes_nn_add_training_problem_impl(celes_nn* n, celes_handle* h) {
    if (!n || !h || h->L != n->L) return CELES_E_ARG;
    const int64_t N = h->N;
    celes::DevBuf dx, dy, fr, nbr;
    if (!dx.ensure(N * n->in_pad * 2) || !dy.ensure(N * n->out_pad * 4)) return CELES_E_OOM;
    int rc = nn_features(n, h, 0, dx.as<unsigned short>(), dy.as<float>(), fr, nbr, true);
    if (rc != CELES_OK) return rc;
    const size_t x0 = n->hX.size(), y0 = n->hY.size();
    n->hX.resize(x0 + N * n->in_pad);
    n->hY.resize(y0 + N * n->out_pad);
    hipMemcpy(n->hX.data() + x0, dx.p, N * n->in_pad * 2, hipMemcpyDeviceToHost);
    hipMemcpy(n->hY.data() + y0, dy.p, N * n->out_pad * 4, hipMemcpyDeviceToHost);
    n->rows += N;
    n->dX.release();   // re-upload on the next train call
    return CELES_OK;
}
int celes_nn_add_training_problem(celes_nn* n, celes_handle* h) {
    return celes_guard([&] { return celes_nn_add_training_problem_impl(n, h); });
}


static int celes_nn_train_impl(celes_nn* n, int epochs, int batch, double lr, uint64_t seed, double* loss_out) {
    if (!n || epochs < 1 || batch < TM) return CELES_E_ARG;
    if (n->rows < 1) return nn_fail(n, CELES_E_STATE, "no training data");
    batch = round_up(batch, TM);
    if (!n->dX.p) {
        if (!n->dX.ensure(n->hX.size() * 2) || !n->dY.ensure(n->hY.size() * 4)) return CELES_E_OOM;
        hipMemcpy(n->dX.p, n->hX.data(), n->hX.size() * 2, hipMemcpyHostToDevice);
        hipMemcpy(n->dY.p, n->hY.data(), n->hY.size() * 4, hipMemcpyHostToDevice);
    }
    celes::DevBuf bx, by, bidx;
    if (!bx.ensure((size_t)batch * n->in_pad * 2) || !by.ensure((size_t)batch * n->out_pad * 4) ||
        !bidx.ensure((size_t)batch * 8) || !nn_work(n, batch))
        return CELES_E_OOM;
    std::vector<int64_t> perm(n->rows);
    double last = 0;
    hipStream_t s = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        std::iota(perm.begin(), perm.end(), 0);
        for (int64_t i = n->rows - 1; i > 0; --i) {
            const int64_t j = (int64_t)(splitmix64(seed ^ ((uint64_t)ep << 40) ^ (uint64_t)i) % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        double sum = 0;
        int64_t nbt = 0;
        for (int64_t r0 = 0; r0 < n->rows; r0 += batch) {
            const int64_t mv = std::min<int64_t>(batch, n->rows - r0);
            // gather the minibatch rows (padding rows get index -1 -> zeros)
            std::vector<int64_t> idx(batch, -1);
            for (int64_t r = 0; r < mv; ++r) idx[r] = perm[r0 + r];
            hipMemcpyAsync(bidx.p, idx.data(), batch * 8, hipMemcpyHostToDevice, s);
            hipLaunchKernelGGL(gather_rows, dim3(nb((int64_t)batch * (n->in_pad + n->out_pad))), dim3(256), 0, s,
                               n->dX.as<unsigned short>(), n->dY.as<float>(), bidx.as<int64_t>(), (int64_t)batch,
                               n->in_pad, n->out_pad, bx.as<unsigned short>(), by.as<float>());
            sum += nn_backward(n, bx.as<unsigned short>(), by.as<float>(), batch, mv, s);
            ++nbt;
            ++n->adam_t;
            const float b1 = 0.9f, b2 = 0.999f;
            const float c1 = 1.f - std::pow(b1, (float)n->adam_t), c2 = 1.f - std::pow(b2, (float)n->adam_t);
            // cosine learning-rate schedule over the epochs
            const float lr_t = (float)(lr * 0.5 * (1.0 + std::cos(M_PI * ep / epochs)));
            hipLaunchKernelGGL(adam_step, dim3(nb(n->nparam)), dim3(256), 0, s, n->w32.as<float>(), n->grad.as<float>(),
                               n->am.as<float>(), n->av.as<float>(), n->wbf.as<unsigned short>(), n->nparam, lr_t, b1,
                               b2, 1e-8f, c1, c2);
        }
        last = sum / std::max<int64_t>(1, nbt);
    }
    hipStreamSynchronize(s);
    if (loss_out) *loss_out = last;
    return hipGetLastError() == hipSuccess ? CELES_OK : nn_fail(n, CELES_E_DEVICE, "training kernels failed");
}
int celes_nn_train(celes_nn* n, int epochs, int batch, double lr, uint64_t seed, double* loss_out) {
    return celes_guard([&] { return celes_nn_train_impl(n, epochs, batch, lr, seed, loss_out); });
}


static int celes_nn_predict_impl(celes_nn* n, celes_handle* h, double* x0_out) {
    if (!n || !h || !x0_out || h->L != n->L) return CELES_E_ARG;
    const int64_t N = h->N, Np = round_up((int)N, TM);
    celes::DevBuf dx, fr, nbr, x0;
    if (!dx.ensure(Np * n->in_pad * 2) || !nn_work(n, Np) || !x0.ensure(N * h->nmax * 16)) return CELES_E_OOM;
    hipMemset(dx.p, 0, Np * n->in_pad * 2);
    int rc = nn_features(n, h, 0, dx.as<unsigned short>(), nullptr, fr, nbr, false);
    if (rc != CELES_OK) return rc;
    nn_forward(n, dx.as<unsigned short>(), Np, 0);
    hipLaunchKernelGGL(unframe, dim3(nb(N * h->nmax)), dim3(256), 0, 0, n->Z[NN_LAYERS - 1].as<float>(), n->out_pad,
                       fr.as<cx<double>>(), (int)N, h->nmax, x0.as<cx<double>>());
    if (hipMemcpy(x0_out, x0.p, N * h->nmax * 16, hipMemcpyDeviceToHost) != hipSuccess) return CELES_E_DEVICE;
    for (int64_t e = 0; e < N * h->nmax; ++e) {      // predicted correction + single scattering
        const celes::cplx t = single_scattering(h, e);
        x0_out[2 * e] += t.real();
        x0_out[2 * e + 1] += t.imag();
    }
    return CELES_OK;
}
int celes_nn_predict(celes_nn* n, celes_handle* h, double* x0_out) {
    return celes_guard([&] { return celes_nn_predict_impl(n, h, x0_out); });
}


}  // extern "C"

#include "precond.hpp"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <numeric>
#include <thread>

namespace celes {

// concurrent block factorisations during set-up (one host thread, stream and
// rocBLAS handle each)
constexpr int PRE_STREAMS = 4;
// tile of the inverse apply: rows per block, columns per partial sum
constexpr int PA_ROWS = 256, PA_COLS = 256;

void partition_cuboids(int64_t N, const double* pos, double edge, std::vector<int64_t>* perm,
                       std::vector<int64_t>* offsets) {
    double lo[3] = {1e300, 1e300, 1e300};
    for (int64_t i = 0; i < N; ++i)
        for (int c = 0; c < 3; ++c) lo[c] = std::min(lo[c], pos[3 * i + c]);
    std::vector<int64_t> cell(3 * N);
    int64_t nc[3] = {0, 0, 0};
    for (int64_t i = 0; i < N; ++i)
        for (int c = 0; c < 3; ++c) {
            cell[3 * i + c] = (int64_t)std::floor((pos[3 * i + c] - lo[c]) / edge);
            nc[c] = std::max(nc[c], cell[3 * i + c] + 1);
        }
    std::vector<int64_t> lin(N);
    for (int64_t i = 0; i < N; ++i) lin[i] = cell[3 * i] + nc[0] * (cell[3 * i + 1] + nc[1] * cell[3 * i + 2]);
    perm->resize(N);
    std::iota(perm->begin(), perm->end(), 0);
    std::stable_sort(perm->begin(), perm->end(), [&](int64_t a, int64_t b) { return lin[a] < lin[b]; });
    offsets->clear();
    for (int64_t t = 0; t < N; ++t)
        if (t == 0 || lin[(*perm)[t]] != lin[(*perm)[t - 1]]) offsets->push_back(t);
    offsets->push_back(N);
}

double BlockPrecond::precond_bytes(int64_t N, int L, const std::vector<int64_t>& offsets) {
    const double nm = 2.0 * L * (L + 2);
    double mats = 0, max_dim = 0;
    for (size_t j = 0; j + 1 < offsets.size(); ++j) {
        const double dim = (double)(offsets[j + 1] - offsets[j]) * nm;
        mats += dim * dim;
        max_dim = std::max(max_dim, dim);
    }
    const double nsplit = std::ceil(max_dim / PA_COLS);
    return mats * (16.0 + 8.0) + nsplit * (double)N * nm * 16.0;
}

int plan_cuboid_edge(int64_t N, const double* pos, int L, double target, double cap, double* edge,
                     std::vector<int64_t>* offsets, std::string* msg) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < N; ++i)
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], pos[3 * i + c]);
            hi[c] = std::max(hi[c], pos[3 * i + c]);
        }
    const double D = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
    if (!(target > 0)) target = 100.0;
    std::vector<int64_t> perm, off;
    double last_bytes = 0;
    for (double e = 1.02 * D; e >= D / 4096.0; e *= 0.92) {
        partition_cuboids(N, pos, e, &perm, &off);
        const double nb = (double)(off.size() - 1);
        const double bytes = BlockPrecond::precond_bytes(N, L, off);
        last_bytes = bytes;
        if ((double)N / nb <= target && (!(cap > 0) || bytes <= cap)) {
            *edge = e;
            *offsets = off;
            return 0;
        }
    }
    *msg = "no cuboid edge fits the preconditioner budget (smallest candidate needs " +
           std::to_string((long long)(last_bytes / (1 << 20))) + " MiB, cap " +
           std::to_string((long long)(cap / (1 << 20))) + " MiB)";
    return CELES_E_OOM_INTERNAL;
}

// ---------------------------------------------------------------------------
// assembly: M_j[r, c] = delta_rc - Q_n(a) W^{ab}_{n n'}, r = a nmax + n,
// c = b nmax + n' (column-major), W^{ab}_{nn'} = A_{n'n}(r_a - r_b).
// One thread per (block, a, b, receiving (l, m)).
// ---------------------------------------------------------------------------
struct AsmArgs {
    const double* pos;          // [N][3]
    const int64_t* perm;
    const int64_t* boff;
    const int64_t* moff;
    const cx<double>* tq;       // [N][2][L]
    const double* a5;           // [L][2L+1][L][2L+1][2L+1]
    const double* b5;
    const cx<double>* lut;      // [n_int][2][4]: h_0, h_1 Horner coefficients
    double lut_lo, lut_inv_dr;
    int lut_n;
    double k;
    int L, hmode, blk;
    cx<double>* mat;
};

__device__ inline void hankel_row(const AsmArgs& g, double d, cx<double>* h) {
    const int P = 2 * g.L;
    if (g.hmode == 0) {
        double s = (d - g.lut_lo) * g.lut_inv_dr;
        int q = (int)s;
        q = q < 0 ? 0 : (q >= g.lut_n ? g.lut_n - 1 : q);
        double t = s - q;
        const cx<double>* c = g.lut + (size_t)q * 8;
        for (int p = 0; p <= 1; ++p) {
            h[p].re = ((c[4 * p + 3].re * t + c[4 * p + 2].re) * t + c[4 * p + 1].re) * t + c[4 * p].re;
            h[p].im = ((c[4 * p + 3].im * t + c[4 * p + 2].im) * t + c[4 * p + 1].im) * t + c[4 * p].im;
        }
        const double inv = 1.0 / (g.k * d);
        for (int p = 1; p < P; ++p) {
            double f = (2.0 * p + 1.0) * inv;
            h[p + 1] = {f * h[p].re - h[p - 1].re, f * h[p].im - h[p - 1].im};
        }
    } else {
        double x = g.k * d, s, cc;
        sincos(x, &s, &cc);
        double inv = 1.0 / x;
        h[0] = {s * inv, -cc * inv};
        h[1] = {(h[0].re - cc) * inv, (h[0].im - s) * inv};
        for (int p = 1; p < P; ++p) {
            double f = (2.0 * p + 1.0) * inv;
            h[p + 1] = {f * h[p].re - h[p - 1].re, f * h[p].im - h[p - 1].im};
        }
    }
}

__global__ void assemble_kernel(AsmArgs g, int64_t ntot) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntot) return;
    const int L = g.L, half = L * (L + 2), nmax = 2 * half, W = 2 * L + 1;
    const int64_t o = g.boff[g.blk], nj = g.boff[g.blk + 1] - o;
    const int c_out = (int)(t % half);
    const int64_t ab = t / half;
    const int64_t a = ab % nj, b = ab / nj;
    const int64_t dim = nj * nmax;
    cx<double>* M = g.mat + g.moff[g.blk];
    const int l = (int)floor(sqrt((double)(c_out + 1)));
    int ll = l;
    while (ll * (ll + 2) < c_out + 1) ++ll;
    while ((ll - 1) * (ll + 1) >= c_out + 1) --ll;
    const int m = c_out + 1 - ll * (ll + 1);
    const int64_t ia = g.perm[o + a], ib = g.perm[o + b];
    if (a == b) {
        for (int tau = 0; tau < 2; ++tau)
            for (int tp = 0; tp < 2; ++tp)
                for (int cp = 0; cp < half; ++cp) {
                    int64_t r = a * nmax + tau * half + c_out, c = b * nmax + tp * half + cp;
                    M[r + c * dim] = {(r == c) ? 1.0 : 0.0, 0.0};
                }
        return;
    }
    const double dx = g.pos[3 * ia] - g.pos[3 * ib], dy = g.pos[3 * ia + 1] - g.pos[3 * ib + 1],
                 dz = g.pos[3 * ia + 2] - g.pos[3 * ib + 2];
    const double rho = sqrt(dx * dx + dy * dy), d = sqrt(dx * dx + dy * dy + dz * dz);
    const double ct = dz / d, st = rho / d;
    const double ph = rho > 0 ? atan2(dy, dx) : 0.0;
    cx<double> h[13];
    hankel_row(g, d, h);
    // normalized Legendre P_p^mu(ct), 0 <= mu <= p <= 2L
    double P[13][13];
    double pmm = 0.70710678118654752440;
    for (int mu = 0; mu <= 2 * L; ++mu) {
        if (mu > 0) pmm *= sqrt((2.0 * mu + 1.0) / (2.0 * mu)) * st;
        P[mu][mu] = pmm;
        if (mu + 1 <= 2 * L) P[mu + 1][mu] = sqrt(2.0 * mu + 3.0) * ct * pmm;
        for (int p = mu + 2; p <= 2 * L; ++p) {
            double aa = sqrt((4.0 * p * p - 1.0) / ((double)p * p - (double)mu * mu));
            double bb = sqrt((2.0 * p + 1.0) * ((p - 1.0) * (p - 1.0) - (double)mu * mu) /
                             ((2.0 * p - 3.0) * ((double)p * p - (double)mu * mu)));
            P[p][mu] = aa * ct * P[p - 1][mu] - bb * P[p - 2][mu];
        }
    }
    const cx<double> q1 = g.tq[(ia * 2 + 0) * L + (ll - 1)], q2 = g.tq[(ia * 2 + 1) * L + (ll - 1)];
    for (int lp = 1; lp <= L; ++lp)
        for (int mp = -lp; mp <= lp; ++mp) {
            const int mu = abs(mp - m);
            double Are = 0, Aim = 0, Bre = 0, Bim = 0;
            for (int p = 0; p <= 2 * L; ++p) {
                if (p < mu) continue;
                // coefficient a5(l', m' | l, m | p) (source first)
                size_t co = ((((size_t)(lp - 1) * W + (mp + L)) * L + (ll - 1)) * W + (m + L)) * W + p;
                const double ca = g.a5[co], cb = g.b5[co];
                const double hp = P[p][mu];
                Are += ca * h[p].re * hp;
                Aim += ca * h[p].im * hp;
                Bre += cb * h[p].re * hp;
                Bim += cb * h[p].im * hp;
            }
            double s, c;
            sincos((double)(mp - m) * ph, &s, &c);
            const cx<double> A = {Are * c - Aim * s, Are * s + Aim * c};
            // B = i * (Bre + i Bim) * e^{i(m'-m) phi}
            const cx<double> Bp = {Bre * c - Bim * s, Bre * s + Bim * c};
            const cx<double> B = {-Bp.im, Bp.re};
            const int cp = lp * (lp + 1) + mp - 1;
            for (int tau = 0; tau < 2; ++tau) {
                const cx<double> q = tau == 0 ? q1 : q2;
                for (int tp = 0; tp < 2; ++tp) {
                    const cx<double> w = (tau == tp) ? A : B;
                    int64_t r = a * nmax + tau * half + c_out, col = b * nmax + tp * half + cp;
                    M[r + col * dim] = {-(q.re * w.re - q.im * w.im), -(q.re * w.im + q.im * w.re)};
                }
            }
        }
}

// Apply: out[perm rows of block j] = Minv_j in[perm rows of block j].  The
// work is split over 256-row x 256-column tiles of every block (HBM-bound:
// each matrix element is read once); the x tile is gathered into LDS, each
// thread owns one row and streams its 256 column entries (column-major, so a
// wave reads 64 consecutive rows = contiguous memory).  Partial sums per
// column tile go to part[s][permuted row] and a second kernel adds them in a
// fixed order and scatters back to the caller's sphere order.

// T: vector precision; TM: matrix precision (FP64 inverse, or its FP32 copy
// for complex64 vectors); accumulation in TM
// streaming load of one complex matrix entry that bypasses cache retention
// (the inverses are read once per apply)
template <typename TM>
__device__ __forceinline__ cx<TM> stream_load(const cx<TM>* p) {
    typedef TM v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return {v.x, v.y};
}

template <typename T, typename TM>
__global__ void __launch_bounds__(PA_ROWS) apply_tiles(const cx<TM>* __restrict__ inv,
                                                       const int64_t* __restrict__ perm,
                                                       const int64_t* __restrict__ boff,
                                                       const int64_t* __restrict__ moff, int nmax,
                                                       const cx<T>* __restrict__ in, cx<double>* __restrict__ part,
                                                       int64_t n) {
    const int j = blockIdx.z, s = blockIdx.y;
    const int64_t o = boff[j], dim = (boff[j + 1] - o) * nmax;
    const int64_t r0 = (int64_t)blockIdx.x * PA_ROWS;
    if (r0 >= dim) return;
    const int64_t r = r0 + threadIdx.x;
    const int64_t c0 = (int64_t)s * PA_COLS;
    cx<double>* dst = part + (int64_t)s * n + o * nmax;
    if (c0 >= dim) {
        if (r < dim) dst[r] = {0.0, 0.0};
        return;
    }
    const int ncol = (int)(dim - c0 < PA_COLS ? dim - c0 : PA_COLS);
    __shared__ cx<TM> xs[PA_COLS];
    if (threadIdx.x < ncol) {
        const int64_t c = c0 + threadIdx.x;
        const cx<T> v = in[perm[o + c / nmax] * nmax + c % nmax];
        xs[threadIdx.x] = {(TM)v.re, (TM)v.im};
    }
    __syncthreads();
    if (r >= dim) return;
    const cx<TM>* M = inv + moff[j] + c0 * dim + r;
    // eight column loads in flight per thread, four accumulator pairs
    TM re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
    int c = 0;
    for (; c + 8 <= ncol; c += 8) {
        cx<TM> a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = stream_load(M + (int64_t)(c + u) * dim);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const cx<TM> x = xs[c + u];
            re[u & 3] = fma(a[u].re, x.re, fma(-a[u].im, x.im, re[u & 3]));
            im[u & 3] = fma(a[u].re, x.im, fma(a[u].im, x.re, im[u & 3]));
        }
    }
    for (; c < ncol; ++c) {
        const cx<TM> a0 = stream_load(M + (int64_t)c * dim), x0 = xs[c];
        re[0] = fma(a0.re, x0.re, fma(-a0.im, x0.im, re[0]));
        im[0] = fma(a0.re, x0.im, fma(a0.im, x0.re, im[0]));
    }
    dst[r] = {(double)((re[0] + re[1]) + (re[2] + re[3])), (double)((im[0] + im[1]) + (im[2] + im[3]))};
}

// grid-stride: the inverses can hold more than 2^32 entries, more work-items
// than one dispatch can address (its grid size is a 32-bit work-item count)
__global__ void narrow_kernel(const cx<double>* __restrict__ a, cx<float>* __restrict__ b, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
        b[t] = {(float)a[t].re, (float)a[t].im};
}
constexpr unsigned NARROW_BLOCKS = 16384;   // 4M work-items per launch

// out[perm[t / nmax] nmax + t % nmax] = sum_s part[s][t], t in permuted order
template <typename T>
__global__ void apply_reduce(const cx<double>* __restrict__ part, int nsplit, const int64_t* __restrict__ perm,
                             int nmax, int64_t n, cx<T>* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    double re = 0, im = 0;
    for (int s = 0; s < nsplit; ++s) {
        const cx<double> v = part[(int64_t)s * n + t];
        re += v.re;
        im += v.im;
    }
    out[perm[t / nmax] * nmax + t % nmax] = {(T)re, (T)im};
}

BlockPrecond::~BlockPrecond() {
    if (d_perm_) hipFree(d_perm_);
    if (d_boff_) hipFree(d_boff_);
    if (d_moff_) hipFree(d_moff_);
    if (d_inv_) hipFree(d_inv_);
    if (d_inv32_) hipFree(d_inv32_);
    if (d_part_) hipFree(d_part_);
}

int BlockPrecond::build(int64_t N, int L, const double* pos, double k, const cplx* tq, double edge, int hmode,
                        const void* lut_dev, double lut_lo, double lut_dr, int lut_n, std::string* msg) {
    N_ = N;
    L_ = L;
    nmax_ = 2 * L * (L + 2);
    edge_ = edge;
    partition_cuboids(N, pos, edge, &perm_, &offsets_);
    const int nb = (int)offsets_.size() - 1;
    std::vector<int64_t> moff(nb);
    mat_elems_ = 0;
    max_dim_ = 0;
    for (int j = 0; j < nb; ++j) {
        int64_t dim = (offsets_[j + 1] - offsets_[j]) * nmax_;
        moff[j] = (int64_t)mat_elems_;
        mat_elems_ += (size_t)dim * dim;
        max_dim_ = std::max<int>(max_dim_, (int)dim);
    }
    auto dev = [&](void** p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; };
    if (!dev((void**)&d_perm_, N * 8) || !dev((void**)&d_boff_, (nb + 1) * 8) || !dev((void**)&d_moff_, nb * 8) ||
        !dev((void**)&d_inv_, mat_elems_ * sizeof(cx<double>)) ||
        !dev((void**)&d_part_, (size_t)((max_dim_ + PA_COLS - 1) / PA_COLS) * N * nmax_ * sizeof(cx<double>))) {
        *msg = "cannot allocate the preconditioner (" + std::to_string(mat_elems_ * 16 / (1 << 20)) + " MiB)";
        return CELES_E_OOM_INTERNAL;
    }
    hipMemcpy(d_perm_, perm_.data(), N * 8, hipMemcpyHostToDevice);
    hipMemcpy(d_boff_, offsets_.data(), (nb + 1) * 8, hipMemcpyHostToDevice);
    hipMemcpy(d_moff_, moff.data(), nb * 8, hipMemcpyHostToDevice);
    // coefficient tables and per-sphere data
    const int W = 2 * L + 1;
    const size_t tsz = (size_t)L * W * L * W * W;
    std::vector<double> a5(tsz, 0.0), b5(tsz, 0.0);
    for (int l = 1; l <= L; ++l)
        for (int m = -l; m <= l; ++m)
            for (int lp = 1; lp <= L; ++lp)
                for (int mp = -lp; mp <= lp; ++mp)
                    for (int p = 0; p <= 2 * L; ++p) {
                        size_t o = ((((size_t)(l - 1) * W + (m + L)) * L + (lp - 1)) * W + (mp + L)) * W + p;
                        a5[o] = a5_coef(l, m, lp, mp, p);
                        b5[o] = b5im_coef(l, m, lp, mp, p);
                    }
    double *d_a5 = nullptr, *d_b5 = nullptr, *d_pos = nullptr;
    cx<double>* d_tq = nullptr;
    std::vector<cx<double>> t64((size_t)N * 2 * L);
    for (size_t i = 0; i < t64.size(); ++i) t64[i] = {tq[i].real(), tq[i].imag()};
    if (!dev((void**)&d_a5, tsz * 8) || !dev((void**)&d_b5, tsz * 8) || !dev((void**)&d_pos, N * 24) ||
        !dev((void**)&d_tq, t64.size() * 16)) {
        *msg = "cannot allocate assembly tables";
        return CELES_E_OOM_INTERNAL;
    }
    hipMemcpy(d_a5, a5.data(), tsz * 8, hipMemcpyHostToDevice);
    hipMemcpy(d_b5, b5.data(), tsz * 8, hipMemcpyHostToDevice);
    hipMemcpy(d_pos, pos, N * 24, hipMemcpyHostToDevice);
    hipMemcpy(d_tq, t64.data(), t64.size() * 16, hipMemcpyHostToDevice);
    AsmArgs g;
    g.pos = d_pos;
    g.perm = d_perm_;
    g.boff = d_boff_;
    g.moff = d_moff_;
    g.tq = d_tq;
    g.a5 = d_a5;
    g.b5 = d_b5;
    g.lut = (const cx<double>*)lut_dev;
    g.lut_lo = lut_lo;
    g.lut_inv_dr = 1.0 / lut_dr;
    g.lut_n = lut_n;
    g.k = k;
    g.L = L;
    g.hmode = hmode;
    g.mat = d_inv_;
    // The blocks are independent: PRE_STREAMS host threads, each with its own
    // stream, rocBLAS handle and pivot array, take blocks largest first from
    // a shared counter, so that one block's latency-bound panel kernels
    // overlap another block's GEMMs.  Each block's arithmetic does not depend
    // on the schedule.  Two info slots per block are checked once at the end.
    rocblas_int* d_info = nullptr;
    int rc = dev((void**)&d_info, (size_t)2 * nb * sizeof(rocblas_int)) ? 0 : CELES_E_OOM_INTERNAL;
    if (rc != 0) *msg = "cannot allocate factorisation info";
    if (rc == 0) hipMemset(d_info, 0, (size_t)2 * nb * sizeof(rocblas_int));
    std::vector<int> order(nb);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return offsets_[x + 1] - offsets_[x] > offsets_[y + 1] - offsets_[y];
    });
    const int nstreams = std::max(1, std::min(PRE_STREAMS, nb));
    std::atomic<int> next{0};
    std::atomic<int> failed{0};
    hipDeviceSynchronize();  // tables and index arrays are on the device before any worker starts
    int device = 0;
    hipGetDevice(&device);
    auto worker = [&]() {
        hipSetDevice(device);
        hipStream_t st = nullptr;
        rocblas_handle rb = nullptr;
        rocblas_int* d_ipiv = nullptr;
        if (hipStreamCreate(&st) != hipSuccess) {
            failed = CELES_E_DEVICE_INTERNAL;
            return;
        }
        if (rocblas_create_handle(&rb) != rocblas_status_success || rocblas_set_stream(rb, st) != rocblas_status_success)
            failed = CELES_E_DEVICE_INTERNAL;
        else if (hipMalloc((void**)&d_ipiv, (size_t)max_dim_ * sizeof(rocblas_int)) != hipSuccess)
            failed = CELES_E_OOM_INTERNAL;
        while (!failed) {
            const int q = next.fetch_add(1);
            if (q >= nb) break;
            const int j = order[q];
            AsmArgs gj = g;
            gj.blk = j;
            const int64_t nj = offsets_[j + 1] - offsets_[j];
            const int64_t ntot = nj * nj * (nmax_ / 2);
            hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, st, gj, ntot);
            const int dim = (int)(nj * nmax_);
            rocblas_double_complex* A = (rocblas_double_complex*)(d_inv_ + moff[j]);
            if (rocsolver_zgetrf(rb, dim, dim, A, dim, d_ipiv, d_info + 2 * j) != rocblas_status_success ||
                rocsolver_zgetri(rb, dim, A, dim, d_ipiv, d_info + 2 * j + 1) != rocblas_status_success)
                failed = CELES_E_DEVICE_INTERNAL;
        }
        if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) failed = CELES_E_DEVICE_INTERNAL;
        if (rb) rocblas_destroy_handle(rb);
        if (d_ipiv) hipFree(d_ipiv);
        hipStreamDestroy(st);
    };
    if (rc == 0) {
        std::vector<std::thread> pool;
        for (int t = 0; t < nstreams; ++t) pool.emplace_back(worker);
        for (auto& th : pool) th.join();
        if (failed) {
            rc = failed;
            *msg = rc == CELES_E_OOM_INTERNAL ? "cannot allocate pivots" : "rocsolver LU/inverse failed";
        }
    }
    if (rc == 0) {
        std::vector<rocblas_int> info(2 * nb, 0);
        hipMemcpy(info.data(), d_info, info.size() * sizeof(rocblas_int), hipMemcpyDeviceToHost);
        for (int j = 0; j < nb && rc == 0; ++j)
            if (info[2 * j] != 0 || info[2 * j + 1] != 0) {
                *msg = "singular preconditioner block " + std::to_string(j);
                rc = CELES_E_DEVICE_INTERNAL;
            }
    }
    // complex64 copy of the inverses for the complex64 inner solves (half the
    // bytes of the HBM-bound apply); the factorisation itself is FP64
    if (rc == 0) {
        if (!dev((void**)&d_inv32_, mat_elems_ * sizeof(cx<float>))) {
            *msg = "cannot allocate the complex64 preconditioner copy";
            rc = CELES_E_OOM_INTERNAL;
        } else {
            const unsigned blocks = (unsigned)std::min<size_t>(NARROW_BLOCKS, (mat_elems_ + 255) / 256);
            hipLaunchKernelGGL(narrow_kernel, dim3(blocks), dim3(256), 0, 0, d_inv_, d_inv32_, (int64_t)mat_elems_);
        }
    }
    hipDeviceSynchronize();
    hipFree(d_info);
    hipFree(d_a5);
    hipFree(d_b5);
    hipFree(d_pos);
    hipFree(d_tq);
    if (hipGetLastError() != hipSuccess && rc == 0) {
        *msg = "preconditioner assembly failed";
        rc = CELES_E_DEVICE_INTERNAL;
    }
    return rc;
}

template <typename T>
int BlockPrecond::apply(const cx<T>* in, cx<T>* out, hipStream_t s) const {
    const int nb = (int)offsets_.size() - 1;
    const int nsplit = (max_dim_ + PA_COLS - 1) / PA_COLS;
    const int64_t n = N_ * nmax_;
    dim3 grid((unsigned)((max_dim_ + PA_ROWS - 1) / PA_ROWS), (unsigned)nsplit, (unsigned)nb);
    if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL((apply_tiles<T, float>), grid, dim3(PA_ROWS), 0, s, d_inv32_, d_perm_, d_boff_, d_moff_,
                           nmax_, in, d_part_, n);
    else
        hipLaunchKernelGGL((apply_tiles<T, double>), grid, dim3(PA_ROWS), 0, s, d_inv_, d_perm_, d_boff_, d_moff_,
                           nmax_, in, d_part_, n);
    hipLaunchKernelGGL(apply_reduce<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_part_, nsplit,
                       d_perm_, nmax_, n, out);
    return hipGetLastError() == hipSuccess ? 0 : CELES_E_DEVICE_INTERNAL;
}

template int BlockPrecond::apply<double>(const cx<double>*, cx<double>*, hipStream_t) const;
template int BlockPrecond::apply<float>(const cx<float>*, cx<float>*, hipStream_t) const;

// Several right-hand sides: block (row tile, cuboid j, group g) owns rows
// r0..r0+255 of M_j^{-1} and right-hand sides 8g..8g+7; it walks all column
// tiles of the block (no split, so no partial sums), staging the group's x
// entries of a column tile in LDS, so each matrix entry is loaded once for up
// to eight right-hand sides.
constexpr int PM_KB = 8;
template <typename T, typename TM>
__global__ void __launch_bounds__(PA_ROWS) apply_tiles_multi(const cx<TM>* __restrict__ inv,
                                                             const int64_t* __restrict__ perm,
                                                             const int64_t* __restrict__ boff,
                                                             const int64_t* __restrict__ moff, int nmax, int nb,
                                                             const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                             int K, int64_t stride, const int* __restrict__ active,
                                                             int sys0) {
    const int j = blockIdx.z % nb, g = blockIdx.z / nb;
    const int k0 = g * PM_KB, kn = min(PM_KB, K - k0);
    if (active) {
        int any = 0;
        for (int q = 0; q < kn; ++q) any |= active[sys0 + k0 + q];
        if (!any) return;
    }
    const int64_t o = boff[j], dim = (boff[j + 1] - o) * nmax;
    const int64_t r0 = (int64_t)blockIdx.x * PA_ROWS;
    if (r0 >= dim) return;
    const int64_t r = r0 + threadIdx.x;
    __shared__ cx<TM> xs[PA_COLS][PM_KB];
    TM re[PM_KB], im[PM_KB];
#pragma unroll
    for (int q = 0; q < PM_KB; ++q) re[q] = im[q] = 0;
    const cx<TM>* Mrow = inv + moff[j] + (r < dim ? r : 0);
    for (int64_t c0 = 0; c0 < dim; c0 += PA_COLS) {
        const int ncol = (int)(dim - c0 < PA_COLS ? dim - c0 : PA_COLS);
        __syncthreads();
        for (int e = threadIdx.x; e < ncol * PM_KB; e += PA_ROWS) {
            const int c = e / PM_KB, q = e % PM_KB;
            cx<TM> v = {0, 0};
            if (q < kn) {
                const int64_t cc = c0 + c;
                const cx<T> w = in[(int64_t)(k0 + q) * stride + perm[o + cc / nmax] * nmax + cc % nmax];
                v = {(TM)w.re, (TM)w.im};
            }
            xs[c][q] = v;
        }
        __syncthreads();
        if (r < dim) {
            for (int c = 0; c < ncol; ++c) {
                const cx<TM> a = stream_load(Mrow + (c0 + c) * dim);
#pragma unroll
                for (int q = 0; q < PM_KB; ++q) {
                    const cx<TM> x = xs[c][q];
                    re[q] = fma(a.re, x.re, fma(-a.im, x.im, re[q]));
                    im[q] = fma(a.re, x.im, fma(a.im, x.re, im[q]));
                }
            }
        }
    }
    if (r >= dim) return;
    const int64_t dst = perm[o + r / nmax] * nmax + r % nmax;
    for (int q = 0; q < kn; ++q) out[(int64_t)(k0 + q) * stride + dst] = {(T)re[q], (T)im[q]};
}

template <typename T>
int BlockPrecond::apply_multi(const cx<T>* in, cx<T>* out, int K, int64_t stride, const int* active, int sys0,
                              hipStream_t s) const {
    if (K < 1) return 0;
    const int nb = (int)offsets_.size() - 1;
    const int ng = (K + PM_KB - 1) / PM_KB;
    dim3 grid((unsigned)((max_dim_ + PA_ROWS - 1) / PA_ROWS), 1, (unsigned)(nb * ng));
    if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL((apply_tiles_multi<T, float>), grid, dim3(PA_ROWS), 0, s, d_inv32_, d_perm_, d_boff_,
                           d_moff_, nmax_, nb, in, out, K, stride, active, sys0);
    else
        hipLaunchKernelGGL((apply_tiles_multi<T, double>), grid, dim3(PA_ROWS), 0, s, d_inv_, d_perm_, d_boff_,
                           d_moff_, nmax_, nb, in, out, K, stride, active, sys0);
    return hipGetLastError() == hipSuccess ? 0 : CELES_E_DEVICE_INTERNAL;
}
template int BlockPrecond::apply_multi<double>(const cx<double>*, cx<double>*, int, int64_t, const int*, int,
                                               hipStream_t) const;
template int BlockPrecond::apply_multi<float>(const cx<float>*, cx<float>*, int, int64_t, const int*, int,
                                              hipStream_t) const;

}  // namespace celes

// Vector kernels of the Krylov solver (complex vectors of length n, stored as
// interleaved (re, im)).  Reductions are two-stage with a fixed block count and
// a fixed summation order, so results are bit-reproducible run to run.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "vec_kernels.hpp"

namespace celes {

constexpr int VB = 256;        // threads per block
constexpr int VRED = 512;      // blocks of the first reduction stage

// partial[b][c] = sum_{i in block b's slice} conj(V[c][i]) w[i], c < m
template <typename T>
__global__ void __launch_bounds__(VB) zdots_stage1(const cx<T>* __restrict__ V, int64_t ldv, int m,
                                                   const cx<T>* __restrict__ w, int64_t n,
                                                   cx<double>* __restrict__ partial) {
    __shared__ double sre[VB], sim[VB];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    for (int c = 0; c < m; ++c) {
        double re = 0, im = 0;
        const cx<T>* v = V + (int64_t)c * ldv;
        for (int64_t i = lo + threadIdx.x; i < hi; i += VB) {
            const cx<T> a = v[i], b = w[i];
            re += (double)a.re * b.re + (double)a.im * b.im;
            im += (double)a.re * b.im - (double)a.im * b.re;
        }
        sre[threadIdx.x] = re;
        sim[threadIdx.x] = im;
        __syncthreads();
        for (int s = VB / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) {
                sre[threadIdx.x] += sre[threadIdx.x + s];
                sim[threadIdx.x] += sim[threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * m + c] = {sre[0], sim[0]};
        __syncthreads();
    }
}

__global__ void __launch_bounds__(VB) zdots_stage2(const cx<double>* __restrict__ partial, int nb, int m,
                                                   cx<double>* __restrict__ out) {
    const int c = blockIdx.x;
    __shared__ double sre[VB], sim[VB];
    double re = 0, im = 0;
    for (int b = threadIdx.x; b < nb; b += VB) {
        re += partial[(int64_t)b * m + c].re;
        im += partial[(int64_t)b * m + c].im;
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int s = VB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sre[threadIdx.x] += sre[threadIdx.x + s];
            sim[threadIdx.x] += sim[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = {sre[0], sim[0]};
}

// w[i] -= sum_c V[c][i] h[c]
template <typename T>
__global__ void __launch_bounds__(VB) zgemv_sub(const cx<T>* __restrict__ V, int64_t ldv, int m,
                                                const cx<double>* __restrict__ h, cx<T>* __restrict__ w,
                                                int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x;
    if (i >= n) return;
    double re = w[i].re, im = w[i].im;
    for (int c = 0; c < m; ++c) {
        const cx<T> v = V[(int64_t)c * ldv + i];
        const cx<double> hc = h[c];
        re -= (double)v.re * hc.re - (double)v.im * hc.im;
        im -= (double)v.re * hc.im + (double)v.im * hc.re;
    }
    w[i] = {(T)re, (T)im};
}

// x[i] += sum_c V[c][i] y[c]
template <typename T>
__global__ void __launch_bounds__(VB) zgemv_add(const cx<T>* __restrict__ V, int64_t ldv, int m,
                                                const cx<double>* __restrict__ y, cx<T>* __restrict__ x,
                                                int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x;
    if (i >= n) return;
    double re = x[i].re, im = x[i].im;
    for (int c = 0; c < m; ++c) {
        const cx<T> v = V[(int64_t)c * ldv + i];
        const cx<double> yc = y[c];
        re += (double)v.re * yc.re - (double)v.im * yc.im;
        im += (double)v.re * yc.im + (double)v.im * yc.re;
    }
    x[i] = {(T)re, (T)im};
}

// y = alpha * x  (alpha real)
template <typename T>
__global__ void zscal_copy(const cx<T>* __restrict__ x, double alpha, cx<T>* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x;
    if (i >= n) return;
    y[i] = {(T)(alpha * x[i].re), (T)(alpha * x[i].im)};
}

// z = x - y
template <typename T>
__global__ void zsub(const cx<T>* __restrict__ x, const cx<T>* __restrict__ y, cx<T>* __restrict__ z, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x;
    if (i >= n) return;
    z[i] = {x[i].re - y[i].re, x[i].im - y[i].im};
}

// out = a x + b y + c z (complex scalars; y and z may be null when b, c are
// unused).  Element-wise, so out may alias any input.
template <typename T>
__global__ void zcomb3(const cx<T>* x, cx<T> a, const cx<T>* y, cx<T> b, const cx<T>* z, cx<T> c, cx<T>* out,
                       int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x;
    if (i >= n) return;
    cx<T> acc = cmul(a, x[i]);
    if (y) cfma(acc, b, y[i]);
    if (z) cfma(acc, c, z[i]);
    out[i] = acc;
}

// precision conversion
template <typename A, typename B>
__global__ void zconvert(const cx<A>* __restrict__ x, cx<B>* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x;
    if (i >= n) return;
    y[i] = {(B)x[i].re, (B)x[i].im};
}

// x64 += (double) d32
__global__ void zacc_from32(const cx<float>* __restrict__ d, cx<double>* __restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x;
    if (i >= n) return;
    x[i].re += (double)d[i].re;
    x[i].im += (double)d[i].im;
}

static inline dim3 grid1(int64_t n) { return dim3((unsigned)((n + VB - 1) / VB)); }

template <typename T>
void vec_dots(const cx<T>* V, int64_t ldv, int m, const cx<T>* w, int64_t n, cx<double>* partial,
              cx<double>* out, hipStream_t s) {
    int nb = (int)((n + VB - 1) / VB);
    nb = nb < VRED ? nb : VRED;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(zdots_stage1<T>, dim3(nb), dim3(VB), 0, s, V, ldv, m, w, n, partial);
    hipLaunchKernelGGL(zdots_stage2, dim3(m), dim3(VB), 0, s, partial, nb, m, out);
}
template <typename T>
void vec_gemv_sub(const cx<T>* V, int64_t ldv, int m, const cx<double>* h, cx<T>* w, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(zgemv_sub<T>, grid1(n), dim3(VB), 0, s, V, ldv, m, h, w, n);
}
template <typename T>
void vec_gemv_add(const cx<T>* V, int64_t ldv, int m, const cx<double>* y, cx<T>* x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(zgemv_add<T>, grid1(n), dim3(VB), 0, s, V, ldv, m, y, x, n);
}
template <typename T>
void vec_scale(const cx<T>* x, double alpha, cx<T>* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(zscal_copy<T>, grid1(n), dim3(VB), 0, s, x, alpha, y, n);
}
template <typename T>
void vec_sub(const cx<T>* x, const cx<T>* y, cx<T>* z, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(zsub<T>, grid1(n), dim3(VB), 0, s, x, y, z, n);
}
template <typename T>
void vec_comb3(const cx<T>* x, cx<double> a, const cx<T>* y, cx<double> b, const cx<T>* z, cx<double> c, cx<T>* out,
               int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(zcomb3<T>, grid1(n), dim3(VB), 0, s, x, cx<T>{(T)a.re, (T)a.im}, y, cx<T>{(T)b.re, (T)b.im}, z,
                       cx<T>{(T)c.re, (T)c.im}, out, n);
}
void vec_to32(const cx<double>* x, cx<float>* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((zconvert<double, float>), grid1(n), dim3(VB), 0, s, x, y, n);
}
void vec_to64(const cx<float>* x, cx<double>* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((zconvert<float, double>), grid1(n), dim3(VB), 0, s, x, y, n);
}
void vec_acc32(const cx<float>* d, cx<double>* x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(zacc_from32, grid1(n), dim3(VB), 0, s, d, x, n);
}

#define CELES_VEC_INST(T)                                                                                  \
    template void vec_dots<T>(const cx<T>*, int64_t, int, const cx<T>*, int64_t, cx<double>*, cx<double>*, \
                              hipStream_t);                                                                \
    template void vec_gemv_sub<T>(const cx<T>*, int64_t, int, const cx<double>*, cx<T>*, int64_t,          \
                                  hipStream_t);                                                            \
    template void vec_gemv_add<T>(const cx<T>*, int64_t, int, const cx<double>*, cx<T>*, int64_t,          \
                                  hipStream_t);                                                            \
    template void vec_scale<T>(const cx<T>*, double, cx<T>*, int64_t, hipStream_t);                        \
    template void vec_sub<T>(const cx<T>*, const cx<T>*, cx<T>*, int64_t, hipStream_t);                    \
    template void vec_comb3<T>(const cx<T>*, cx<double>, const cx<T>*, cx<double>, const cx<T>*, cx<double>, \
                               cx<T>*, int64_t, hipStream_t);
CELES_VEC_INST(double)
CELES_VEC_INST(float)

}  // namespace celes

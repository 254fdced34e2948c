#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "device_common.hpp"

namespace celes {
constexpr int VEC_PARTIAL_BLOCKS = 512;
// out[c] = sum_i conj(V[c][i]) w[i], c < m (partial: VEC_PARTIAL_BLOCKS * m scratch)
template <typename T>
void vec_dots(const cx<T>* V, int64_t ldv, int m, const cx<T>* w, int64_t n, cx<double>* partial,
              cx<double>* out, hipStream_t s);
template <typename T>
void vec_gemv_sub(const cx<T>* V, int64_t ldv, int m, const cx<double>* h, cx<T>* w, int64_t n, hipStream_t s);
template <typename T>
void vec_gemv_add(const cx<T>* V, int64_t ldv, int m, const cx<double>* y, cx<T>* x, int64_t n, hipStream_t s);
template <typename T>
void vec_scale(const cx<T>* x, double alpha, cx<T>* y, int64_t n, hipStream_t s);
template <typename T>
void vec_sub(const cx<T>* x, const cx<T>* y, cx<T>* z, int64_t n, hipStream_t s);
// out = a x + b y + c z (y, z may be null; out may alias an input)
template <typename T>
void vec_comb3(const cx<T>* x, cx<double> a, const cx<T>* y, cx<double> b, const cx<T>* z, cx<double> c, cx<T>* out,
               int64_t n, hipStream_t s);
void vec_to32(const cx<double>* x, cx<float>* y, int64_t n, hipStream_t s);
void vec_to64(const cx<float>* x, cx<double>* y, int64_t n, hipStream_t s);
void vec_acc32(const cx<float>* d, cx<double>* x, int64_t n, hipStream_t s);
}  // namespace celes

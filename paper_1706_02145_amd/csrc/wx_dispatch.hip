// Dispatch of the coupling mat-vec: prep (sum/difference form), the per-L
// pass kernels (wx_kernels.hip), and the chunk reduction with the optional
// M = I - T W epilogue (paper, Section 2.2 eq. M).
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "wx_launch.hpp"
#include "wx_mfma.hpp"

namespace celes {

// x [K][N][nmax] (tau blocks) -> xsd [N][K][2][HALF], s = x1 + x2, d = x1 - x2
template <typename T>
__global__ void wx_prep_kernel(const cx<T>* __restrict__ x, cx<T>* __restrict__ xsd, int n, int half, int K) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * half * K) return;
    const int c = (int)(t % half);
    const int64_t ik = t / half;
    const int i = (int)(ik % n), k = (int)(ik / n);
    const cx<T> a = x[((size_t)k * n + i) * 2 * half + c], b = x[((size_t)k * n + i) * 2 * half + half + c];
    cx<T>* o = xsd + ((size_t)i * K + k) * 2 * half;
    o[c] = {a.re + b.re, a.im + b.im};
    o[half + c] = {a.re - b.re, a.im - b.im};
}

// sum partials over chunks, convert to (tau, l, m), optional y = x - T (W x)
template <typename T>
__global__ void wx_finish_kernel(const cx<T>* __restrict__ part, int nchunk, int ldp, int n, int L, int K,
                                 const cx<T>* __restrict__ x, const cx<T>* __restrict__ tq,
                                 cx<T>* __restrict__ y, int epilogue) {
    const int half = L * (L + 2);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * half * K) return;
    const int i = (int)(t % n);          // consecutive lanes: consecutive spheres (coalesced part reads)
    const int64_t ck = t / n;
    const int c = (int)(ck % half), k = (int)(ck / half);
    cx<T> sp = {0, 0}, sm = {0, 0};
    for (int ch = 0; ch < nchunk; ++ch) {
        const size_t base = ((size_t)ch * K + k) * 2 * half;
        const cx<T> a = part[(base + c) * ldp + i];
        const cx<T> b = part[(base + half + c) * ldp + i];
        sp.re += a.re; sp.im += a.im;
        sm.re += b.re; sm.im += b.im;
    }
    cx<T> y1 = {(T)0.5 * (sp.re + sm.re), (T)0.5 * (sp.im + sm.im)};
    cx<T> y2 = {(T)0.5 * (sp.re - sm.re), (T)0.5 * (sp.im - sm.im)};
    const size_t b1 = ((size_t)k * n + i) * 2 * half + c, b2 = b1 + half;
    if (epilogue) {
        // l of the (l, m) index c: l(l+1)+m-1 = c  ->  l = floor(sqrt(c+1))
        int l = (int)sqrtf((float)(c + 1));
        while (l * (l + 2) < c + 1) ++l;
        while ((l - 1) * (l + 1) >= c + 1) --l;
        const cx<T> q1 = tq[((size_t)i * 2 + 0) * L + (l - 1)];
        const cx<T> q2 = tq[((size_t)i * 2 + 1) * L + (l - 1)];
        const cx<T> x1 = x[b1], x2 = x[b2];
        const cx<T> t1 = cmul(q1, y1), t2 = cmul(q2, y2);
        y1 = {x1.re - t1.re, x1.im - t1.im};
        y2 = {x2.re - t2.re, x2.im - t2.im};
    }
    y[b1] = y1;
    y[b2] = y2;
}

int wx_num_groups(int L) {
    switch (L) {
        case 1: return wx_num_groups_L<1>();
        case 2: return wx_num_groups_L<2>();
        case 3: return wx_num_groups_L<3>();
        case 4: return wx_num_groups_L<4>();
        case 5: return wx_num_groups_L<5>();
        case 6: return wx_num_groups_L<6>();
        default: return 1;
    }
}

template <typename T>
int wx_max_kb(int L) {
    switch (L) {
        case 1: return wx_max_kb_L<T, 1>();
        case 2: return wx_max_kb_L<T, 2>();
        case 3: return wx_max_kb_L<T, 3>();
        case 4: return wx_max_kb_L<T, 4>();
        case 5: return wx_max_kb_L<T, 5>();
        case 6: return wx_max_kb_L<T, 6>();
        default: return 1;
    }
}
template int wx_max_kb<double>(int);
template int wx_max_kb<float>(int);

template <typename T>
int wx_batch_run(int L, const WxArgs<T>* args, const int* item_off, const int* nbx, const int* nchunk, int nprob,
                 int* counter, int nblocks, int kb, int hmode, hipStream_t s) {
    switch (L) {
        case 1: wx_batch_run_L<T, 1>(args, item_off, nbx, nchunk, nprob, counter, nblocks, kb, hmode, s); break;
        case 2: wx_batch_run_L<T, 2>(args, item_off, nbx, nchunk, nprob, counter, nblocks, kb, hmode, s); break;
        case 3: wx_batch_run_L<T, 3>(args, item_off, nbx, nchunk, nprob, counter, nblocks, kb, hmode, s); break;
        case 4: wx_batch_run_L<T, 4>(args, item_off, nbx, nchunk, nprob, counter, nblocks, kb, hmode, s); break;
        case 5: wx_batch_run_L<T, 5>(args, item_off, nbx, nchunk, nprob, counter, nblocks, kb, hmode, s); break;
        case 6: wx_batch_run_L<T, 6>(args, item_off, nbx, nchunk, nprob, counter, nblocks, kb, hmode, s); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
template int wx_batch_run<double>(int, const WxArgs<double>*, const int*, const int*, const int*, int, int*, int,
                                  int, int, hipStream_t);
template int wx_batch_run<float>(int, const WxArgs<float>*, const int*, const int*, const int*, int, int*, int, int,
                                 int, hipStream_t);

template <typename T>
int wx_rtr_batch_run(int L, const WxArgs<T>* args, const int* item_off, const int* nbx, const int* nchunk, int nprob,
                     int* counter, int nblocks, int hmode, hipStream_t s) {
    switch (L) {
        case 1: wx_rtr_batch_run_L<T, 1>(args, item_off, nbx, nchunk, nprob, counter, nblocks, hmode, s); break;
        case 2: wx_rtr_batch_run_L<T, 2>(args, item_off, nbx, nchunk, nprob, counter, nblocks, hmode, s); break;
        case 3: wx_rtr_batch_run_L<T, 3>(args, item_off, nbx, nchunk, nprob, counter, nblocks, hmode, s); break;
        case 4: wx_rtr_batch_run_L<T, 4>(args, item_off, nbx, nchunk, nprob, counter, nblocks, hmode, s); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
template int wx_rtr_batch_run<double>(int, const WxArgs<double>*, const int*, const int*, const int*, int, int*, int,
                                      int, hipStream_t);
template int wx_rtr_batch_run<float>(int, const WxArgs<float>*, const int*, const int*, const int*, int, int*, int,
                                     int, hipStream_t);

template <typename T>
int wx_launch(const WxArgs<T>& a, int L, int hmode, int nchunk, const cx<T>* x, const cx<T>* tq,
              cx<T>* y, int epilogue, hipStream_t s, const hipEvent_t* ev, int scheme) {
    const int half = L * (L + 2);
    const int64_t tot = (int64_t)a.n * half * a.nrhs;
    if (L < 1 || L > 6) return -1;
    hipLaunchKernelGGL(wx_prep_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x,
                       const_cast<cx<T>*>(a.xsd), a.n, half, a.nrhs);
    if (ev) hipEventRecord(ev[0], s);
    if (scheme == 1) {
        switch (L) {
            case 1: wx_rtr_run_L<T, 1>(a, hmode, nchunk, s); break;
            case 2: wx_rtr_run_L<T, 2>(a, hmode, nchunk, s); break;
            case 3: wx_rtr_run_L<T, 3>(a, hmode, nchunk, s); break;
            case 4: wx_rtr_run_L<T, 4>(a, hmode, nchunk, s); break;
            case 5: wx_rtr_run_L<T, 5>(a, hmode, nchunk, s); break;
            case 6: wx_rtr_run_L<T, 6>(a, hmode, nchunk, s); break;
        }
    } else {
        switch (L) {
            case 1: wx_run_L<T, 1>(a, hmode, nchunk, s); break;
            case 2: wx_run_L<T, 2>(a, hmode, nchunk, s); break;
            case 3: wx_run_L<T, 3>(a, hmode, nchunk, s); break;
            case 4: wx_run_L<T, 4>(a, hmode, nchunk, s); break;
            case 5: wx_run_L<T, 5>(a, hmode, nchunk, s); break;
            case 6: wx_run_L<T, 6>(a, hmode, nchunk, s); break;
        }
    }
    if (ev) hipEventRecord(ev[1], s);
    hipLaunchKernelGGL(wx_finish_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a.part, nchunk,
                       a.ldp, a.n, L, a.nrhs, x, tq, y, epilogue);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int wx_launch_mfma(const WxMfmaArgs& a, int L, int width, int hmode, int nchunk, const cx<float>* x,
                   const cx<float>* tq, cx<float>* y, int epilogue, hipStream_t s, const hipEvent_t* ev) {
    const int half = L * (L + 2);
    const int64_t tot = (int64_t)a.n * half * a.nrhs;
    const int rc = wx_mfma_launch(a, L, width, hmode, nchunk, s, ev);
    if (rc != 0) return rc;
    hipLaunchKernelGGL(wx_finish_kernel<float>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a.part, nchunk,
                       a.ldp, a.n, L, a.nrhs, x, tq, y, epilogue);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template int wx_launch<double>(const WxArgs<double>&, int, int, int, const cx<double>*, const cx<double>*,
                               cx<double>*, int, hipStream_t, const hipEvent_t*, int);
template int wx_launch<float>(const WxArgs<float>&, int, int, int, const cx<float>*, const cx<float>*,
                              cx<float>*, int, hipStream_t, const hipEvent_t*, int);

}  // namespace celes

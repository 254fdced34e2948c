// Kernels of the batched solver: many independent systems (problem p,
// right-hand side k) of different lengths stored back to back in one flat
// vector.  Every GMRES quantity lives on the device (Hessenberg columns,
// Givens rotations, residual estimates, the current Arnoldi index), so one
// Arnoldi step of all systems is a fixed kernel sequence that can be
// captured once in a hipGraph and replayed.  Reductions are two-stage in a
// fixed order (bit-reproducible).
#include <hip/hip_runtime.h>

#include "batch_kernels.hpp"
#include "device_common.hpp"

namespace celes {

constexpr int BB = 256;

// -------------------------------------------------------------------------
// batched prep / finish of the coupling mat-vec (all problems in one launch)
// -------------------------------------------------------------------------
__device__ __forceinline__ int find_prob(const int64_t* off, int nprob, int64_t t) {
    int lo = 0, hi = nprob;  // off[lo] <= t < off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (off[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// x = V + slot * total (slot = *kstep + kadd, or 0 when kstep == nullptr);
// per problem p: xsd_p[i][k][2 HALF] from x_p[k][i][nmax]
template <typename T>
__global__ void batch_prep(const BatchGeom g, const cx<T>* __restrict__ V, int64_t total, const int* kstep, int kadd,
                           cx<T>* __restrict__ xsd) {
    const int64_t t = (int64_t)blockIdx.x * BB + threadIdx.x;
    const int64_t nh = g.elem_off[g.nprob] / 2;   // half-vector elements over all problems
    if (t >= nh) return;
    const int64_t slot = kstep ? (int64_t)(*kstep + kadd) : 0;
    const cx<T>* x = V + slot * total;
    // element t of the "half" index space: problem p, right-hand side k, sphere i, (l,m) c
    const int p = find_prob(g.half_off, g.nprob, t);
    const int64_t loc = t - g.half_off[p];
    const int half = g.half;
    const int n = g.n[p], K = g.nrhs[p];
    const int c = (int)(loc % half);
    const int64_t ik = loc / half;
    const int i = (int)(ik % n), k = (int)(ik / n);
    const int64_t base = g.elem_off[p];
    const cx<T> a = x[base + ((int64_t)k * n + i) * 2 * half + c];
    const cx<T> b = x[base + ((int64_t)k * n + i) * 2 * half + half + c];
    cx<T>* o = xsd + base + ((int64_t)i * K + k) * 2 * half;
    o[c] = {a.re + b.re, a.im + b.im};
    o[half + c] = {a.re - b.re, a.im - b.im};
}

// y = W x or x - T W x (epilogue), y = V + (*kstep + kadd_out) * total
template <typename T>
__global__ void batch_finish(const BatchGeom g, const cx<T>* __restrict__ part, const cx<T>* __restrict__ V,
                             int64_t total, const int* kstep, int kadd_in, int kadd_out, cx<T>* __restrict__ Yout,
                             int epilogue) {
    const int64_t t = (int64_t)blockIdx.x * BB + threadIdx.x;
    const int64_t nh = g.elem_off[g.nprob] / 2;
    if (t >= nh) return;
    const int64_t sin_ = kstep ? (int64_t)(*kstep + kadd_in) : 0;
    const int64_t sout = kstep ? (int64_t)(*kstep + kadd_out) : 0;
    const cx<T>* x = V + sin_ * total;
    cx<T>* y = Yout + sout * total;
    const int p = find_prob(g.half_off, g.nprob, t);
    const int64_t loc = t - g.half_off[p];
    const int half = g.half, L = g.L;
    const int n = g.n[p], K = g.nrhs[p], nchunk = g.nchunk[p];
    const int i = (int)(loc % n);
    const int64_t ck = loc / n;
    const int c = (int)(ck % half), k = (int)(ck / half);
    const cx<T>* pp = part + g.part_off[p];
    cx<T> sp = {0, 0}, sm = {0, 0};
    for (int ch = 0; ch < nchunk; ++ch) {
        const size_t b = ((size_t)ch * K + k) * 2 * half;
        const cx<T> u = pp[(b + c) * n + i], v = pp[(b + half + c) * n + i];
        sp.re += u.re; sp.im += u.im;
        sm.re += v.re; sm.im += v.im;
    }
    cx<T> y1 = {(T)0.5 * (sp.re + sm.re), (T)0.5 * (sp.im + sm.im)};
    cx<T> y2 = {(T)0.5 * (sp.re - sm.re), (T)0.5 * (sp.im - sm.im)};
    const int64_t b1 = g.elem_off[p] + ((int64_t)k * n + i) * 2 * half + c, b2 = b1 + half;
    if (epilogue) {
        int l = (int)sqrtf((float)(c + 1));
        while (l * (l + 2) < c + 1) ++l;
        while ((l - 1) * (l + 1) >= c + 1) --l;
        const cx<T>* tq = (const cx<T>*)g.tq[p];
        const cx<T> q1 = tq[((size_t)i * 2 + 0) * L + (l - 1)], q2 = tq[((size_t)i * 2 + 1) * L + (l - 1)];
        const cx<T> x1 = x[b1], x2 = x[b2];
        const cx<T> t1 = cmul(q1, y1), t2 = cmul(q2, y2);
        y1 = {x1.re - t1.re, x1.im - t1.im};
        y2 = {x2.re - t2.re, x2.im - t2.im};
    }
    y[b1] = y1;
    y[b2] = y2;
}

__global__ void copy_int(const int* __restrict__ a, int* __restrict__ b, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = a[t];
}

__global__ void zero_int(int* p, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0;
}

// -------------------------------------------------------------------------
// segmented reductions over systems.  Block b of the first stage covers
// [blo[b], bhi[b]) of system bseg[b]; the blocks of system s are
// [sblk[s], sblk[s+1]).
// -------------------------------------------------------------------------
// partial[b][c] = sum conj(V_c) w over block b's range, c = 0..nv-1 with
// nv = *kstep + kadd (or kadd when kstep is null); w = W + wslot * total.
template <typename T>
__global__ void __launch_bounds__(BB) seg_dots1(const SegInfo si, const cx<T>* __restrict__ V, int64_t total,
                                                const cx<T>* __restrict__ Wb, const int* kstep, int kadd, int wadd,
                                                int selfdot, const int* __restrict__ active,
                                                cx<double>* __restrict__ partial, int ldp) {
    __shared__ double sre[BB], sim[BB];
    const int b = blockIdx.x;
    const int s = si.bseg[b];
    const int nv = selfdot ? 1 : (kstep ? *kstep + kadd : kadd);
    const cx<T>* w = Wb + (kstep ? (int64_t)(*kstep + wadd) : (int64_t)wadd) * total;
    const bool on = !active || active[s];
    for (int c = 0; c < nv; ++c) {
        double re = 0, im = 0;
        if (on) {
            const cx<T>* v = selfdot ? w : V + (int64_t)c * total;
            for (int64_t i = si.blo[b] + threadIdx.x; i < si.bhi[b]; i += BB) {
                const cx<T> a = v[i], x = w[i];
                re += (double)a.re * x.re + (double)a.im * x.im;
                im += (double)a.re * x.im - (double)a.im * x.re;
            }
        }
        sre[threadIdx.x] = re;
        sim[threadIdx.x] = im;
        __syncthreads();
        for (int st = BB / 2; st > 0; st >>= 1) {
            if (threadIdx.x < st) {
                sre[threadIdx.x] += sre[threadIdx.x + st];
                sim[threadIdx.x] += sim[threadIdx.x + st];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(int64_t)b * ldp + c] = {sre[0], sim[0]};
        __syncthreads();
    }
}

// out[s][c] = sum of partial[b][c] over the blocks of system s
__global__ void seg_dots2(const SegInfo si, const cx<double>* __restrict__ partial, int ldp, const int* kstep,
                          int kadd, int selfdot, cx<double>* __restrict__ out, int ldo) {
    const int s = blockIdx.x;
    const int nv = selfdot ? 1 : (kstep ? *kstep + kadd : kadd);
    for (int c = threadIdx.x; c < nv; c += blockDim.x) {
        double re = 0, im = 0;
        for (int b = si.sblk[s]; b < si.sblk[s + 1]; ++b) {
            re += partial[(int64_t)b * ldp + c].re;
            im += partial[(int64_t)b * ldp + c].im;
        }
        out[(int64_t)s * ldo + c] = {re, im};
    }
}

// w[i] -= sum_c V_c[i] h[s][c] (sign = -1) or x[i] += sum_c V_c[i] y[s][c]
// (sign = +1) over the block's range; number of vectors per system from
// cnt[s] if given, else *kstep + kadd
template <typename T>
__global__ void __launch_bounds__(BB) seg_gemv(const SegInfo si, const cx<T>* __restrict__ V, int64_t total,
                                               const cx<double>* __restrict__ h, int ldh, const int* kstep, int kadd,
                                               const int* __restrict__ cnt, const int* __restrict__ active,
                                               cx<T>* __restrict__ Wb, int wadd, double sign) {
    const int b = blockIdx.y;
    const int s = si.bseg[b];
    if (active && !active[s]) return;
    const int nv = cnt ? cnt[s] : (kstep ? *kstep + kadd : kadd);
    cx<T>* w = Wb + (kstep ? (int64_t)(*kstep + wadd) : (int64_t)wadd) * total;
    const int64_t i = si.blo[b] + (int64_t)blockIdx.x * BB + threadIdx.x;
    if (i >= si.bhi[b]) return;
    double re = w[i].re, im = w[i].im;
    for (int c = 0; c < nv; ++c) {
        const cx<T> v = V[(int64_t)c * total + i];
        const cx<double> hc = h[(int64_t)s * ldh + c];
        re += sign * ((double)v.re * hc.re - (double)v.im * hc.im);
        im += sign * ((double)v.re * hc.im + (double)v.im * hc.re);
    }
    w[i] = {(T)re, (T)im};
}

// one Arnoldi step's Hessenberg update for every active system (one thread
// per system): H[:,k] = h1 + h2, H[k+1,k] = ||w||, previous rotations,
// new rotation G = [[conj(c), conj(s)], [-s, c]] with c = a/r, s = b/r,
// residual estimate |g[k+1]| / ||rhs||; scale[s] = 1/||w||.
__global__ void gmres_givens(GmresState st, const int* kstep, double tol) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= st.nsys || !st.active[s]) return;
    const int k = *kstep, m = st.m;
    cx<double>* H = st.H + (int64_t)s * (m + 1) * m;   // H[i*m + k]
    const cx<double>* h1 = st.h1 + (int64_t)s * (m + 1);
    const cx<double>* h2 = st.h2 + (int64_t)s * (m + 1);
    const double hn = sqrt(fmax(0.0, st.hn[(int64_t)s * (m + 1)].re));
    for (int i = 0; i <= k; ++i) H[i * m + k] = {h1[i].re + h2[i].re, h1[i].im + h2[i].im};
    H[(k + 1) * m + k] = {hn, 0.0};
    cx<double>* cs = st.cs + (int64_t)s * m;
    cx<double>* sn = st.sn + (int64_t)s * m;
    cx<double>* g = st.g + (int64_t)s * (m + 1);
    for (int i = 0; i < k; ++i) {
        const cx<double> a = H[i * m + k], b = H[(i + 1) * m + k];
        const cx<double> c = cs[i], sv = sn[i];
        // conj(c) a + conj(s) b ; -s a + c b
        H[i * m + k] = {c.re * a.re + c.im * a.im + sv.re * b.re + sv.im * b.im,
                        c.re * a.im - c.im * a.re + sv.re * b.im - sv.im * b.re};
        H[(i + 1) * m + k] = {-(sv.re * a.re - sv.im * a.im) + (c.re * b.re - c.im * b.im),
                              -(sv.re * a.im + sv.im * a.re) + (c.re * b.im + c.im * b.re)};
    }
    const cx<double> a = H[k * m + k], b = H[(k + 1) * m + k];
    const double r = sqrt(a.re * a.re + a.im * a.im + b.re * b.re + b.im * b.im);
    cx<double> c = {1.0, 0.0}, sv = {0.0, 0.0};
    if (r > 0) {
        c = {a.re / r, a.im / r};
        sv = {b.re / r, b.im / r};
    }
    cs[k] = c;
    sn[k] = sv;
    H[k * m + k] = {r, 0.0};
    H[(k + 1) * m + k] = {0.0, 0.0};
    const cx<double> gk = g[k];
    g[k + 1] = {-(sv.re * gk.re - sv.im * gk.im), -(sv.re * gk.im + sv.im * gk.re)};
    g[k] = {c.re * gk.re + c.im * gk.im, c.re * gk.im - c.im * gk.re};
    const double est = sqrt(g[k + 1].re * g[k + 1].re + g[k + 1].im * g[k + 1].im) / st.bnorm[s];
    st.est[s] = est;
    st.used[s] = k + 1;
    st.iters[s] += 1;
    st.scale[s] = hn > 0 ? 1.0 / hn : 0.0;
    if (!(est > tol) || hn == 0.0 || k + 1 >= m) st.active[s] = 0;
}

// V_{k+1} *= scale[s] on active-at-step systems (inactive ones get scale 0
// only if they stopped with hn = 0; harmless)
template <typename T>
__global__ void seg_scale(const SegInfo si, cx<T>* __restrict__ V, int64_t total, const int* kstep, int kadd,
                          const double* __restrict__ scale) {
    const int b = blockIdx.y;
    const int s = si.bseg[b];
    cx<T>* w = V + (int64_t)(*kstep + kadd) * total;
    const int64_t i = si.blo[b] + (int64_t)blockIdx.x * BB + threadIdx.x;
    if (i >= si.bhi[b]) return;
    const double f = scale[s];
    w[i] = {(T)(f * w[i].re), (T)(f * w[i].im)};
}

__global__ void incr_int(int* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p += 1;
}

// y[s] = H^{-1} g for the used[s] leading columns (back substitution)
__global__ void gmres_backsolve(GmresState st) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= st.nsys) return;
    const int m = st.m, u = st.used[s];
    const cx<double>* H = st.H + (int64_t)s * (m + 1) * m;
    const cx<double>* g = st.g + (int64_t)s * (m + 1);
    cx<double>* y = st.y + (int64_t)s * (m + 1);
    for (int i = u - 1; i >= 0; --i) {
        double re = g[i].re, im = g[i].im;
        for (int j = i + 1; j < u; ++j) {
            const cx<double> hij = H[i * m + j], yj = y[j];
            re -= hij.re * yj.re - hij.im * yj.im;
            im -= hij.re * yj.im + hij.im * yj.re;
        }
        const cx<double> d = H[i * m + i];
        const double den = d.re * d.re + d.im * d.im;
        y[i] = den > 0 ? cx<double>{(re * d.re + im * d.im) / den, (im * d.re - re * d.im) / den}
                       : cx<double>{0.0, 0.0};
    }
}

// start of a cycle: beta[s] = sqrt(selfdot), V_0 = r / beta, g = (beta, 0, ...)
__global__ void gmres_cycle_start(GmresState st, double tol) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= st.nsys) return;
    const double beta = sqrt(fmax(0.0, st.hn[(int64_t)s * (st.m + 1)].re));
    cx<double>* g = st.g + (int64_t)s * (st.m + 1);
    for (int i = 0; i <= st.m; ++i) g[i] = {0.0, 0.0};
    g[0] = {beta, 0.0};
    st.used[s] = 0;
    st.est[s] = beta / st.bnorm[s];
    st.scale[s] = beta > 0 ? 1.0 / beta : 0.0;
    st.active[s] = st.est[s] > tol && st.enabled[s] ? 1 : 0;
}

template <typename T>
__global__ void seg_copy_scaled(const SegInfo si, const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
                                const double* __restrict__ scale) {
    const int b = blockIdx.y;
    const int s = si.bseg[b];
    const int64_t i = si.blo[b] + (int64_t)blockIdx.x * BB + threadIdx.x;
    if (i >= si.bhi[b]) return;
    const double f = scale ? scale[s] : 1.0;
    y[i] = {(T)(f * x[i].re), (T)(f * x[i].im)};
}

template <typename A, typename B>
__global__ void flat_convert(const cx<A>* __restrict__ x, cx<B>* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * BB + threadIdx.x;
    if (i < n) y[i] = {(B)x[i].re, (B)x[i].im};
}

template <typename T>
__global__ void flat_sub(const cx<T>* __restrict__ a, const cx<T>* __restrict__ b, cx<T>* __restrict__ c, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * BB + threadIdx.x;
    if (i < n) c[i] = {a[i].re - b[i].re, a[i].im - b[i].im};
}

template <typename T>
__global__ void flat_add(const cx<T>* __restrict__ a, const cx<T>* __restrict__ b, cx<T>* __restrict__ c, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * BB + threadIdx.x;
    if (i < n) c[i] = {a[i].re + b[i].re, a[i].im + b[i].im};
}

__global__ void flat_acc32(const cx<float>* __restrict__ d, cx<double>* __restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * BB + threadIdx.x;
    if (i < n) {
        x[i].re += (double)d[i].re;
        x[i].im += (double)d[i].im;
    }
}

template <typename T>
__global__ void flat_zero(cx<T>* __restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * BB + threadIdx.x;
    if (i < n) x[i] = {(T)0, (T)0};
}

// -------------------------------------------------------------------------
// host wrappers
// -------------------------------------------------------------------------
static inline unsigned nblk(int64_t n) { return (unsigned)((n + BB - 1) / BB); }

template <typename T>
void bk_prep(const BatchGeom& g, const cx<T>* V, int64_t total, const int* kstep, int kadd, cx<T>* xsd,
             hipStream_t s) {
    const int64_t nh = g.host_elems / 2;
    hipLaunchKernelGGL(batch_prep<T>, dim3(nblk(nh)), dim3(BB), 0, s, g, V, total, kstep, kadd, xsd);
}
template <typename T>
void bk_finish(const BatchGeom& g, const cx<T>* part, const cx<T>* V, int64_t total, const int* kstep, int kin,
               int kout, cx<T>* Y, int epilogue, hipStream_t s) {
    const int64_t nh = g.host_elems / 2;
    hipLaunchKernelGGL(batch_finish<T>, dim3(nblk(nh)), dim3(BB), 0, s, g, part, V, total, kstep, kin, kout, Y,
                       epilogue);
}
void bk_zero_int(int* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}
void bk_copy_int(const int* a, int* b, int n, hipStream_t s) {
    hipLaunchKernelGGL(copy_int, dim3((n + 255) / 256), dim3(256), 0, s, a, b, n);
}
void bk_incr(int* p, hipStream_t s) { hipLaunchKernelGGL(incr_int, dim3(1), dim3(64), 0, s, p); }

template <typename T>
void bk_dots(const SegInfo& si, const cx<T>* V, int64_t total, const cx<T>* W, const int* kstep, int kadd, int wadd,
             int selfdot, const int* active, cx<double>* partial, int ldp, cx<double>* out, int ldo, hipStream_t s) {
    hipLaunchKernelGGL(seg_dots1<T>, dim3(si.nblocks), dim3(BB), 0, s, si, V, total, W, kstep, kadd, wadd, selfdot,
                       active, partial, ldp);
    hipLaunchKernelGGL(seg_dots2, dim3(si.nsys), dim3(64), 0, s, si, partial, ldp, kstep, kadd, selfdot, out, ldo);
}
template <typename T>
void bk_gemv(const SegInfo& si, const cx<T>* V, int64_t total, const cx<double>* h, int ldh, const int* kstep,
             int kadd, const int* cnt, const int* active, cx<T>* W, int wadd, double sign, hipStream_t s) {
    dim3 grid((unsigned)((si.maxblk + BB - 1) / BB), (unsigned)si.nblocks);
    hipLaunchKernelGGL(seg_gemv<T>, grid, dim3(BB), 0, s, si, V, total, h, ldh, kstep, kadd, cnt, active, W, wadd,
                       sign);
}
void bk_givens(const GmresState& st, const int* kstep, double tol, hipStream_t s) {
    hipLaunchKernelGGL(gmres_givens, dim3((st.nsys + 63) / 64), dim3(64), 0, s, st, kstep, tol);
}
template <typename T>
void bk_scale(const SegInfo& si, cx<T>* V, int64_t total, const int* kstep, int kadd, const double* scale,
              hipStream_t s) {
    dim3 grid((unsigned)((si.maxblk + BB - 1) / BB), (unsigned)si.nblocks);
    hipLaunchKernelGGL(seg_scale<T>, grid, dim3(BB), 0, s, si, V, total, kstep, kadd, scale);
}
void bk_backsolve(const GmresState& st, hipStream_t s) {
    hipLaunchKernelGGL(gmres_backsolve, dim3((st.nsys + 63) / 64), dim3(64), 0, s, st);
}
void bk_cycle_start(const GmresState& st, double tol, hipStream_t s) {
    hipLaunchKernelGGL(gmres_cycle_start, dim3((st.nsys + 63) / 64), dim3(64), 0, s, st, tol);
}
template <typename T>
void bk_copy_scaled(const SegInfo& si, const cx<T>* x, cx<T>* y, const double* scale, hipStream_t s) {
    dim3 grid((unsigned)((si.maxblk + BB - 1) / BB), (unsigned)si.nblocks);
    hipLaunchKernelGGL(seg_copy_scaled<T>, grid, dim3(BB), 0, s, si, x, y, scale);
}
void bk_to32(const cx<double>* x, cx<float>* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((flat_convert<double, float>), dim3(nblk(n)), dim3(BB), 0, s, x, y, n);
}
template <typename T>
void bk_sub(const cx<T>* a, const cx<T>* b, cx<T>* c, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(flat_sub<T>, dim3(nblk(n)), dim3(BB), 0, s, a, b, c, n);
}
template <typename T>
void bk_add(const cx<T>* a, const cx<T>* b, cx<T>* c, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(flat_add<T>, dim3(nblk(n)), dim3(BB), 0, s, a, b, c, n);
}
void bk_acc32(const cx<float>* d, cx<double>* x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(flat_acc32, dim3(nblk(n)), dim3(BB), 0, s, d, x, n);
}
template <typename T>
void bk_zero(cx<T>* x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(flat_zero<T>, dim3(nblk(n)), dim3(BB), 0, s, x, n);
}

// b[slot sb] = a[slot sa] with slot = (*k if k else 0) + offset, slots of
// `total` elements (reads the device-side Arnoldi step index at run time)
template <typename T>
__global__ void slot_copy(const cx<T>* __restrict__ a, const int* ka, int oa, cx<T>* __restrict__ b, const int* kb,
                          int ob, int64_t total) {
    const int64_t t = (int64_t)blockIdx.x * BB + threadIdx.x;
    if (t >= total) return;
    const int64_t sa = (int64_t)((ka ? *ka : 0) + oa) * total, sb = (int64_t)((kb ? *kb : 0) + ob) * total;
    b[sb + t] = a[sa + t];
}
template <typename T>
void bk_slot_copy(const cx<T>* a, const int* ka, int oa, cx<T>* b, const int* kb, int ob, int64_t total,
                  hipStream_t s) {
    hipLaunchKernelGGL(slot_copy<T>, dim3(nblk(total)), dim3(BB), 0, s, a, ka, oa, b, kb, ob, total);
}

#define CELES_BK_INST(T)                                                                                        \
    template void bk_prep<T>(const BatchGeom&, const cx<T>*, int64_t, const int*, int, cx<T>*, hipStream_t);    \
    template void bk_finish<T>(const BatchGeom&, const cx<T>*, const cx<T>*, int64_t, const int*, int, int,     \
                               cx<T>*, int, hipStream_t);                                                       \
    template void bk_dots<T>(const SegInfo&, const cx<T>*, int64_t, const cx<T>*, const int*, int, int, int,    \
                             const int*, cx<double>*, int, cx<double>*, int, hipStream_t);                      \
    template void bk_gemv<T>(const SegInfo&, const cx<T>*, int64_t, const cx<double>*, int, const int*, int,    \
                             const int*, const int*, cx<T>*, int, double, hipStream_t);                         \
    template void bk_scale<T>(const SegInfo&, cx<T>*, int64_t, const int*, int, const double*, hipStream_t);    \
    template void bk_copy_scaled<T>(const SegInfo&, const cx<T>*, cx<T>*, const double*, hipStream_t);          \
    template void bk_sub<T>(const cx<T>*, const cx<T>*, cx<T>*, int64_t, hipStream_t);                          \
    template void bk_add<T>(const cx<T>*, const cx<T>*, cx<T>*, int64_t, hipStream_t);                          \
    template void bk_zero<T>(cx<T>*, int64_t, hipStream_t);                                                    \
    template void bk_slot_copy<T>(const cx<T>*, const int*, int, cx<T>*, const int*, int, int64_t, hipStream_t);
CELES_BK_INST(double)
CELES_BK_INST(float)

}  // namespace celes

// Argument block and launcher of the on-the-fly coupling mat-vec.
#pragma once
#include <hip/hip_runtime.h>
#include "device_common.hpp"

namespace celes {

template <typename T>
struct LutView {
    const cx<T>* coef;   // [n_int][2][4]: Horner coefficients in t of h_0 and h_1
    double d_lo;
    double inv_dr;
    double inv_k;        // 1 / k (orders >= 2 come from the recurrence in 1/(k d))
    int n_int;
};

template <typename T>
struct WxArgs {
    const double* px;    // sphere centres, SoA, FP64
    const double* py;
    const double* pz;
    const cx<T>* xsd;    // [N][nrhs][2][HALF] source sums/differences (scratch, written by prep)
    const T* coef;       // a5 / b5im table in kernel enumeration order
    cx<T>* part;         // [nchunk][nrhs][2 HALF][ldp] partial sums
    LutView<T> lut;
    double k;            // background wavenumber
    int n;               // number of spheres
    int chunk_len;       // sources per chunk
    int ldp;             // leading dimension of part (>= n)
    int nrhs;            // right-hand sides in xsd / part
    int kb;              // right-hand sides per kernel block (1, 2 or 4; divides nrhs)
    const int* active;   // batch only: per-system flags; items whose systems are all inactive are skipped
    int sys0;            // batch only: system index of this problem's first right-hand side
};

// per-L pass launcher (defined in wx_kernels.hip, one translation unit per L)
template <typename T, int L>
void wx_run_L(const WxArgs<T>& a, int hmode, int nchunk, hipStream_t s);
// rotation-translation-rotation launcher (defined in wx_rtr.hip, one unit per L):
// grid (receiver tiles of 64, source chunks, 2 passes x right-hand sides)
template <typename T, int L>
void wx_rtr_run_L(const WxArgs<T>& a, int hmode, int nchunk, hipStream_t s);
constexpr int WX_RTR_BLOCK_SIZE = 64;   // receivers per block of the rotation kernel
// number of pass groups (third grid dimension) of cut-off L
template <int L>
int wx_num_groups_L();
int wx_num_groups(int L);
// persistent multi-problem launcher (one launch, all problems' work items)
template <typename T, int L>
void wx_batch_run_L(const WxArgs<T>* args, const int* item_off, const int* nbx, const int* nchunk, int nprob,
                    int* counter, int nblocks, int kb, int hmode, hipStream_t s);
template <typename T>
int wx_batch_run(int L, const WxArgs<T>* args, const int* item_off, const int* nbx, const int* nchunk, int nprob,
                 int* counter, int nblocks, int kb, int hmode, hipStream_t s);
// persistent multi-problem launcher of the rotation scheme (defined in
// wx_rtr.hip): work items (problem, receiver tile of 64, source chunk,
// pass x right-hand side), compiled for L <= 4 like the direct one
template <typename T, int L>
void wx_rtr_batch_run_L(const WxArgs<T>* args, const int* item_off, const int* nbx, const int* nchunk, int nprob,
                        int* counter, int nblocks, int hmode, hipStream_t s);
template <typename T>
int wx_rtr_batch_run(int L, const WxArgs<T>* args, const int* item_off, const int* nbx, const int* nchunk, int nprob,
                     int* counter, int nblocks, int hmode, hipStream_t s);
// largest compiled right-hand-side block of cut-off L
template <typename T, int L>
int wx_max_kb_L();
template <typename T>
int wx_max_kb(int L);

constexpr int WX_BLOCK_SIZE = 256;  // receivers per block
constexpr int WX_TILE_SIZE = 16;    // sources per LDS tile

// y = W x (epilogue = 0) or y = x - T (W x) (epilogue = 1) for a.nrhs
// right-hand sides; x, y: [nrhs][N][nmax]; tq: [N][2][L] Mie coefficients.
// ev[0], ev[1] (if ev is given) are recorded on s right before and after the
// coupling kernel.  Returns 0 on success.
// scheme 0: direct block evaluation (wx_fused_kernel); 1: rotation,
// translation along z, rotation back (wx_rtr_kernel; a.kb must be 1)
template <typename T>
int wx_launch(const WxArgs<T>& a, int L, int hmode, int nchunk, const cx<T>* x, const cx<T>* tq,
              cx<T>* y, int epilogue, hipStream_t s, const hipEvent_t* ev = nullptr, int scheme = 0);

}  // namespace celes

// Interfaces of the batched-solver kernels (batch_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.hpp"

namespace celes {

// geometry of a batch of problems in one flat coefficient vector; every
// pointer is a device pointer
struct BatchGeom {
    const int64_t* elem_off;   // [nprob+1] start of problem p's [K_p][N_p][nmax] block
    const int64_t* half_off;   // [nprob+1] elem_off / 2
    const int* n;              // [nprob] spheres
    const int* nrhs;           // [nprob] right-hand sides
    const int* nchunk;         // [nprob] source chunks of the mat-vec
    const int64_t* part_off;   // [nprob] offset of problem p's partial sums
    const void* const* tq;     // [nprob] Mie coefficients [N][2][L] (precision of the kernel)
    int nprob, half, L;
    int64_t host_elems;        // total elements (host copy, for launch sizes)
};

// first-stage reduction blocks: block b covers [blo[b], bhi[b]) of system bseg[b]
struct SegInfo {
    int nsys, nblocks;
    int64_t maxblk;            // longest block range
    const int* bseg;
    const int64_t* blo;
    const int64_t* bhi;
    const int* sblk;           // [nsys+1] blocks of system s
};

// device-resident GMRES state of every system (restart length m)
struct GmresState {
    int nsys, m;
    cx<double>* H;             // [nsys][(m+1) m]
    cx<double>* cs;            // [nsys][m]
    cx<double>* sn;
    cx<double>* g;             // [nsys][m+1]
    cx<double>* y;             // [nsys][m+1]
    cx<double>* h1;            // [nsys][m+1] first Gram-Schmidt pass
    cx<double>* h2;            // [nsys][m+1] second pass
    cx<double>* hn;            // [nsys][m+1] squared norms (element 0)
    double* bnorm;             // [nsys] norm of the right-hand side of the current solve
    double* est;               // [nsys] implicit relative residual estimate
    double* scale;             // [nsys]
    int* active;               // [nsys] still iterating in this cycle
    int* enabled;              // [nsys] taking part in this solve
    int* used;                 // [nsys] Arnoldi steps of this cycle
    int* iters;                // [nsys] total Arnoldi steps
};

template <typename T>
void bk_prep(const BatchGeom& g, const cx<T>* V, int64_t total, const int* kstep, int kadd, cx<T>* xsd,
             hipStream_t s);
template <typename T>
void bk_finish(const BatchGeom& g, const cx<T>* part, const cx<T>* V, int64_t total, const int* kstep, int kin,
               int kout, cx<T>* Y, int epilogue, hipStream_t s);
void bk_zero_int(int* p, int n, hipStream_t s);
void bk_incr(int* p, hipStream_t s);
void bk_copy_int(const int* a, int* b, int n, hipStream_t s);
template <typename T>
void bk_dots(const SegInfo& si, const cx<T>* V, int64_t total, const cx<T>* W, const int* kstep, int kadd, int wadd,
             int selfdot, const int* active, cx<double>* partial, int ldp, cx<double>* out, int ldo, hipStream_t s);
template <typename T>
void bk_gemv(const SegInfo& si, const cx<T>* V, int64_t total, const cx<double>* h, int ldh, const int* kstep,
             int kadd, const int* cnt, const int* active, cx<T>* W, int wadd, double sign, hipStream_t s);
void bk_givens(const GmresState& st, const int* kstep, double tol, hipStream_t s);
template <typename T>
void bk_scale(const SegInfo& si, cx<T>* V, int64_t total, const int* kstep, int kadd, const double* scale,
              hipStream_t s);
void bk_backsolve(const GmresState& st, hipStream_t s);
void bk_cycle_start(const GmresState& st, double tol, hipStream_t s);
template <typename T>
void bk_copy_scaled(const SegInfo& si, const cx<T>* x, cx<T>* y, const double* scale, hipStream_t s);
void bk_to32(const cx<double>* x, cx<float>* y, int64_t n, hipStream_t s);
template <typename T>
void bk_sub(const cx<T>* a, const cx<T>* b, cx<T>* c, int64_t n, hipStream_t s);
template <typename T>
void bk_add(const cx<T>* a, const cx<T>* b, cx<T>* c, int64_t n, hipStream_t s);
void bk_acc32(const cx<float>* d, cx<double>* x, int64_t n, hipStream_t s);
template <typename T>
void bk_zero(cx<T>* x, int64_t n, hipStream_t s);
// b[slot (*kb or 0) + ob] = a[slot (*ka or 0) + oa], slots of `total` elements
template <typename T>
void bk_slot_copy(const cx<T>* a, const int* ka, int oa, cx<T>* b, const int* kb, int ob, int64_t total,
                  hipStream_t s);

}  // namespace celes

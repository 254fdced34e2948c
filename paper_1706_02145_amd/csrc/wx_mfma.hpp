// Multi-right-hand-side coupling mat-vec on the matrix cores (complex64,
// lmax <= 4): per sphere pair the translation block is built once on the
// VALU and applied to 16, 32 or 64 right-hand sides with MFMA.
#pragma once
#include <hip/hip_runtime.h>
#include <vector>
#include "device_common.hpp"
#include "wx_launch.hpp"

namespace celes {

constexpr int WXM_MAX_L = 4;
constexpr int WXM_REC = 16;   // floats per block-entry record
// row stride of a pair's H_p^mu table (p = 0..2L).  A record reads a fixed
// number of terms from its first H offset; the terms past a row carry zero
// coefficients and land on the next row, the next source's table or a zeroed
// tail of at most 2L entries, all finite.
constexpr int wxm_h_stride(int L) { return 2 * L + 1; }

struct WxMfmaArgs {
    const double* px;          // sphere centres, SoA, FP64
    const double* py;
    const double* pz;
    const cx<float>* x;        // [nrhs][N][nmax] source vectors (tau blocks), at x + slot * slot_stride
    const int* kstep;          // device slot index (slot = *kstep + kin), or null for slot 0
    int kin;
    int64_t slot_stride;
    const int* active;         // per-system flags (batches): blocks whose systems are all inactive exit, or null
    int sys0;                  // system index of right-hand side 0
    float* xb;                 // [nrhs / width][N][2][R x width] operand-ordered source records (scratch)
    cx<float>* part;           // [nchunk][nrhs][2 HALF][ldp] partial sums (reduced by the finish kernel)
    const float* rec;          // [(HALF^2 + L^2) / 2][WXM_REC] block-entry records (wx_mfma_records)
    LutView<float> lut;
    double k;
    int n;
    int chunk_len;             // sources per chunk
    int ldp;
    int nrhs;                  // right-hand sides in xsd / part (a multiple of the block width)
};

// Host: records of the reduced block entries (receiving n = (l, m), source
// n' = (l', m')), one per entry pair {(m, m'), (-m, -m')}: packed H offsets
// of the first A and B terms, the phase index and the mirror flag; the LDS
// offsets of the entry's four real-form operand positions and of its
// mirror's; then the a5 and b5 coefficients of the p terms (zero-padded to
// L + 1 and L terms).
void wx_mfma_records(int L, std::vector<float>* rec);

// floats of the operand-ordered source records for N spheres, K right-hand sides
size_t wx_mfma_xb_floats(int L, int64_t N, int K);

// right-hand-side block width for K right-hand sides (64, 32 or 16), or 0
// where the VALU kernel is faster or the path does not apply (L > 4, K not
// a multiple of 16); any = true returns every applicable width
int wx_mfma_block(int L, int K, bool any = false);

// Prep (x -> operand-ordered xb) and the kernel on grid (ceil(N / 4),
// nchunk, nrhs / width), with ev[0], ev[1] (if given) recorded around the
// kernel; returns 0, -1 (not applicable) or -2 (launch error)
int wx_mfma_launch(const WxMfmaArgs& a, int L, int width, int hmode, int nchunk, hipStream_t s,
                   const hipEvent_t* ev = nullptr);

// wx_mfma_launch, then the chunk reduction with the optional
// y = x - T (W x) epilogue; x, y: [nrhs][N][nmax] complex64
int wx_launch_mfma(const WxMfmaArgs& a, int L, int width, int hmode, int nchunk, const cx<float>* x,
                   const cx<float>* tq, cx<float>* y, int epilogue, hipStream_t s, const hipEvent_t* ev = nullptr);

}  // namespace celes

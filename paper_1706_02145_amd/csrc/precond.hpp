// Block-diagonal preconditioner (paper, Section 3.2.1): the spheres are
// partitioned into cuboids, the diagonal blocks M_j = I - T W_jj are
// assembled on the device and factorised in FP64, and applying the
// preconditioner multiplies each block of a vector by M_j^{-1}.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "device_common.hpp"
#include "host_math.hpp"

namespace celes {

// error codes returned by BlockPrecond (same values as the C ABI's)
constexpr int CELES_E_OOM_INTERNAL = -7;
constexpr int CELES_E_DEVICE_INTERNAL = -8;

class BlockPrecond {
   public:
    ~BlockPrecond();
    // pos [N][3], tq [N][2][L] (host); lut_dev: FP64 Hankel table (LUT mode)
    int build(int64_t N, int L, const double* pos, double k, const cplx* tq, double edge, int hmode,
              const void* lut_dev, double lut_lo, double lut_dr, int lut_n, std::string* msg);
    // out = P^{-1} in (in, out: [N][nmax] device vectors, must not alias);
    // complex64 vectors use the complex64 copy of the inverses
    template <typename T>
    int apply(const cx<T>* in, cx<T>* out, hipStream_t s) const;
    // out_k = P^{-1} in_k for K right-hand sides k at element stride `stride`
    // (layout [K][N][nmax]): each inverse tile is read once per group of up to
    // 8 right-hand sides; groups whose systems are all inactive
    // (active[sys0 + k] == 0, active may be null) are skipped and their
    // outputs left as they are.  Allocates nothing (graph-capture safe).
    template <typename T>
    int apply_multi(const cx<T>* in, cx<T>* out, int K, int64_t stride, const int* active, int sys0,
                    hipStream_t s) const;

    int num_blocks() const { return (int)offsets_.size() - 1; }
    const std::vector<int64_t>& perm() const { return perm_; }
    const std::vector<int64_t>& offsets() const { return offsets_; }
    double edge() const { return edge_; }
    // device bytes held (the budgeted quantity of precond_bytes)
    double bytes() const { return precond_bytes(N_, L_, offsets_); }

    // bytes a preconditioner over this partition holds on the device: FP64
    // inverses and their complex64 copy, sum_j (N_j nmax)^2 (16 + 8), plus the
    // apply's partial sums, ceil(max_j N_j nmax / 256) N nmax 16
    static double precond_bytes(int64_t N, int L, const std::vector<int64_t>& offsets);

   private:
    double edge_ = 0;
    int L_ = 0, nmax_ = 0;
    int64_t N_ = 0;
    std::vector<int64_t> perm_, offsets_;
    size_t mat_elems_ = 0;
    int max_dim_ = 0;
    int64_t* d_perm_ = nullptr;      // [N] new -> old sphere index
    int64_t* d_boff_ = nullptr;      // [nb+1] sphere offsets
    int64_t* d_moff_ = nullptr;      // [nb] matrix element offsets
    cx<double>* d_inv_ = nullptr;    // block inverses, column-major, concatenated
    cx<float>* d_inv32_ = nullptr;   // complex64 copy (applied to complex64 vectors)
    cx<double>* d_part_ = nullptr;   // [column tiles][N nmax] partial sums of the apply
};

// partition of Section 3.2.1 step 1: cubes of edge `edge` anchored at the
// minimum corner of the centres' bounding box; spheres ordered by (cell linear
// index with x fastest, then y, then z; original index); empty cells skipped.
void partition_cuboids(int64_t N, const double* pos, double edge, std::vector<int64_t>* perm,
                       std::vector<int64_t>* offsets);

// Budgeted cuboid edge (host only): among e_q = 1.02 D 0.92^q, D the largest
// extent of the centres' bounding box, q = 0, 1, ... while e_q >= D / 4096,
// the largest edge whose mean spheres per occupied cuboid is <= target and
// whose precond_bytes is <= cap (cap <= 0: no cap).  Returns 0, or
// CELES_E_OOM_INTERNAL when no candidate fits (msg says why).
int plan_cuboid_edge(int64_t N, const double* pos, int L, double target, double cap, double* edge,
                     std::vector<int64_t>* offsets, std::string* msg);

}  // namespace celes

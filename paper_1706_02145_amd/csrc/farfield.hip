// Far-field sphere sums c_n(d) = sum_i e^{-ik rhat_d . r_i} b^i_n (Appendix D):
// one lane per direction, the spheres' centres and coefficients staged in LDS
// tiles and read as broadcasts, one sincos per (direction, sphere) pair and a
// complex multiply-add per coefficient, FP64 throughout.  Coefficients are
// split into chunks of NC over the grid's y dimension to bound registers.
#include "farfield.hpp"

namespace celes {
namespace {

constexpr int FF_THREADS = 256;  // directions per workgroup
constexpr int FF_TILE = 64;      // spheres per LDS tile

template <int NC>
__global__ void __launch_bounds__(FF_THREADS)
    ff_sums_kernel(const double* __restrict__ px, const double* __restrict__ py, const double* __restrict__ pz,
                   const cx<double>* __restrict__ b, int64_t N, int nmax, const double* __restrict__ dirs,
                   int64_t ndir, double k, cx<double>* __restrict__ c) {
    __shared__ double sp[FF_TILE][3];
    __shared__ cx<double> sb[FF_TILE][NC];
    const int64_t d = (int64_t)blockIdx.x * FF_THREADS + threadIdx.x;
    const int n0 = blockIdx.y * NC;
    const int nc = min(NC, nmax - n0);
    double ux = 0, uy = 0, uz = 0;
    if (d < ndir) {
        ux = -k * dirs[3 * d];
        uy = -k * dirs[3 * d + 1];
        uz = -k * dirs[3 * d + 2];
    }
    cx<double> acc[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) acc[q] = {0.0, 0.0};
    for (int64_t t0 = 0; t0 < N; t0 += FF_TILE) {
        const int nt = (int)min((int64_t)FF_TILE, N - t0);
        __syncthreads();
        for (int q = threadIdx.x; q < nt * NC; q += FF_THREADS) {
            const int s = q / NC, e = q % NC;
            sb[s][e] = e < nc ? b[(t0 + s) * nmax + n0 + e] : cx<double>{0.0, 0.0};
        }
        for (int q = threadIdx.x; q < nt; q += FF_THREADS) {
            sp[q][0] = px[t0 + q];
            sp[q][1] = py[t0 + q];
            sp[q][2] = pz[t0 + q];
        }
        __syncthreads();
        for (int s = 0; s < nt; ++s) {
            double sn, cs;
            sincos(ux * sp[s][0] + uy * sp[s][1] + uz * sp[s][2], &sn, &cs);
            const cx<double> e = {cs, sn};
#pragma unroll
            for (int q = 0; q < NC; ++q) cfma(acc[q], e, sb[s][q]);
        }
    }
    if (d < ndir)
        for (int q = 0; q < nc; ++q) c[d * nmax + n0 + q] = acc[q];
}

template <int NC>
int launch_nc(const double* px, const double* py, const double* pz, const cx<double>* b, int64_t N, int nmax,
              const double* dirs, int64_t ndir, double k, cx<double>* c, hipStream_t s) {
    dim3 grid((unsigned)((ndir + FF_THREADS - 1) / FF_THREADS), (unsigned)((nmax + NC - 1) / NC));
    hipLaunchKernelGGL(ff_sums_kernel<NC>, grid, dim3(FF_THREADS), 0, s, px, py, pz, b, N, nmax, dirs, ndir, k, c);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int ff_sums_launch(const double* px, const double* py, const double* pz, const cx<double>* b, int64_t N, int nmax,
                   const double* dirs, int64_t ndir, double k, cx<double>* c, hipStream_t s) {
    if (ndir <= 0 || N <= 0 || nmax <= 0) return 0;
    // chunk width: the coefficients split into the fewest chunks of at most
    // 24, rounded up to a multiple of 8
    const int nchunk = (nmax + 23) / 24;
    const int per = (nmax + nchunk - 1) / nchunk;
    if (per <= 8) return launch_nc<8>(px, py, pz, b, N, nmax, dirs, ndir, k, c, s);
    if (per <= 16) return launch_nc<16>(px, py, pz, b, N, nmax, dirs, ndir, k, c, s);
    return launch_nc<24>(px, py, pz, b, N, nmax, dirs, ndir, k, c, s);
}

}  // namespace celes

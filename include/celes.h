/*
 * celes.h -- C ABI of the MI355X (gfx950) multi-sphere T-matrix library.
 *
 * Method: Egel, Pattelli, Mazzamuto, Wiersma, Lemmer, "CELES: CUDA-accelerated
 * simulation of electromagnetic scattering by large ensembles of spheres"
 * (JQSRT 2017, arXiv:1706.02145).  Section and equation names below refer to
 * that paper.
 *
 * Conventions shared by every entry point
 *   - Lengths are in one consistent unit (the tests use nanometres); the
 *     wavelength is the vacuum wavelength in that unit.
 *   - Complex numbers are interleaved (re, im) pairs: complex128 = 2 doubles,
 *     complex64 = 2 floats.
 *   - Multi-index n = (tau, l, m), tau in {1,2}, l = 1..lmax, m = -l..l
 *     (Section 2.1).  Linear order (0-based):
 *         n = (tau-1) lmax(lmax+2) + l(l+1) + m - 1,   nmax = 2 lmax (lmax+2).
 *   - Coefficient vectors have layout [K][N][nmax] (right-hand side, sphere,
 *     multi-index), sphere order as given to celes_create.
 *   - Host pointers are owned by the caller and only read or written during
 *     the call.  Device pointers (the *_dev arguments) must be HIP device
 *     memory on the handle's device, owned by the caller.
 *   - Every int-returning call returns CELES_OK (0) or a negative error code;
 *     celes_last_error() then describes the failure.  No C++ exception
 *     crosses this boundary.  Calls on one handle are not thread-safe.
 */
#ifndef CELES_H
#define CELES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CELES_VERSION 100

/* error codes */
#define CELES_OK 0
#define CELES_E_ARG -1          /* invalid argument (null pointer, size < 1, ...) */
#define CELES_E_OVERLAP -2      /* two spheres overlap: |r_i - r_j| <= R_i + R_j   */
#define CELES_E_LUT_RANGE -3    /* a pair distance falls outside the Hankel table */
#define CELES_E_NONFINITE -4    /* NaN or Inf in an input                          */
#define CELES_E_NOCONV -5       /* solver hit maxiter; best iterate returned       */
#define CELES_E_BREAKDOWN -6    /* Krylov breakdown / non-finite iterate           */
#define CELES_E_OOM -7          /* device or host allocation failed                */
#define CELES_E_DEVICE -8       /* HIP runtime error                               */
#define CELES_E_UNSUPPORTED -9  /* e.g. lmax beyond the compiled kernels           */
#define CELES_E_STATE -10       /* call order violated (e.g. solve before incident) */

/* arithmetic of the coupling mat-vec */
#define CELES_FP64 0            /* complex128 everywhere                            */
#define CELES_MIXED 1           /* complex64 inner solve, FP64 residual/refinement  */

/* spherical Hankel evaluation inside the mat-vec */
#define CELES_HANKEL_LUT 0      /* h_0, h_1 from a cubic-Hermite table at spacing lut_dr (Section
                                 * 3.2.2), higher orders by the upward three-term recurrence   */
#define CELES_HANKEL_DIRECT 1   /* h_0, h_1 from sin/cos per pair, then the same recurrence    */

/* evaluation of the translation blocks inside the single-problem mat-vec */
#define CELES_TRANSLATION_DIRECT 0   /* each block entry from the a5/b5 sums (Appendix A.2), O(lmax^4) */
#define CELES_TRANSLATION_ROTATE 1   /* rotate the source into the pair frame, translate along z,
                                      * rotate back (Section 5, Discussion), O(lmax^3) per pair */

/* iterative solver of the master equation (Section 3.2 offers both) */
#define CELES_SOLVER_GMRES 0    /* restarted GMRES (default)                                  */
#define CELES_SOLVER_BICGSTAB 1 /* BiCGSTAB: two mat-vecs per iteration, seven work vectors  */

#define CELES_MAX_LMAX 6

typedef struct celes_handle celes_handle;

typedef struct celes_options {
    int precision;          /* CELES_FP64 or CELES_MIXED                                     */
    int hankel;             /* CELES_HANKEL_LUT or CELES_HANKEL_DIRECT                        */
    double lut_dr;          /* lookup-table spacing in length units (paper: 1 nm)            */
    double tol;             /* GMRES relative residual ||T a_in - M b|| / ||T a_in||          */
    double inner_tol;       /* mixed precision: inner complex64 GMRES tolerance               */
    int restart;            /* GMRES restart length                                           */
    int maxiter;            /* total inner iterations allowed                                 */
    int max_refinements;    /* mixed precision: outer refinement steps allowed                */
    double cuboid_edge;     /* preconditioner built by celes_create: 0 none, > 0 cubes of this
                             * edge, CELES_CUBOID_AUTO the budgeted edge (as
                             * celes_build_preconditioner)                                    */
    int device;             /* HIP device ordinal                                             */
    int verbose;            /* 0 silent, 1 per-restart residuals on stderr                    */
    int solver;             /* CELES_SOLVER_GMRES or CELES_SOLVER_BICGSTAB (single problems;
                             * batches run GMRES only)                                        */
    double target_Nj;       /* automatic cuboid edge (celes_build_preconditioner with
                             * CELES_CUBOID_AUTO): largest edge whose mean number of spheres
                             * per occupied cuboid is <= target_Nj (<= 0: 100)               */
    double mem_cap_bytes;   /* device bytes the preconditioner may hold: FP64 inverses,
                             * their complex64 copy and the apply's partial sums,
                             * sum_j (N_j nmax)^2 (16 + 8) + ceil(max_j N_j nmax / 256) N nmax 16
                             * (<= 0: 90% of the device memory free at build time)            */
    int autotune;           /* 1: the first mat-vec of each precision on a handle times the
                             * candidate source-chunk splits and keeps the fastest             */
    int translation;        /* CELES_TRANSLATION_DIRECT (default) or CELES_TRANSLATION_ROTATE:
                             * how the VALU mat-vec evaluates each pair's block, for single
                             * problems (celes_apply_W/M, celes_solve,
                             * celes_apply_W_noalloc) and for batches (celes_batch_create);
                             * the matrix-core kernel and the preconditioner assembly
                             * always use the direct form                                    */
    int deterministic;      /* 1: bitwise the same results from run to run on one device:
                             * no timing-based choice of the work split (autotune is
                             * ignored; celes_batch_autotune fails with CELES_E_STATE), every
                             * split follows from the sizes alone.  The reductions of the
                             * mat-vec, dots and preconditioner apply are fixed-order in
                             * either mode (no floating-point atomics)                        */
} celes_options;

typedef struct celes_solve_info {
    int status;             /* CELES_OK, CELES_E_NOCONV or CELES_E_BREAKDOWN                   */
    int iterations;         /* inner GMRES iterations or BiCGSTAB iterations (two mat-vecs
                             * each), over all restarts and refinements                        */
    int refinements;        /* outer FP64 refinement steps (mixed) or restarts (FP64)          */
    int matvecs;            /* coupling mat-vecs performed (any precision)                     */
    double rel_residual;    /* final true relative residual, evaluated in FP64                 */
    double seconds;         /* wall time of the solve (excludes preconditioner set-up)         */
    double matvec_seconds;  /* part of `seconds` spent in the coupling mat-vec kernels         */
    int x0_used;            /* 1 if the given initial guess was used (see celes_solve)         */
    double x0_residual;     /* relative residual ||T a_in - M x0|| / ||T a_in|| of the initial
                             * iterate actually used (after its weighting; 1 for x0 = 0),
                             * largest over the right-hand sides                              */
} celes_solve_info;

/* Fill *opt with defaults: FP64, LUT, lut_dr = 1, tol = 1e-8, inner_tol = 1e-4,
 * restart = 100, maxiter = 2000, max_refinements = 30, cuboid_edge = 0, device 0,
 * solver GMRES, target_Nj = 100, mem_cap_bytes = 0 (free device memory),
 * autotune = 0, translation = CELES_TRANSLATION_DIRECT, deterministic = 0. */
void celes_default_options(celes_options* opt);

/* Library version (CELES_VERSION). */
int celes_version(void);

/* Create a problem (Section 2: N disjoint spheres with centres pos [N][3],
 * radii radius [N], complex refractive indices n_sphere [N][2] in a medium
 * of real index n0, vacuum wavelength `wavelength`, multipole cut-off lmax).
 * Computes the Mie T-matrix of every sphere (Appendix B), the a5/b5 tables
 * (Appendix A.2) and, in LUT mode, the Hankel table (Section 3.2.2), and
 * copies the geometry to the device.  On success *h owns device memory until
 * celes_destroy.  Errors: CELES_E_ARG, CELES_E_NONFINITE, CELES_E_OVERLAP,
 * CELES_E_UNSUPPORTED (lmax > CELES_MAX_LMAX), CELES_E_DEVICE, CELES_E_OOM.
 * On error *h is NULL.  opt may be NULL (defaults). */
int celes_create(celes_handle** h, int64_t N, const double* pos, const double* radius,
                 const double* n_sphere, double n0, double wavelength, int lmax,
                 const celes_options* opt);

/* Release everything the handle owns.  NULL is allowed. */
void celes_destroy(celes_handle* h);

/* Replace the solver settings of a handle for its next solves: precision,
 * tol, inner_tol, restart, maxiter, max_refinements, verbose, solver,
 * target_Nj, mem_cap_bytes, autotune and translation are taken from *opt;
 * the fields fixed at creation (hankel, lut_dr, device, cuboid_edge) are
 * kept, and so are the
 * geometry, incident field and preconditioner (so FP64 and mixed solves can
 * share one preconditioner).  Errors: CELES_E_ARG (null, unknown solver,
 * precision or translation scheme). */
int celes_set_solve_options(celes_handle* h, const celes_options* opt);

/* Text of the last error on this handle (or of the last failed create when
 * h is NULL).  Valid until the next call on the handle. */
const char* celes_last_error(const celes_handle* h);

/* Incident field: K plane waves (Appendix A.1 PVWFs; coefficients from the
 * PVWF-to-SVWF expansion of Appendix A.2).  Wave k propagates along polar
 * angle beta[k] and azimuth alpha[k]; pol[k] = 1 (TE, e_alpha) or 2 (TM,
 * e_beta); amplitude E0 [K][2] complex (NULL = 1).  Replaces any previous
 * incident field and invalidates earlier solutions.  Errors: CELES_E_ARG. */
int celes_set_plane_waves(celes_handle* h, int K, const double* beta, const double* alpha,
                          const int* pol, const double* E0);

/* Incident field: one Gaussian beam along +z (Appendix C) with waist w,
 * focus r_G = focus [3], polarisation angle alpha_G (E0 direction
 * (-sin alpha_G, cos alpha_G, 0)), complex amplitude (E0_re, E0_im); the
 * polar-angle integral uses n_beta Gauss-Legendre nodes on [0, pi/2]
 * (n_beta <= 0: 512).  Sets K = 1.  Errors: CELES_E_ARG. */
int celes_set_gaussian_beam(celes_handle* h, double waist, const double* focus, double alpha_G,
                            double E0_re, double E0_im, int n_beta);

/* Copy the incident coefficients a_in [K][N][nmax] complex128 to host memory
 * a_out.  Errors: CELES_E_STATE (no incident field), CELES_E_ARG. */
int celes_get_incident(const celes_handle* h, double* a_out);

/* Number of right-hand sides of the current incident field (0 if none). */
int celes_num_rhs(const celes_handle* h);

/* cuboid_edge value of celes_build_preconditioner that picks the edge itself */
#define CELES_CUBOID_AUTO (-1.0)

/* Block-diagonal preconditioner (Section 3.2.1): partition the spheres into
 * cubes of edge `cuboid_edge` anchored at the minimum corner of the centres'
 * bounding box, assemble M_j = I - T W_jj per cube and factorise it (LU with
 * partial pivoting, FP64).  The LU storage grows as sum_j N_j^2 (Section
 * 3.2.1), so the edge is budgeted: with cuboid_edge = CELES_CUBOID_AUTO (any
 * negative value) the edge is chosen as by celes_plan_preconditioner from
 * the handle's target_Nj and mem_cap_bytes; with cuboid_edge > 0 that edge is
 * used as given.  Either way the build fails with CELES_E_OOM, before any
 * device allocation or launch, when the preconditioner's bytes (see
 * celes_options.mem_cap_bytes) exceed the cap.  cuboid_edge = 0 removes the
 * preconditioner.  A failed build leaves the handle without a preconditioner.
 * Errors: CELES_E_OOM, CELES_E_DEVICE. */
int celes_build_preconditioner(celes_handle* h, double cuboid_edge);

/* Cuboid edge of the block-diagonal preconditioner (Section 3.2.1) for N
 * centres pos [N][3] at cut-off lmax, planned on the host without a device:
 * among the edges e_q = 1.02 D 0.92^q (D the largest extent of the centres'
 * bounding box, q = 0, 1, ... while e_q >= D / 4096) the largest one whose
 * mean number of spheres per occupied cuboid is <= target_Nj (<= 0: 100) and
 * whose preconditioner bytes (formula at celes_options.mem_cap_bytes) are <=
 * mem_cap_bytes (<= 0: no cap).  Outputs (any may be NULL): the edge, the
 * number of cuboids, the bytes, the largest cuboid's sphere count.
 * Errors: CELES_E_ARG, CELES_E_OOM (no candidate edge fits the cap). */
int celes_plan_preconditioner(int64_t N, const double* pos, int lmax, double target_Nj, double mem_cap_bytes,
                              double* edge_out, int64_t* nblocks_out, double* bytes_out, int64_t* max_Nj_out);

/* Cuboid edge, number of cuboids and device bytes of the handle's current
 * preconditioner (all zero when there is none).  Any output may be NULL. */
int celes_preconditioner_info(const celes_handle* h, double* edge, int64_t* nblocks, double* bytes);

/* y = P^{-1} x for the block-diagonal preconditioner of the last
 * celes_build_preconditioner (Section 3.2.1): every cuboid's block of x is
 * multiplied by the inverse of M_j = I - T W_jj, for K right-hand sides.
 * precision CELES_FP64: x_dev, y_dev complex128 [K][N][nmax], FP64 inverses;
 * CELES_MIXED: complex64 vectors and the complex64 copy of the inverses.
 * K = 1 splits each block's columns over work-groups (a fixed-order
 * reduction of partial sums follows); K > 1 reads each inverse tile once per
 * group of eight right-hand sides.  Enqueued on `stream` (NULL = default
 * stream).  x_dev and y_dev must not alias.  Errors: CELES_E_ARG, CELES_E_STATE
 * (no preconditioner), CELES_E_DEVICE. */
int celes_apply_preconditioner(celes_handle* h, int precision, int K, const void* x_dev, void* y_dev,
                               void* stream);

/* Solve the master equation M b = T a_in (Section 2.2, eqs. masterequation
 * and M) for every right-hand side by right-preconditioned restarted GMRES
 * or, with opt.solver = CELES_SOLVER_BICGSTAB, right-preconditioned BiCGSTAB
 * (Section 3.2), W applied on the fly on the device.  BiCGSTAB runs until
 * its updated residual reaches tol (or breaks down), then checks the true
 * residual and starts a new run from the current iterate if needed; its
 * maxiter counts BiCGSTAB iterations.  With CELES_MIXED the complex64
 * correction solves use the chosen solver.  x0 [K][N][nmax]
 * complex128 is the initial guess (NULL: zero; the custom initial condition
 * of Section 4.2): per right-hand side it is multiplied by the complex weight
 * alpha = (M x0)^H rhs / ||M x0||^2 that minimises the residual of alpha x0
 * (one FP64 mat-vec; alpha = 1 when x0 is the solution) and used if that
 * residual is below ||rhs||, otherwise the solve starts from zero
 * (info->x0_used tells which, info->x0_residual the residual it starts from).  b_out [K][N][nmax]
 * receives the scattered-field coefficients (may be NULL: kept internally
 * for celes_cross_sections / celes_far_field).  info may be NULL.
 * Returns CELES_OK, CELES_E_NOCONV (b_out holds the best iterate),
 * CELES_E_BREAKDOWN, CELES_E_STATE, CELES_E_DEVICE. */
int celes_solve(celes_handle* h, const double* x0, double* b_out, celes_solve_info* info);

/* Initial guess from a sub-ensemble (Section 4.2: the solver accepts a custom
 * initial condition, typically the solution of a smaller system made of a
 * subset of the spheres).  Solves the master equation of the n_sub spheres
 * idx [n_sub] (distinct indices into this problem) alone, under this
 * problem's incident field (their rows of a_in) and options (precision,
 * solver, tolerance, Hankel mode), with a block-diagonal preconditioner of
 * cuboid edge `cuboid_edge` (<= 0: none), and writes x0_out [K][N][nmax]
 * complex128 (host): the sub-ensemble's coefficients at its spheres, zero at
 * all others, ready for celes_solve.  info (may be NULL) receives the
 * sub-solve's statistics.  Device memory of the sub-problem is released on
 * return.  Errors: CELES_E_ARG (range, repeats, null), CELES_E_STATE (no
 * incident field), CELES_E_NOCONV (x0_out holds the sub-solve's best
 * iterate), those of celes_create and celes_solve. */
int celes_subsystem_guess(celes_handle* h, int64_t n_sub, const int64_t* idx, double cuboid_edge, double* x0_out,
                          celes_solve_info* info);

/* Hot path, device pointers: y = W x for K right-hand sides (Section 2.2,
 * eq. a: (W x)^i_n = sum_{i' != i} sum_{n'} A_{n'n}(r_i - r_{i'}) x^{i'}_{n'}),
 * W evaluated on the fly per sphere pair (Section 3.2.2).  precision
 * CELES_FP64: x_dev, y_dev are complex128 [K][N][nmax]; CELES_MIXED:
 * complex64.  Enqueued on `stream` (a hipStream_t; NULL = default stream),
 * asynchronous.  x_dev and y_dev must not alias.  The handle keeps a device
 * scratch, allocated on first use and reused: one [K][N][nmax] vector of
 * source sums/differences plus the source-chunk partial sums (at most 2 GiB
 * on the VALU path, unless even a split of about 4,096 blocks needs more).
 * Errors: CELES_E_ARG, CELES_E_DEVICE, CELES_E_OOM (scratch). */
int celes_apply_W(celes_handle* h, int precision, int K, const void* x_dev, void* y_dev,
                  void* stream);

/* Bytes of the fixed device scratch buffer of celes_apply_W_noalloc. */
#define CELES_NOALLOC_SCRATCH_BYTES (128u << 20)

/* For callers that cannot allocate device memory (code under stream
 * capture, serving loops, harnesses that forbid allocation): y = W x exactly
 * as celes_apply_W computes it, on the same coupling kernels, but every
 * scratch byte of the call (the source sums/differences, K N nmax complex,
 * and the source-chunk partial sums, a multiple of that) is taken from one
 * fixed device array of CELES_NOALLOC_SCRATCH_BYTES per GPU, which the
 * library holds from the first call on that GPU until the process ends; the
 * number of source chunks is capped to fit it.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine) and always runs the
 * VALU kernel (celes_apply_W takes the matrix-core kernel for complex64
 * blocks of 16 or more right-hand sides).  Every call on one GPU shares that
 * array: calls that overlap in time on one GPU (other streams, other host
 * threads) race and must be serialised by the caller; the array keeps the
 * last call's contents, and each call overwrites every byte it reads.
 * Arguments and layouts as celes_apply_W.  Errors: CELES_E_ARG (null, K < 1,
 * unknown precision, or 2 K N nmax complex values of the precision larger
 * than the array), CELES_E_DEVICE (symbol lookup or launch), CELES_E_UNSUPPORTED. */
int celes_apply_W_noalloc(celes_handle* h, int precision, int K, const void* x_dev, void* y_dev,
                          void* stream);

/* As celes_apply_W but y = M x = x - T (W x) (eq. M). */
int celes_apply_M(celes_handle* h, int precision, int K, const void* x_dev, void* y_dev,
                  void* stream);

/* Cross sections for every right-hand side, E0 = 1 normalisation, from the
 * last solution: C_ext = -(pi/k^2) Re sum conj(a_in) b, C_abs =
 * -(pi/k^2) sum |b|^2 (Re(1/Q) + 1), C_sca = (1/k^2) oint |F|^2 dOmega by
 * quadrature of the far field (Appendix D).  Each output has K entries
 * (any may be NULL).  Errors: CELES_E_STATE (no solution), CELES_E_OOM,
 * CELES_E_DEVICE (far-field sums on the device). */
int celes_cross_sections(celes_handle* h, double* C_ext, double* C_sca, double* C_abs);

/* Far-field amplitude F(theta, phi) of the scattered field, E_sca ->
 * e^{ikr}/(kr) F (Appendix D), at ndir directions; F_out [K][ndir][3][2]
 * cartesian complex.  The sphere sums c_n = sum_i e^{-ik rhat.r_i} b^i_n run
 * on the device (FP64), the angular functions on the host; the same path
 * serves C_sca, S11 and the power flux.  Errors: CELES_E_STATE, CELES_E_ARG,
 * CELES_E_OOM, CELES_E_DEVICE. */
int celes_far_field(celes_handle* h, int64_t ndir, const double* theta, const double* phi,
                    double* F_out);

/* (1,1) element of the phase matrix as the paper's validation obtains it
 * (Section 4): the far-field intensity |F(theta, phi)|^2 averaged over every
 * solved right-hand side of the nh problems hs (e.g. one TE and one TM run,
 * or one problem with both plane waves) and over n_phi azimuths
 * phi_j = 2 pi j / n_phi, at n_theta polar angles theta.  out [n_theta]:
 * k^2 times the polarisation-averaged differential scattering cross section
 * (unnormalised; divide by the value at theta = 0 for S11(0) = 1).  The
 * sphere sums of the far field run on the device of each problem.  Errors:
 * CELES_E_ARG (null, sizes,
 * problems of different wavenumbers), CELES_E_STATE (a problem without a
 * solution; its last error says so). */
int celes_s11(celes_handle* const* hs, int nh, int64_t n_theta, const double* theta, int n_phi, double* out);

/* Electric near field at npt points outside all spheres (Section 2.1, eq.
 * Escat summed over spheres), plus the incident field when add_incident != 0
 * (plane wave, or the Gaussian beam's angular spectrum of Appendix C on
 * 256 x 256 nodes); E_out [K][npt][3][2] cartesian complex.  Evaluated on
 * the device in FP64.  Errors: CELES_E_STATE, CELES_E_ARG, CELES_E_OOM,
 * CELES_E_DEVICE. */
int celes_near_field(celes_handle* h, int64_t npt, const double* pts, int add_incident,
                     double* E_out);

/* Mie T-matrix entries of one sphere (Appendix B) for size parameter kR =
 * k R and relative index m = n_sphere / n0: Q_out [2][lmax][2] =
 * (Q_{1l}, Q_{2l}) complex.  Errors: CELES_E_ARG. */
int celes_mie_coefficients(int lmax, double kR, double m_re, double m_im, double* Q_out);

/* Power balance of the last solution under a Gaussian beam (Appendix D),
 * per right-hand side: out[4k + 0] = incident power divided by the
 * intensity of a unit plane wave (area units), out[4k + 1] = reflected
 * fraction R (scattered flux through the lower hemisphere at infinity),
 * out[4k + 2] = transmitted fraction T (flux of incident + scattered field
 * through the upper hemisphere), out[4k + 3] = absorbed fraction A; energy
 * conservation gives R + T + A = 1.  n_beta, n_alpha: polar nodes per
 * hemisphere and azimuthal nodes (<= 0: from the band limit lmax + k D,
 * D = 2 max |r_i|); the far-field sphere sums run on the device.  Errors:
 * CELES_E_STATE (no solution, or the incident field is not a Gaussian beam),
 * CELES_E_ARG, CELES_E_OOM, CELES_E_DEVICE. */
int celes_power_flux(celes_handle* h, int n_beta, int n_alpha, double* out);

/* Kernel timing for measurement: enable = 1 starts recording HIP events on
 * the launch stream right before and after every coupling kernel that
 * celes_apply_W / celes_apply_M / celes_solve launch on this handle (the
 * prep and finish kernels are outside); enable = 0 stops and returns the
 * average kernel duration in ms and the number of launches (either output may
 * be NULL).  At most the first 4096 launches of a window are recorded.
 * Errors: CELES_E_ARG, CELES_E_DEVICE. */
int celes_kernel_timing(celes_handle* h, int enable, double* avg_ms, int* count);

/* Geometry of the Hankel lookup table (Section 3.2.2): nodes d_lo + q*dr,
 * q = 0..n_int; d_lo = max(dr, (floor(2 min R / dr) - 1) dr), n_int =
 * ceil((d_max - d_lo)/dr) + 1 with d_max the diagonal of the centres'
 * bounding box.  Any output may be NULL.  Errors: CELES_E_ARG. */
int celes_lut_info(const celes_handle* h, double* d_lo, double* dr, int64_t* n_int);

/* Number of spheres, lmax and nmax of a handle. */
int celes_dims(const celes_handle* h, int64_t* N, int* lmax, int* nmax);

/* Translation coefficient tables used by the kernels (Appendix A.2):
 * writes a5 [L][2L+1][L][2L+1][2L+1] and Im(b5) for l, l' = 1..L,
 * m = -l..l (offset by L), p = 0..2L, with a5(l,m|l',m'|p) at
 * [((((l-1)(2L+1) + m+L) L + l'-1)(2L+1) + m'+L)(2L+1) + p].  For tests of
 * the host tables.  Errors: CELES_E_ARG. */
int celes_translation_tables(int lmax, double* a5_out, double* b5im_out);

/* Copy the scattered-field coefficients of the last solve of this problem
 * (by celes_solve or by a batch containing it) to b_out [K][N][nmax]
 * complex128.  Errors: CELES_E_STATE (no solution), CELES_E_ARG. */
int celes_get_solution(const celes_handle* h, double* b_out);

/* ---------------------------------------------------------------------------
 * Batched solves.  A batch couples nothing: it solves the master equation
 * (Section 2.2) of every right-hand side of every problem independently, but
 * advances all of them together: one persistent mat-vec launch per Arnoldi
 * step covers all problems and right-hand sides (ragged sizes allowed), the
 * Krylov state of every system stays on the device, and one Arnoldi step is
 * captured once in a hipGraph and replayed.  precision CELES_MIXED runs
 * complex64 inner GMRES with FP64 residuals and refinement; CELES_FP64 runs
 * FP64 throughout.  A problem whose handle has a block-diagonal
 * preconditioner (celes_build_preconditioner, Section 3.2.1) has it applied
 * to each of its systems (right preconditioning, complex64 inverses in the
 * inner solves of CELES_MIXED); the other problems run unpreconditioned.
 * Rebuilding or removing a preconditioner between solves is allowed.
 * ------------------------------------------------------------------------- */
typedef struct celes_batch celes_batch;

/* Build a batch over nprob problems (all with the same lmax, each with its
 * incident field set).  The handles stay owned by the caller and must
 * outlive the batch; opt (precision, tol, inner_tol, restart, maxiter,
 * max_refinements, hankel, translation, deterministic) applies to the whole
 * batch (NULL: defaults); translation selects the scheme of the persistent
 * VALU mat-vec (problems on the matrix cores use the direct form).
 * Batches are compiled for lmax <= 4.  Errors: CELES_E_ARG, CELES_E_STATE,
 * CELES_E_UNSUPPORTED, CELES_E_OOM, CELES_E_DEVICE. */
int celes_batch_create(celes_batch** b, int nprob, celes_handle* const* probs, const celes_options* opt);

/* Release the batch (not the problems).  NULL is allowed. */
void celes_batch_destroy(celes_batch* b);

/* Number of systems (sum of the problems' right-hand sides). */
int celes_batch_num_systems(const celes_batch* b);

/* Text of the last error of the batch (or of a failed create when b is NULL). */
const char* celes_batch_last_error(const celes_batch* b);

/* y = M x for every system at once on device buffers in the batch's flat
 * layout (problem after problem, each [K_p][N_p][nmax]); complex128 for
 * CELES_FP64, complex64 for CELES_MIXED.  Enqueued on `stream`.
 * Errors: CELES_E_ARG, CELES_E_DEVICE. */
int celes_batch_apply_M(celes_batch* b, int precision, const void* x_dev, void* y_dev, void* stream);

/* Choose the batched mat-vec's source-chunk length and right-hand-side block
 * width by timing the candidates on this batch; the choice is kept by the
 * batch.  Outputs (may be NULL): the best time of one batched M x in ms, the
 * chunk length, the block width.  Errors: CELES_E_ARG, CELES_E_STATE (the
 * batch was created with opt.deterministic = 1). */
int celes_batch_autotune(celes_batch* b, int precision, double* best_ms, int* best_chunk, int* best_kb);

/* Solve every system from a zero initial guess to opt.tol; solutions are
 * stored in the problems (celes_get_solution, celes_cross_sections).  infos
 * [num_systems] (may be NULL) receives per-system iterations and residuals,
 * summary (may be NULL) totals and wall time.  Returns CELES_OK,
 * CELES_E_NOCONV, CELES_E_BREAKDOWN, CELES_E_OOM or CELES_E_DEVICE. */
int celes_batch_solve(celes_batch* b, celes_solve_info* infos, celes_solve_info* summary);

/* ---------------------------------------------------------------------------
 * Learned initial guess.  A small network predicts every sphere's scattered
 * coefficients from its own and its 16 nearest neighbours' radii, relative
 * positions and incident coefficients (all in the sphere's incident-phase
 * frame, scaled by ||a_in^i||); the prediction is passed to celes_solve as
 * x0 (the custom initial condition the paper's solver accepts, Section 4.2).
 * Features of sphere i: R_i/lambda; a_in^i rotated into its own phase
 * frame and normalised; for each of the 16 nearest spheres the relative
 * position/lambda, R_j/lambda and a_in^j in sphere i's frame.
 * Layers: in_pad -> 128 -> 128 -> 128 -> out_pad, SiLU, bf16 weights and
 * activations with FP32 accumulation, FP32 master weights, Adam.  It is
 * trained on coefficients the solver produced: its output is the
 * multiple-scattering correction b^i - T^i a_in^i to the single-scattering
 * response (in the sphere's frame), so an untrained or uninformed network
 * falls back to single scattering.  Intended for training sets
 * and problems of one lmax; only the first right-hand side is used.
 * ------------------------------------------------------------------------- */
typedef struct celes_nn celes_nn;

/* Create a network for cut-off lmax with weights drawn from `seed`
 * (SplitMix64 counters, uniform in +-1/sqrt(fan_in)).  Errors: CELES_E_ARG,
 * CELES_E_OOM. */
int celes_nn_create(celes_nn** net, int lmax, uint64_t seed);
void celes_nn_destroy(celes_nn* net);
const char* celes_nn_last_error(const celes_nn* net);

/* Feature width (real and padded), hidden width, output width (real, padded:
 * 2 nmax reals), number of parameters.  Any output may be NULL. */
int celes_nn_dims(const celes_nn* net, int* in_dim, int* in_pad, int* hidden, int* out_dim, int* out_pad,
                  int64_t* nparam);

/* FP32 master parameters, flat: for each layer W [in][out] row-major then b
 * [out].  set also resets the optimiser state.  Errors: CELES_E_ARG. */
int celes_nn_get_params(const celes_nn* net, float* params);
int celes_nn_set_params(celes_nn* net, const float* params);

/* Features X [N][in_pad] (as the network sees them, bf16 values) and, if the
 * problem is solved, targets Y [N][out_pad] (b - T a_in in the sphere's
 * frame, divided by ||a_in^i||) of a problem.  Either may be
 * NULL.  Errors: CELES_E_ARG, CELES_E_STATE. */
int celes_nn_features(celes_nn* net, celes_handle* h, float* X, float* Y);

/* Mean-squared loss and its gradient (flat, like the parameters) on M rows
 * of host data X [M][in_pad], Y [M][out_pad] (X rounded to bf16).  For
 * gradient checks.  Errors: CELES_E_ARG, CELES_E_OOM. */
int celes_nn_loss_grad(celes_nn* net, int64_t M, const float* X, const float* Y, double* loss, float* grad);

/* Network output Z [M][out_pad] for host features X [M][in_pad]. */
int celes_nn_forward(celes_nn* net, int64_t M, const float* X, float* Z);

/* Append a solved problem's features and targets to the training set. */
int celes_nn_add_training_problem(celes_nn* net, celes_handle* h);

/* Train for `epochs` passes over the training set in shuffled minibatches
 * (SplitMix64 from `seed`), Adam with a cosine learning-rate schedule from
 * lr.  *loss receives the mean loss of the last epoch.  Errors:
 * CELES_E_ARG, CELES_E_STATE (no data), CELES_E_OOM, CELES_E_DEVICE. */
int celes_nn_train(celes_nn* net, int epochs, int batch, double lr, uint64_t seed, double* loss);

/* Predicted scattered coefficients x0 [N][nmax] complex128 of a problem's
 * first right-hand side, T a_in plus the predicted correction (pass to
 * celes_solve as x0).  Errors: CELES_E_ARG,
 * CELES_E_STATE, CELES_E_OOM, CELES_E_DEVICE. */
int celes_nn_predict(celes_nn* net, celes_handle* h, double* x0);

#ifdef __cplusplus
}
#endif

#endif /* CELES_H */

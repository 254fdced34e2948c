"""Benchmark of the hot path on one MI355X.

Workload (default): the 20,000-sphere slab (lognormal radii, mean 150 nm,
sigma 10%, n = 1.52, volume fraction 0.3, thickness 3 um), lmax = 4,
Gaussian beam (waist 2 um) at 550 nm, Hankel lookup table at 1 nm.

A step is one FP64 coupling mat-vec W.b over all N(N-1) sphere pairs
(complex128).  `value` is the number of pair-multipole updates executed in
the timed steps, N(N-1) nmax^2 per mat-vec, divided by their wall time.

Also reported: the coupling kernel alone (HIP events on its launch stream,
used for the roofline), the complex64 mat-vec of the mixed path, time to
relative residual 1e-6 of block-diagonal preconditioned GMRES in FP64 and in
mixed precision on the same seed and the same cuboid partition (one
preconditioner, set up once and reported separately), the 2,000-sphere slab's
preconditioned FP64 solve to 1e-8, and the CPU oracle timed on a bounded
sample of receiver rows.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-multipole updates/s of W·b; time-to-residual 1e-6, mixed vs FP64"
PEAK_FP32_MFMA_TFLOPS = 157.3   # MI355X dense FP32 matrix
PEAK_FP64_VALU_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_FP32_VALU_TFLOPS = 157.3  # MI355X FP32 vector peak (twice the FP64 rate)


def _pass_counts(L):
    """Per-pair terms of the coupling kernel's arithmetic, in flops (real
    add, mul = 1, FMA = 2; complex multiply 6, complex multiply-accumulate 8;
    sqrt, divide and sincos 1 each): the set-up shared by every receiving
    |m| (geometry, Hankel orders, Legendre columns and azimuthal phases for
    mu = 0..2L) and the work of each receiving |m| = M0 (source rotations,
    A and B sums, A +- iB, accumulations)."""
    def iabs(a):
        return -a if a < 0 else a

    def pa(l, lp, mu):
        p = max(iabs(l - lp), mu)
        p += (l + lp + p) & 1
        return max(0, (l + lp - p) // 2 + 1) if p <= l + lp else 0

    def pb(l, lp, mu):
        p = max(iabs(l - lp) + 1, mu)
        if not ((l + lp + p) & 1):
            p += 1
        return max(0, (l + lp - 1 - p) // 2 + 1) if p <= l + lp - 1 else 0

    P = 2 * L

    def setup(lut, mumax):
        f = 19                                             # geometry
        # Hankel: table index + Horner for h_0, h_1 (24) + 1/(kd) (1), or
        # sincos + 1/(kd) + h_0, h_1 (6); then the recurrence, 5 per order
        f += (4 + 24 + 1 + 5 * (P - 1)) if lut else (4 + 6 + 5 * (P - 1))
        for mu in range(mumax + 1):
            if mu > 0:
                f += 2 + 6                                 # P_mu^mu and e^{i mu phi}
            ncol = P - mu + 1
            f += 3 * max(0, ncol - 2) + (2 if ncol >= 2 else 0) + 2 * ncol   # Legendre column + H
        return f

    def work(M0):
        f = 0
        for mu in range(min(2 * L, L + M0) + 1):
            for sgn in (1, -1):
                if sgn < 0 and (mu == 0 or M0 == 0):
                    continue
                mp = M0 + sgn * mu
                if iabs(mp) > L:
                    continue
                two = M0 > 0 or mu > 0
                for lp in range(max(1, iabs(mp)), L + 1):
                    f += 6 * (4 if two else 2)              # source rotations
                    for l in range(max(1, M0), L + 1):
                        f += 4 * (pa(l, lp, mu) + pb(l, lp, mu))   # A and B sums
                        f += 4                               # P = A + iB, Q = A - iB
                        f += 8 * (4 if two else 2)           # accumulations
        return f

    return setup, work


def flops_per_pair(L, hankel_lut=True):
    """Algorithmic flops per sphere pair of one W.b (one right-hand side):
    the pair set-up once (mu = 0..2L) plus the work of every receiving |m|.
    This is what the roofline fraction is computed from."""
    setup, work = _pass_counts(L)
    return setup(hankel_lut, 2 * L) + sum(work(M0) for M0 in range(L + 1))


def flops_per_pair_executed(L, groups, hankel_lut=True):
    """Flops per pair as the kernel executes them: the pair set-up is
    repeated in each pass group (a group covers the mu its passes need)."""
    setup, work = _pass_counts(L)
    f = sum(work(M0) for M0 in range(L + 1))
    for g in groups:
        f += setup(hankel_lut, max(min(2 * L, L + M0) for M0 in g))
    return f


def _delta_pi2(l, k, m):
    # d^l_{km}(pi/2) (Wigner's sum), to count the nonzero constants the
    # rotation kernel multiplies by
    F = math.factorial
    s = 0
    for j in range(2 * l + 1):
        a, b, c = l + m - j, k - m + j, l - k - j
        if a < 0 or b < 0 or c < 0:
            continue
        s += (-1) ** ((k - m + j) % 2) * F(2 * l) // (F(a) * F(j) * F(b) * F(c))
    return s


def flops_per_pair_rotate(L, hankel_lut=True, executed=False):
    """Flops per sphere pair of the rotation-translation-rotation mat-vec
    (one right-hand side; counting as in flops_per_pair): geometry, Hankel
    orders and the powers of q and e^{i theta} once; the axial A_z, B_z sums
    for m >= 0 once (executed: once per polarisation pass); per pass the two
    rotations (phases, sum/difference pairs, the two constant d(pi/2)
    products over m >= 0 or k >= 0) and the axial translation for +-m."""
    P = 2 * L
    f = 19 + ((4 + 24 + 1 + 5 * (P - 1)) if hankel_lut else (4 + 6 + 5 * (P - 1))) + 12 * (L - 1)
    # nonzero d(pi/2) entries over one half (the other half follows by symmetry)
    nzh = {l: sum(1 for k in range(-l, l + 1) for m in range(0, l + 1) if _delta_pi2(l, k, m) != 0)
           for l in range(1, L + 1)}
    sums = 0
    per_pass = 0
    for l in range(1, L + 1):
        rot = 8 * l + 4 * nzh[l] + 12 * l + 8 * l + 4 * nzh[l]          # S/D, Delta, phase, P/Q, Delta^T
        per_pass += 12 * l + rot                                        # rotate in (source phases + rotation)
        per_pass += rot + 2 + 16 * l                                    # rotate out + accumulate
        for m in range(0, l + 1):
            for lp in range(max(1, m), L + 1):
                # A terms: |l-l'| <= p <= l+l', l+l'+p even; B terms: |l-l'|+1 <= p <= l+l'-1, odd
                sums += 4 * ((min(l, lp) + 1) + min(l, lp))
                per_pass += (4 + 8) * (2 if m > 0 else 1)               # A +- iB, multiply-accumulate
    return f + 2 * per_pass + (2 * sums if executed else sums)


# pass groups of the coupling kernel per cut-off (receiving |m| per group)
KERNEL_GROUPS = {1: [(0, 1)], 2: [(0, 2), (1,)], 3: [(1,), (0, 3), (2,)], 4: [(2, 4), (0, 3), (1,)],
                 5: [(3, 4), (2, 5), (1,), (0,)], 6: [(3, 5), (2, 6), (0, 4), (1,)]}


def kernel_source_digest():
    """sha256 of what fixes the coupling kernel and its launch: the kernel
    sources and the host mat-vec driver that sizes the launch (counters are
    only valid for them)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1706_02145_amd", "csrc")
    for f in ("wx_kernels.hip", "wx_plan.hpp", "wx_launch.hpp", "device_common.hpp", "wx_dispatch.hip"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(d, "celes_lib.cpp"), encoding="utf-8") as fh:
        src = fh.read()
    a = src.index("// right-hand-side block width: largest compiled width")
    b = src.index("// GMRES (right-preconditioned", a)
    h.update(src[a:b].encode())
    return h.hexdigest()


def measured_traffic(name, N, L, hankel):
    """HBM bytes per mat-vec launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None if it was taken on other kernel sources or
    another workload."""
    f = os.path.join(ROOT, "profiles", f"wx_fused_{name}_hbm_traffic.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha256") != kernel_source_digest() or t.get("N") != N or t.get("lmax") != L \
            or t.get("hankel") != hankel:
        return None
    return t["bytes_per_launch"]


def _oracle_rows_worker(args):
    """CPU baseline worker: the oracle's W.b rows r0, r0 + stride, ... for
    `seconds` of wall time; returns (rows done, seconds)."""
    pos, radii, k, L, dr, r0, stride, seconds = args
    from threadpoolctl import threadpool_limits
    from celes_inputs import random_coefficients
    from oracle.lut import lut_for
    from oracle.translation import apply_W_rows
    N = pos.shape[0]
    nm = 2 * L * (L + 2)
    lut = lut_for(pos, radii, k, L, dr)
    xs = random_coefficients(1, 1, N, nm)[0]
    rows, t = 0, 0.0
    with threadpool_limits(limits=1):
        apply_W_rows(pos, xs, k, L, [r0], hankel=lut)    # warm the coefficient caches
        t1 = time.perf_counter()
        r = r0
        while t < seconds and r < N:
            apply_W_rows(pos, xs, k, L, [r], hankel=lut)
            rows += 1
            r += stride
            t = time.perf_counter() - t1
    return rows, t


def _realisation(args):
    seed, n = args
    from celes_inputs import workload
    w = workload("slab5000_l3", seed=seed, n=n)
    return w.positions, w.radii


def batched_mode(a):
    """Batched workload: one 10,000-sphere slab (lmax 3) with 64 right-hand
    sides (32 polar angles 0..60 deg x TE/TM) plus 32 disorder realisations
    of uneven N in [500, 5000] (2 right-hand sides each, normal incidence),
    all advanced together by the batched solver (complex64 inner GMRES, FP64
    refinement, autotuned mat-vec work split)."""
    import numpy as np
    import torch
    import paper_1706_02145_amd as P
    from celes_inputs import workload
    from concurrent.futures import ProcessPoolExecutor
    def log(msg):
        print(f"[batched] {msg} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    w = workload("slab10000_l3")
    log("10,000-sphere slab generated")
    rng = np.random.Generator(np.random.PCG64(40))
    sizes = [int(v) for v in rng.integers(500, 5001, size=a.realisations)]
    with ProcessPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        reals = list(ex.map(_realisation, [(4001 + r, n) for r, n in enumerate(sizes)]))
    t_gen = time.perf_counter() - t0
    log(f"{len(reals)} realisations generated")
    probs = []
    big = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, 3, hankel=P.CELES_HANKEL_LUT)
    betas = np.repeat(np.arange(32) * (np.pi / 3) / 31, 2)
    big.set_plane_waves(betas, np.zeros(64), np.tile([1, 2], 32))
    probs.append(big)
    for pos, rad in reals:
        q = P.Problem(pos, rad, 1.52, 1.0, 550.0, 3, hankel=P.CELES_HANKEL_LUT)
        q.set_plane_waves([0.0, 0.0], [0.0, 0.0], [1, 2])
        probs.append(q)
    t_pre = 0.0
    if a.batch_precond > 0:
        t1 = time.perf_counter()
        for q in probs:
            q.build_preconditioner(a.batch_precond)
        torch.cuda.synchronize()
        t_pre = time.perf_counter() - t1
        log(f"block-diagonal preconditioners ({a.batch_precond:g} nm cuboids) for {len(probs)} problems "
            f"in {t_pre:.1f} s")
    updates = sum(q.N * (q.N - 1) * q.nmax ** 2 * q.num_rhs for q in probs)
    log(f"{len(probs)} problems set up, {updates:.3e} updates per batched mat-vec")
    scheme = P.CELES_TRANSLATION_ROTATE if a.batch_translation == "rotate" else P.CELES_TRANSLATION_DIRECT
    bt = P.Batch(probs, precision=P.CELES_MIXED, tol=a.batch_tol, inner_tol=1e-3, restart=a.batch_restart,
                 maxiter=a.batch_maxiter, max_refinements=4, verbose=1, translation=scheme)
    tune = bt.autotune(P.CELES_MIXED)
    log(f"autotuned: {tune}")
    # one batched M x in complex64 over every system (HIP events on the caller's stream)
    n_total = sum(q.N * q.nmax * q.num_rhs for q in probs)
    x = torch.randn(n_total, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    bt.apply_M(x, y, P.CELES_MIXED)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(3):
        bt.apply_M(x, y, P.CELES_MIXED)
    ev1.record()
    torch.cuda.synchronize()
    mv_ms = ev0.elapsed_time(ev1) / 3
    log(f"batched M x: {mv_ms:.1f} ms")
    # the 64-right-hand-side slab alone: its W x runs on the matrix cores
    xb = torch.randn(big.num_rhs * big.N * big.nmax, dtype=torch.complex64, device="cuda")
    yb = torch.empty_like(xb)
    big.apply_W(xb, yb, P.CELES_MIXED, K=big.num_rhs)
    torch.cuda.synchronize()
    big.kernel_timing(True)
    ev0.record()
    for _ in range(3):
        big.apply_W(xb, yb, P.CELES_MIXED, K=big.num_rhs)
    ev1.record()
    torch.cuda.synchronize()
    big_kernel_ms, _ = big.kernel_timing(False)
    big_ms = ev0.elapsed_time(ev1) / 3
    big_pairs = big.N * (big.N - 1)
    apply_flops = 4 * big.nmax ** 2 * big.num_rhs * big_pairs      # (A+-B) block products, all RHS
    log(f"64-RHS slab W x: {big_ms:.1f} ms (kernel {big_kernel_ms:.1f} ms)")
    if a.batch_no_solve:
        print(json.dumps({"batched_matvec_ms": mv_ms, "big_matvec_ms": big_ms, "big_kernel_ms": big_kernel_ms,
                          "big_kernel_tflops": apply_flops / (big_kernel_ms * 1e-3) / 1e12,
                          "frac": apply_flops / (big_kernel_ms * 1e-3) / 1e12 / PEAK_FP32_MFMA_TFLOPS}))
        return
    t1 = time.perf_counter()
    per, summ = bt.solve(check=False)
    log("solve done")
    t_solve = time.perf_counter() - t1
    its = [i["iterations"] for i in per]
    print(json.dumps({
        "metric": "batched pair-multipole updates/s of W·b (complex64) and batched time to residual",
        "value": updates / (mv_ms * 1e-3), "unit": "updates/s", "n_gpus": 1, "dtype": "f32 (FP64 refinement)",
        "data": "synthetic",
        "config": {"workload": f"slab10000_l3 (N={w.N}, 64 RHS: 32 polar angles 0-60 deg x TE/TM) + "
                               f"{a.realisations} realisations N in [500,5000] x 2 RHS, lmax 3, LUT 1 nm",
                   "realisation_sizes": sizes,
                   "valu_translation": a.batch_translation},
        "systems": bt.num_systems, "updates_per_batched_matvec": updates, "batched_matvec_ms": mv_ms,
        "roofline": {"kernel": "wx_mfma_kernel<3, 4, 0> (64-RHS slab alone)",
                     "bound": "mfma", "achieved": apply_flops / (big_kernel_ms * 1e-3) / 1e12,
                     "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": apply_flops / (big_kernel_ms * 1e-3) / 1e12 / PEAK_FP32_MFMA_TFLOPS,
                     "kernel_ms": big_kernel_ms,
                     "flops_counted": "4 nmax^2 K per pair (the block products); the per-pair block build "
                                      "runs on the VALU and is not counted",
                     "matvec_ms": big_ms, "updates_per_s": big_pairs * big.nmax ** 2 * big.num_rhs / (big_ms * 1e-3)},
        "autotune": tune, "solve_seconds": t_solve, "solve_status": summ["status"],
        "worst_rel_residual": summ["rel_residual"], "tol": a.batch_tol, "restart": a.batch_restart,
        "iterations_max": max(its), "iterations_mean": float(np.mean(its)), "refinements": summ["refinements"],
        "preconditioner_edge_nm": a.batch_precond if a.batch_precond > 0 else None,
        "preconditioner_setup_s": t_pre, "geometry_seconds": t_gen}))


def mixed_mode(a):
    """Mixed precision against all-FP64 on the 20,000-sphere slab (lmax 4,
    Gaussian beam, block-diagonal preconditioner, same seed): complex64 inner
    GMRES with FP64 residual refinement vs FP64 GMRES, each solved to 1e-8
    (solutions compared) and to 1e-6 (time to residual), with the direct and
    the rotation-translation-rotation mat-vec, on one handle and one
    preconditioner (celes_set_solve_options switches between the runs)."""
    import numpy as np
    import torch
    import paper_1706_02145_amd as P
    from celes_inputs import workload

    t0 = time.perf_counter()

    def log(msg):
        print(f"[mixed] {msg} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)

    w = workload(a.mixed_workload)
    il = w.illumination
    log(f"{w.name} generated (N={w.N})")
    p = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, hankel=P.CELES_HANKEL_LUT,
                  lut_dr=w.lut_dr, restart=100, maxiter=3000, max_refinements=8, verbose=1)
    p.set_gaussian_beam(il["waist"], il["focus"], il["alpha_G"], il["E0"])
    t1 = time.perf_counter()
    p.build_preconditioner(a.cuboid_edge)
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t1
    log(f"preconditioner built in {t_pre:.1f} s")
    schemes = (("", P.CELES_TRANSLATION_DIRECT), ("_rotate", P.CELES_TRANSLATION_ROTATE))
    results, sols = {}, {}
    for tol in (1e-8, 1e-6):
        for suffix, scheme in schemes:
            for name, prec in (("fp64", P.CELES_FP64), ("mixed", P.CELES_MIXED)):
                key = name + suffix
                p.set_solve_options(precision=prec, tol=tol, inner_tol=1e-4 if tol < 1e-7 else 1e-3,
                                    translation=scheme)
                t1 = time.perf_counter()
                b, info = p.solve()
                torch.cuda.synchronize()
                t_sol = time.perf_counter() - t1
                log(f"{key} tol {tol:g}: solved in {t_sol:.1f} s, {info['iterations']} iterations")
                results[f"{key}_tol_{tol:g}"] = {"seconds": t_sol, "iterations": info["iterations"],
                                                 "refinements": info["refinements"], "matvecs": info["matvecs"],
                                                 "rel_residual": info["rel_residual"], "status": info["status"]}
                if tol < 1e-7:
                    sols[key] = b
    p.close()

    def diff(u, v):
        return float(np.linalg.norm(sols[u] - sols[v]) / np.linalg.norm(sols[v]))

    t64, t32 = results["fp64_tol_1e-06"]["seconds"], results["mixed_tol_1e-06"]["seconds"]
    print(json.dumps({
        "metric": "time to residual 1e-6, mixed precision (complex64 inner GMRES, FP64 refinement) vs FP64",
        "value": t32, "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f32 / f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: N={w.N} RSA slab, radii lognormal(150 nm, 10%), n=1.52, vf 0.3, "
                               f"lmax={w.lmax}, Gaussian beam w=2 um, LUT 1 nm, block-diagonal preconditioner "
                               f"(cuboid edge {a.cuboid_edge:g} nm), restart 100",
                   "N": w.N, "lmax": w.lmax},
        "preconditioner_setup_s": t_pre,
        "speedup_mixed_vs_fp64_1e-6": t64 / t32,
        "speedup_mixed_vs_fp64_1e-8": results["fp64_tol_1e-08"]["seconds"] / results["mixed_tol_1e-08"]["seconds"],
        "speedup_mixed_rotate_vs_fp64_1e-6": t64 / results["mixed_rotate_tol_1e-06"]["seconds"],
        "solution_rel_diff_mixed_vs_fp64_at_1e-8": diff("mixed", "fp64"),
        "solution_rel_diff_rotate_vs_direct_fp64_at_1e-8": diff("fp64_rotate", "fp64"),
        "solution_rel_diff_mixed_rotate_vs_fp64_at_1e-8": diff("mixed_rotate", "fp64"),
        "results": results}))


def _cyl_workload(args):
    n, vf = args
    from celes_inputs import cylinder_workload
    return cylinder_workload(n, vf)


def paper_mode(a):
    """The paper's run-time comparison setting (Section 4, Table 1: N = 1e4
    and 2e4 at vf 10 % and 50 %): spheres of R = 100 nm, n = 1.5, in a
    cylindrical slab, lambda = 532 nm, lmax 3, Gaussian beam (waist 4 um),
    solved to 1e-4 with and without a block-diagonal preconditioner of about
    200 spheres per cuboid; FP64 and mixed precision; GMRES and
    (--paper-solvers) BiCGSTAB, the two solvers of Section 3.2.  One BiCGSTAB
    iteration costs two mat-vecs."""
    import numpy as np
    import torch
    import paper_1706_02145_amd as P
    from concurrent.futures import ProcessPoolExecutor

    t0 = time.perf_counter()

    def log(msg):
        print(f"[paper] {msg} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)

    rows = [(int(r.split(":")[0]), float(r.split(":")[1])) for r in a.paper_rows.split(",")]
    with ProcessPoolExecutor(min(16, len(rows), os.cpu_count() or 1)) as ex:
        wls = list(ex.map(_cyl_workload, rows))
    log(f"{len(wls)} geometries generated")
    solvers = {"gmres": P.CELES_SOLVER_GMRES, "bicgstab": P.CELES_SOLVER_BICGSTAB}
    results, summary = {}, {}
    for (n, vf), w in zip(rows, wls):
        il = w.illumination
        edge = (200 * 4.0 / 3.0 * np.pi * 100.0 ** 3 / vf) ** (1.0 / 3.0)   # ~200 spheres per cuboid
        row = f"N={n} vf={vf:g}"
        res = {}
        runs = [(sv, name, prec, pre) for sv in a.paper_solvers.split(",")
                for name, prec in (("fp64", P.CELES_FP64), ("mixed", P.CELES_MIXED)) for pre in (False, True)]
        for sv, name, prec, pre in runs:
            p = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax,
                          hankel=P.CELES_HANKEL_LUT, lut_dr=w.lut_dr, precision=prec, tol=w.tol, restart=100,
                          maxiter=5000, inner_tol=1e-3, verbose=1, solver=solvers[sv])
            p.set_gaussian_beam(il["waist"], il["focus"], il["alpha_G"], il["E0"])
            t_pre = 0.0
            if pre:
                t1 = time.perf_counter()
                p.build_preconditioner(edge)
                torch.cuda.synchronize()
                t_pre = time.perf_counter() - t1
            t1 = time.perf_counter()
            _, info = p.solve(check=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            key = ("" if sv == "gmres" else sv + "_") + name + ("_preconditioned" if pre else "")
            res[key] = {"seconds": dt, "iterations": info["iterations"], "matvecs": info["matvecs"],
                        "rel_residual": info["rel_residual"], "status": info["status"],
                        "preconditioner_setup_s": t_pre}
            log(f"{row} {key}: {dt:.2f} s (+{t_pre:.2f} s set-up), {info['iterations']} iterations, "
                f"{info['matvecs']} mat-vecs, residual {info['rel_residual']:.2e}")
            p.close()
        results[row] = {"cylinder_radius_nm": w.extra["cylinder_radius"], "cuboid_edge_nm": edge, "runs": res}
        summary[row] = min(v["seconds"] + v["preconditioner_setup_s"] for v in res.values() if v["status"] == 0)
    head = "N=20000 vf=0.1" if "N=20000 vf=0.1" in summary else next(iter(summary))
    print(json.dumps({
        "metric": "solve time to relative residual 1e-4 (the paper's Table 1 setting)", "value": summary[head],
        "unit": "s", "higher_is_better": False, "n_gpus": 1, "dtype": "f64 / f32", "data": "synthetic",
        "config": {"workload": f"paper Table 1 rows {list(summary)}: R=100 nm, n=1.5, cylindrical slab t=2 um "
                               f"(radius from N and vf; RSA at vf 0.1, overlap-relaxation packing at vf 0.5), "
                               f"lambda=532 nm, lmax 3, Gaussian beam waist 4 um focused on the entry face, "
                               f"LUT 1 nm, restart 100; value = best time incl. preconditioner set-up for {head}"},
        "best_seconds_per_row": summary, "results": results,
        "paper_context": "CELES (paper, Table 1, GTX Titan X, single precision): N=1e4 vf 10 % 1096 s, vf 50 % "
                         "3463 s; N=2e4 vf 10 % 5663 s, vf 50 % 15951 s; packing (Lubachevsky-Stillinger) and "
                         "slab size differ, so this is context, not a like-for-like baseline"}))


def validation_mode(a):
    """The paper's validation target (Section 4): 2,500 spheres (R = 100 nm,
    n = 1.5) at volume fraction 10 % in a ball centred on the origin, Gaussian
    beam (waist 4 um, lambda = 532 nm) focused on the centre, lmax 3, LUT
    1 nm, solved to 1e-6 (block-diagonal preconditioner) once with TE and once
    with TM polarisation.  Reports the reflected and transmitted power
    fractions with the energy balance R + T + A - 1, and S11(theta) (far-field
    intensity averaged over both runs and the azimuth, S11(0) = 1)."""
    import numpy as np
    import torch
    import paper_1706_02145_amd as P
    from celes_inputs import workload

    t0 = time.perf_counter()

    def log(msg):
        print(f"[validation] {msg} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)

    w = workload("paper_ball2500_vf10")
    il = w.illumination
    log(f"{w.name} generated (N={w.N}, ball radius {w.extra['ball_radius']:.0f} nm)")
    runs, res = [], {}
    for name, alpha_G in (("TE", 0.0), ("TM", np.pi / 2)):
        p = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, hankel=P.CELES_HANKEL_LUT,
                      lut_dr=w.lut_dr, tol=w.tol, restart=100, maxiter=3000)
        p.set_gaussian_beam(il["waist"], il["focus"], alpha_G, il["E0"])
        p.build_preconditioner(a.cuboid_edge)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, info = p.solve()
        dt = time.perf_counter() - t1
        Pin, R, T, A = p.power_flux()[0]
        res[name] = {"seconds": dt, "iterations": info["iterations"], "rel_residual": info["rel_residual"],
                     "R": R, "T": T, "A": A, "energy_balance": R + T + A - 1.0}
        log(f"{name}: {info['iterations']} iterations, {dt:.2f} s; R {R:.4%} T {T:.4%} A {A:.2e} "
            f"R+T+A-1 {R + T + A - 1:.2e}")
        runs.append(p)
    theta_deg = np.arange(0, 181, 5)
    t1 = time.perf_counter()
    s11 = P.s11(runs, np.radians(theta_deg), n_phi=64)
    log(f"S11 at {theta_deg.size} angles x 64 azimuths x 2 runs in {time.perf_counter() - t1:.2f} s")
    # near-field map in the plane y = 0 (the paper's validation figure), points outside all spheres
    g = np.linspace(-1.5 * w.extra["ball_radius"], 1.5 * w.extra["ball_radius"], 201)
    pts = np.array([[x, 0.0, z] for z in g for x in g])
    dmin = np.full(len(pts), np.inf)
    for c0 in range(0, w.N, 500):
        dmin = np.minimum(dmin, (np.linalg.norm(pts[:, None, :] - w.positions[None, c0:c0 + 500], axis=-1)
                                 - w.radii[None, c0:c0 + 500]).min(axis=1))
    pts = pts[dmin > 0]
    t1 = time.perf_counter()
    E = runs[0].near_field(pts, add_incident=True)[0]
    t_nf = time.perf_counter() - t1
    log(f"near field (scattered + incident Gaussian beam) at {len(pts)} points in {t_nf:.2f} s, "
        f"max |E| {np.abs(E).max():.3f}")
    res["TE"]["near_field_points"] = int(len(pts))
    res["TE"]["near_field_seconds"] = t_nf
    print(json.dumps({
        "metric": "energy balance R + T + A - 1 of the validation target (TE and TM)",
        "value": max(abs(v["energy_balance"]) for v in res.values()), "unit": "relative",
        "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{w.name}: N={w.N}, R=100 nm, n=1.5, vf 0.10 in a ball of radius "
                               f"{w.extra['ball_radius']:.0f} nm (RSA), lambda=532 nm, lmax 3, Gaussian beam waist "
                               f"4 um focused on the centre, LUT 1 nm, tolerance {w.tol:g}, preconditioner cuboid "
                               f"edge {a.cuboid_edge:g} nm"},
        "results": res,
        "s11_theta_deg": theta_deg.tolist(), "s11_normalised": (s11 / s11[0]).tolist(),
        "paper_context": "paper (Section 4 validation, Lubachevsky-Stillinger packing, its own geometry): "
                         "R 16.25 %, T 83.73 %, R + T = 1 within 1e-3"}))


def large_mode(a):
    """The paper's large example (Section 4): 1e5 spheres (R = 100 nm,
    n = 1.5) at volume fraction 10 % in a ball (radius 10 um), Gaussian beam
    (waist 4 um, lambda = 532 nm) focused on the centre, lmax 3, LUT 1 nm,
    GMRES to 1e-4 in mixed precision without and with the block-diagonal
    preconditioner (a.large_cuboid spheres per cuboid); reflected and
    transmitted power fractions and the energy balance from the far field."""
    import numpy as np
    import torch
    import paper_1706_02145_amd as P
    from celes_inputs import workload

    t0 = time.perf_counter()

    def log(msg):
        print(f"[large] {msg} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)

    w = workload("paper_ball100000_vf10")
    il = w.illumination
    log(f"{w.name} generated (N={w.N}, ball radius {w.extra['ball_radius']:.0f} nm)")
    edge = (a.large_cuboid * 4.0 / 3.0 * np.pi * 100.0 ** 3 / 0.10) ** (1.0 / 3.0)
    res = {}
    for pre in [False, True][: 2 if a.large_cuboid > 0 else 1]:
        p = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, hankel=P.CELES_HANKEL_LUT,
                      lut_dr=w.lut_dr, precision=P.CELES_MIXED, tol=1e-4, inner_tol=1e-3, restart=100,
                      maxiter=3000, verbose=1)
        p.set_gaussian_beam(il["waist"], il["focus"], il["alpha_G"], il["E0"])
        t_pre = 0.0
        if pre:
            t1 = time.perf_counter()
            try:
                p.build_preconditioner(edge)
            except P.CelesError as e:
                log(f"preconditioner not built: {e}")
                res["mixed_preconditioned"] = {"error": str(e)}
                break
            torch.cuda.synchronize()
            t_pre = time.perf_counter() - t1
            log(f"preconditioner built ({edge:.0f} nm cuboids) in {t_pre:.1f} s")
        t1 = time.perf_counter()
        _, info = p.solve(check=False)
        dt = time.perf_counter() - t1
        t1 = time.perf_counter()
        Pin, R, T, A = p.power_flux()[0]
        t_pf = time.perf_counter() - t1
        key = "mixed" + ("_preconditioned" if pre else "")
        res[key] = {"seconds": dt, "preconditioner_setup_s": t_pre, "iterations": info["iterations"],
                    "matvecs": info["matvecs"], "rel_residual": info["rel_residual"], "status": info["status"],
                    "R": R, "T": T, "A": A, "energy_balance": R + T + A - 1.0, "power_flux_seconds": t_pf}
        log(f"{key}: {dt:.1f} s (+{t_pre:.1f} s set-up), {info['iterations']} iterations, residual "
            f"{info['rel_residual']:.2e}; R {R:.4%} T {T:.4%} A {A:.1e} R+T+A-1 {R + T + A - 1:.1e} "
            f"(power flux {t_pf:.1f} s)")
        p.close()
    ok = [v for v in res.values() if v.get("status") == 0]
    print(json.dumps({
        "metric": "time to solve the paper's 1e5-sphere example to 1e-4", "unit": "s",
        "value": min(v["seconds"] + v["preconditioner_setup_s"] for v in ok) if ok else None,
        "higher_is_better": False, "n_gpus": 1, "dtype": "f32 inner / f64 refinement", "data": "synthetic",
        "config": {"workload": f"{w.name}: N={w.N}, R=100 nm, n=1.5, vf 0.10 in a ball of radius "
                               f"{w.extra['ball_radius']:.0f} nm (RSA), lambda=532 nm, lmax 3, Gaussian beam waist "
                               f"4 um focused on the centre, LUT 1 nm, restart 100, preconditioner cuboid edge "
                               f"{edge:.0f} nm (~{a.large_cuboid} spheres)"},
        "results": res,
        "paper_context": "paper (Section 4, GTX Titan X, its own Lubachevsky-Stillinger aggregate): "
                         "3.15e5 s with the block-diagonal preconditioner, R 55.42 %, T 44.54 %"}))


def scaling_mode(a):
    """Convergence and run time against system size (the analogue of the
    paper's Figs. 4-5): the paper's setting (R = 100 nm, lambda = 532 nm,
    lmax 3, Gaussian beam, tolerance 1e-4) in cylindrical slabs of
    N = 2,500 ... 20,000 spheres at volume fractions 0.1, 0.3 and 0.5
    (--scaling-vfs; 0.5 packed by overlap relaxation), FP64 GMRES with and
    without the block-diagonal preconditioner of about 200 spheres per
    cuboid.  One JSON line per run, then a summary."""
    import numpy as np
    import torch
    import paper_1706_02145_amd as P
    from concurrent.futures import ProcessPoolExecutor

    t0 = time.perf_counter()
    rows = []
    vfs = [float(v) for v in a.scaling_vfs.split(",")]
    cases = [(n, vf) for vf in vfs for n in (2500, 5000, 10000, 20000)]
    with ProcessPoolExecutor(min(16, len(cases), os.cpu_count() or 1)) as ex:
        wls = dict(zip(cases, ex.map(_cyl_workload, cases)))
    print(f"[scaling] {len(wls)} geometries generated ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    for vf in vfs:
        edge = (200 * 4.0 / 3.0 * np.pi * 100.0 ** 3 / vf) ** (1.0 / 3.0)
        for n in (2500, 5000, 10000, 20000):
            w = wls[(n, vf)]
            il = w.illumination
            for pre in (False, True):
                p = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax,
                              hankel=P.CELES_HANKEL_LUT, tol=w.tol, restart=100, maxiter=5000, verbose=1)
                p.set_gaussian_beam(il["waist"], il["focus"], il["alpha_G"], il["E0"])
                t_pre = 0.0
                if pre:
                    t1 = time.perf_counter()
                    p.build_preconditioner(edge)
                    torch.cuda.synchronize()
                    t_pre = time.perf_counter() - t1
                t1 = time.perf_counter()
                _, info = p.solve()
                torch.cuda.synchronize()
                row = {"N": n, "vf": vf, "preconditioner": pre, "iterations": info["iterations"],
                       "seconds": time.perf_counter() - t1, "preconditioner_setup_s": t_pre,
                       "rel_residual": info["rel_residual"], "cuboid_edge_nm": edge if pre else None}
                rows.append(row)
                print(f"[scaling] {json.dumps(row)} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
                p.close()
    print(json.dumps({"metric": "GMRES iterations and solve time against N (paper setting, tolerance 1e-4)",
                      "unit": "s", "n_gpus": 1, "dtype": "f64", "data": "synthetic", "runs": rows}))


def warmstart_mode(a):
    """Learned initial guess (the custom initial condition of Section 4.2):
    train the network on solver output of a.train_slabs slabs (lmax 3,
    N = a.train_n each, vf 0.3, 2 um thick), evaluate on an unseen slab of
    a.eval_n spheres: GMRES iterations and time to residual 1e-6 from x0 = 0
    and from the network's prediction (and optionally from x0 = T a_in and a
    central sub-ensemble's solution), with and/or without the block-diagonal
    preconditioner.  Precision and translation scheme of all solves are
    options (default: mixed precision, rotation scheme)."""
    import numpy as np
    import torch
    import paper_1706_02145_amd as P
    from concurrent.futures import ProcessPoolExecutor
    tw = time.perf_counter()

    def log(msg):
        print(f"[warmstart] {msg} ({time.perf_counter() - tw:.1f} s)", file=sys.stderr, flush=True)

    prec = P.CELES_MIXED if a.ws_precision == "mixed" else P.CELES_FP64
    tr = P.CELES_TRANSLATION_ROTATE if a.ws_translation == "rotate" else P.CELES_TRANSLATION_DIRECT
    opts = dict(precision=prec, translation=tr, inner_tol=1e-3, hankel=P.CELES_HANKEL_LUT)
    net = P.Network(3, seed=11)
    ex = ProcessPoolExecutor(min(16, os.cpu_count() or 1))
    eval_geo = ex.submit(_realisation, (5000, a.eval_n))       # generated while the training data is solved
    t0 = time.perf_counter()
    n_train = 0
    for gi, (pos, rad) in enumerate(ex.map(_realisation, [(5001 + s, a.train_n) for s in range(a.train_slabs)])):
        q = P.Problem(pos, rad, 1.52, 1.0, 550.0, 3, tol=1e-6, restart=100, maxiter=4000, **opts)
        q.set_plane_waves([0.0], [0.0], [2])
        q.solve()
        net.add_training_problem(q)
        q.close()
        n_train += len(rad)
        if gi % 10 == 9:
            log(f"solved {gi + 1} training slabs")
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    loss = net.train(epochs=a.epochs, batch=2048, lr=2e-3, seed=3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"trained on {n_train} rows, loss {loss:.3e}")
    pos, rad = eval_geo.result()
    ex.shutdown()
    log(f"evaluation geometry ready (N={len(rad)})")
    p = P.Problem(pos, rad, 1.52, 1.0, 550.0, 3, tol=1e-6, restart=100, maxiter=6000, verbose=1, **opts)
    p.set_plane_waves([0.0], [0.0], [2])
    t1 = time.perf_counter()
    x_net = net.predict(p)
    t_pred = time.perf_counter() - t1
    guesses = {"zero": None, "network": x_net[None]}
    names = [g for g in a.ws_guesses.split(",") if g]
    if "T_a_in" in names:
        a_in = p.incident()
        tq = np.stack([P.mie_coefficients(3, 2 * np.pi / 550.0 * r, 1.52) for r in rad])   # [N][2][L]
        ls = [l for t in (0, 1) for l in range(1, 4) for m in range(-l, l + 1)]
        ts = [t for t in (0, 1) for l in range(1, 4) for m in range(-l, l + 1)]
        guesses["T_a_in"] = (tq[:, ts, [l - 1 for l in ls]] * a_in[0])[None]
    if "subsystem" in names:
        sub = np.nonzero(np.hypot(pos[:, 0], pos[:, 1]) < a.sub_radius)[0]
        t1 = time.perf_counter()
        x_sub, sub_info = p.subsystem_guess(sub, cuboid_edge=a.cuboid_edge)
        log(f"sub-ensemble guess: {sub.size} spheres, {sub_info['iterations']} iterations")
        guesses["subsystem"] = x_sub
    res = {}
    for pre in [v == "1" for v in a.ws_precond.split(",")]:
        if pre:
            t1 = time.perf_counter()
            info_pre = p.build_preconditioner(a.cuboid_edge)
            log(f"preconditioner {info_pre} in {time.perf_counter() - t1:.1f} s")
        else:
            p.build_preconditioner(0.0)
        for name in names:
            x0 = guesses[name]
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, info = p.solve(x0=x0)
            dt = time.perf_counter() - t1
            key = name + ("_preconditioned" if pre else "")
            res[key] = {"iterations": info["iterations"], "seconds": dt, "x0_used": info["x0_used"],
                        "initial_rel_residual": info["x0_residual"], "rel_residual": info["rel_residual"],
                        "refinements": info["refinements"]}
            log(f"x0 = {key}: {info['iterations']} iterations, {dt:.2f} s, initial residual "
                f"{info['x0_residual']:.3f}")
    gains = {}
    for key in res:
        if key.startswith("network") and key.replace("network", "zero") in res:
            z = res[key.replace("network", "zero")]
            gains[key] = {"iterations_saved": z["iterations"] - res[key]["iterations"],
                          "fraction_saved": 1 - res[key]["iterations"] / z["iterations"],
                          "time_ratio": res[key]["seconds"] / z["seconds"]}
    print(json.dumps({
        "metric": "GMRES iterations and time to residual 1e-6 with a learned initial guess",
        "value": res[[k for k in res if k.startswith("network")][0]]["seconds"], "unit": "s",
        "higher_is_better": False, "n_gpus": 1,
        "dtype": f"{a.ws_precision} solve ({a.ws_translation} scheme), bf16/f32 network", "data": "synthetic",
        "config": {"workload": f"train {a.train_slabs} slabs N={a.train_n}, evaluate N={a.eval_n}, lmax 3, "
                               f"vf 0.3, t=2 um, normal incidence x-pol, LUT 1 nm, restart 100, "
                               f"preconditioner edge {a.cuboid_edge:g} nm where used"},
        "results": res, "gains": gains, "training_loss": loss, "training_rows": n_train,
        "predict_seconds": t_pred, "data_generation_seconds": t_data, "training_seconds": t_train}))


def translation_mode(a):
    """Direct block evaluation against rotation-translation-rotation (Section
    5, Discussion) on one geometry (the 2,000-sphere slab) at lmax 1..6, FP64
    and complex64: kernel time per W.b (HIP events around the coupling
    kernel), algorithmic flops of the direct scheme, and the crossover."""
    import torch
    import paper_1706_02145_amd as P
    from celes_inputs import workload, random_coefficients
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = workload(a.workload if a.workload != "slab20000_l4" else "slab2000_l4")
    N = w.N
    stream = torch.cuda.current_stream()
    rows = []
    for L in [int(v) for v in a.translation_lmax.split(",")]:
        nm = 2 * L * (L + 2)
        row = {"lmax": L}
        x64 = torch.from_numpy(random_coefficients(7, 1, N, nm)[0]).to("cuda")
        for scheme, tr in (("direct", P.CELES_TRANSLATION_DIRECT), ("rotate", P.CELES_TRANSLATION_ROTATE)):
            p = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, L, lut_dr=w.lut_dr, translation=tr)
            for prec, xx in (("fp64", x64), ("fp32", x64.to(torch.complex64))):
                yy = torch.empty_like(xx)
                pr = P.CELES_FP64 if prec == "fp64" else P.CELES_MIXED
                p.apply_W(xx, yy, pr, stream=stream)
                torch.cuda.synchronize()
                p.kernel_timing(True)
                for _ in range(a.matvec_reps):
                    p.apply_W(xx, yy, pr, stream=stream)
                torch.cuda.synchronize()
                ms, _ = p.kernel_timing(False)
                row[f"{scheme}_{prec}_ms"] = ms
            p.close()
        row["direct_flops_per_pair"] = flops_per_pair(L)
        row["speedup_rotate_fp64"] = row["direct_fp64_ms"] / row["rotate_fp64_ms"]
        row["speedup_rotate_fp32"] = row["direct_fp32_ms"] / row["rotate_fp32_ms"]
        print(f"[translation] {row}", file=sys.stderr, flush=True)
        rows.append(row)

    def crossover(prec):
        for r in rows:
            if r[f"speedup_rotate_{prec}"] > 1.0:
                return r["lmax"]
        return None
    print(json.dumps({"metric": "coupling kernel time per W.b, direct vs rotation-translation-rotation",
                      "unit": "ms", "config": {"workload": f"{w.name} geometry (N={N}), LUT 1 nm, one right-hand side"},
                      "rows": rows, "crossover_lmax_fp64": crossover("fp64"),
                      "crossover_lmax_fp32": crossover("fp32")}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--matvec-reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", default="slab20000_l4")
    ap.add_argument("--small-workload", default="slab2000_l4", help="second workload ('' to skip)")
    ap.add_argument("--cuboid-edge", type=float, default=1500.0,
                    help="preconditioner cuboid edge in nm (-1: budgeted automatic edge, 0: none)")
    ap.add_argument("--hankel", choices=["lut", "direct"], default="lut")
    ap.add_argument("--profile", action="store_true", help="mat-vec launches only (for rocprofv3)")
    ap.add_argument("--profile-scheme", choices=["direct", "rotate"], default="direct",
                    help="profile mode: translation scheme of the timed mat-vecs")
    ap.add_argument("--translation-lmax", default="1,2,3,4,5,6", help="translation mode: cut-offs")
    ap.add_argument("--mode", choices=["solve", "batched", "warmstart", "mixed", "paper", "scaling", "validation",
                                       "large", "translation"],
                    default="solve")
    ap.add_argument("--mixed-workload", default="slab20000_l4")
    ap.add_argument("--paper-solvers", default="gmres", help="paper mode: comma-separated gmres,bicgstab")
    ap.add_argument("--paper-rows", default="10000:0.1,10000:0.5,20000:0.1,20000:0.5",
                    help="paper mode: comma-separated N:vf rows of Table 1")
    ap.add_argument("--realisations", type=int, default=32)
    ap.add_argument("--batch-tol", type=float, default=1e-6)
    ap.add_argument("--batch-maxiter", type=int, default=600)
    ap.add_argument("--batch-restart", type=int, default=150)
    ap.add_argument("--batch-no-solve", action="store_true", help="batched mode: mat-vec timings only")
    ap.add_argument("--batch-translation", choices=["rotate", "direct"], default="rotate",
                    help="batched mode: translation scheme of the persistent VALU mat-vec (the realisations)")
    ap.add_argument("--batch-precond", type=float, default=0.0,
                    help="batched mode: block-diagonal preconditioner cuboid edge (nm) for every problem, 0 = none")
    ap.add_argument("--train-slabs", type=int, default=200)
    ap.add_argument("--train-n", type=int, default=5000)
    ap.add_argument("--eval-n", type=int, default=100000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--large-cuboid", type=int, default=50,
                    help="large mode: spheres per preconditioner cuboid (0: no preconditioned run)")
    ap.add_argument("--scaling-vfs", default="0.1,0.3,0.5", help="scaling mode: volume fractions")
    ap.add_argument("--sub-radius", type=float, default=5000.0, help="warmstart: sub-ensemble radius (nm)")
    ap.add_argument("--ws-precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--ws-translation", choices=["rotate", "direct"], default="rotate")
    ap.add_argument("--ws-guesses", default="zero,network", help="warmstart: zero,network,T_a_in,subsystem")
    ap.add_argument("--ws-precond", default="0,1", help="warmstart: runs without (0) and with (1) preconditioner")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    if a.mode == "batched":
        return batched_mode(a)
    if a.mode == "warmstart":
        return warmstart_mode(a)
    if a.mode == "mixed":
        return mixed_mode(a)
    if a.mode == "paper":
        return paper_mode(a)
    if a.mode == "scaling":
        return scaling_mode(a)
    if a.mode == "validation":
        return validation_mode(a)
    if a.mode == "large":
        return large_mode(a)
    if a.mode == "translation":
        return translation_mode(a)

    import numpy as np
    import torch
    import paper_1706_02145_amd as P
    from celes_inputs import workload, random_coefficients

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t_start = time.perf_counter()

    def log(msg):
        print(f"[bench] {msg} ({time.perf_counter() - t_start:.1f} s)", file=sys.stderr, flush=True)

    w = workload(a.workload)
    log(f"{w.name} generated (N={w.N})")
    il = w.illumination
    N, L, nm = w.N, w.lmax, w.nmax
    updates_per_mv = N * (N - 1) * nm * nm
    hk = P.CELES_HANKEL_LUT if a.hankel == "lut" else P.CELES_HANKEL_DIRECT
    hmode = 0 if a.hankel == "lut" else 1

    def problem(wl, **kw):
        p = P.Problem(wl.positions, wl.radii, wl.n_sphere, wl.n0, wl.wavelength, wl.lmax, hankel=hk,
                      lut_dr=wl.lut_dr, **kw)
        ill = wl.illumination
        if ill["kind"] == "gaussian":
            p.set_gaussian_beam(ill["waist"], ill["focus"], ill["alpha_G"], ill["E0"])
        else:
            p.set_plane_waves([ill["beta"]], [ill["alpha"]], [ill["pol"]])
        return p

    t0 = time.perf_counter()
    p = problem(w, restart=100, maxiter=3000)
    t_setup = time.perf_counter() - t0
    if a.profile and a.profile_scheme == "rotate":
        p.set_solve_options(translation=P.CELES_TRANSLATION_ROTATE)
    stream = torch.cuda.current_stream()
    x = torch.from_numpy(random_coefficients(1, 1, N, nm)[0]).to("cuda")
    y = torch.empty_like(x)
    steps = a.steps if not a.profile else min(a.steps, 5)

    # ---- timed steps: one FP64 W.b each; the coupling kernel timed by HIP
    # events on its launch stream over the same launches ----
    for _ in range(a.warmup):
        p.apply_W(x, y, P.CELES_FP64, stream=stream)
    torch.cuda.synchronize()
    p.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        p.apply_W(x, y, P.CELES_FP64, stream=stream)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    kernel_ms, kernel_launches = p.kernel_timing(False)
    log(f"{steps} FP64 mat-vecs: {1e3 * t_steps / steps:.2f} ms each, kernel {kernel_ms:.2f} ms")
    if a.profile:
        # calibration copy of known size for the HBM byte counters
        src = torch.empty(64 * 2 ** 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"workload": w.name, "matvec_ms": 1e3 * t_steps / steps, "kernel_ms": kernel_ms, "N": N,
                          "lmax": L, "copy_bytes_each_way": src.numel() * 4}))
        return
    value = steps * updates_per_mv / t_steps
    fpp = flops_per_pair(L, a.hankel == "lut")
    fpp_exec = flops_per_pair_executed(L, KERNEL_GROUPS[L], a.hankel == "lut")
    mv_flops = fpp * N * (N - 1)
    achieved = mv_flops / (kernel_ms * 1e-3) / 1e12

    # the complex64 VALU kernel of the mixed path (one right-hand side), same problem
    x32 = x.to(torch.complex64)
    y32 = torch.empty_like(x32)
    p.apply_W(x32, y32, P.CELES_MIXED, stream=stream)
    torch.cuda.synchronize()
    p.kernel_timing(True)
    for _ in range(a.matvec_reps):
        p.apply_W(x32, y32, P.CELES_MIXED, stream=stream)
    torch.cuda.synchronize()
    k32_ms, _ = p.kernel_timing(False)
    log(f"complex64 kernel {k32_ms:.2f} ms")

    # ablation: the other Hankel evaluation mode on the same geometry
    other = "direct" if a.hankel == "lut" else "lut"
    q = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, L, lut_dr=w.lut_dr,
                  hankel=P.CELES_HANKEL_DIRECT if other == "direct" else P.CELES_HANKEL_LUT)
    q.apply_W(x, y, P.CELES_FP64, stream=stream)
    torch.cuda.synchronize()
    q.kernel_timing(True)
    for _ in range(a.matvec_reps):
        q.apply_W(x, y, P.CELES_FP64, stream=stream)
    torch.cuda.synchronize()
    other_kernel_ms, _ = q.kernel_timing(False)
    other_fpp = flops_per_pair(L, other == "lut")
    q.close()
    log(f"{other} Hankel kernel {other_kernel_ms:.2f} ms")
    traffic = measured_traffic(w.name, N, L, a.hankel)

    # the rotation-translation-rotation scheme on the same geometry and vector
    p.set_solve_options(translation=P.CELES_TRANSLATION_ROTATE)
    rot = {}
    for prec, xx, yy in (("fp64", x, y), ("fp32", x32, y32)):
        pr = P.CELES_FP64 if prec == "fp64" else P.CELES_MIXED
        p.apply_W(xx, yy, pr, stream=stream)
        torch.cuda.synchronize()
        p.kernel_timing(True)
        for _ in range(a.matvec_reps):
            p.apply_W(xx, yy, pr, stream=stream)
        torch.cuda.synchronize()
        rot[prec] = p.kernel_timing(False)[0]
    p.set_solve_options(translation=P.CELES_TRANSLATION_DIRECT)
    fpp_rot = flops_per_pair_rotate(L, a.hankel == "lut")
    rotate = {"kernel": f"wx_rtr_kernel<T, {L}, {hmode}> (rotation into the pair frame, translation along z, "
                        "rotation back)",
              "flops_per_pair": fpp_rot,
              "flops_per_pair_executed": flops_per_pair_rotate(L, a.hankel == "lut", executed=True)}
    for prec, peak in (("fp64", PEAK_FP64_VALU_TFLOPS), ("fp32", PEAK_FP32_VALU_TFLOPS)):
        rotate[prec] = {"kernel_ms": rot[prec], "updates_per_s": updates_per_mv / (rot[prec] * 1e-3),
                        "tflops": fpp_rot * N * (N - 1) / (rot[prec] * 1e-3) / 1e12,
                        "frac": fpp_rot * N * (N - 1) / (rot[prec] * 1e-3) / 1e12 / peak}
    log(f"rotation scheme kernels: FP64 {rot['fp64']:.2f} ms, complex64 {rot['fp32']:.2f} ms")

    # ---- time to residual 1e-6: FP64 vs mixed, one preconditioner for both ----
    ttr = {}
    t_pre, pre_info = 0.0, None
    if not a.no_mixed:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if a.cuboid_edge != 0:
            pre_info = p.build_preconditioner(a.cuboid_edge)
        torch.cuda.synchronize()
        t_pre = time.perf_counter() - t0
        log(f"preconditioner {pre_info} in {t_pre:.1f} s")
        for name, prec, tr in (("fp64", P.CELES_FP64, P.CELES_TRANSLATION_DIRECT),
                               ("mixed", P.CELES_MIXED, P.CELES_TRANSLATION_DIRECT),
                               ("fp64_rotate", P.CELES_FP64, P.CELES_TRANSLATION_ROTATE),
                               ("mixed_rotate", P.CELES_MIXED, P.CELES_TRANSLATION_ROTATE)):
            p.set_solve_options(tol=1e-6, precision=prec, restart=100, maxiter=3000, inner_tol=1e-3,
                                translation=tr)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, inf = p.solve()
            torch.cuda.synchronize()
            ttr[name] = {"seconds": time.perf_counter() - t1, "iterations": inf["iterations"],
                         "refinements": inf["refinements"], "matvec_seconds": inf["matvec_seconds"],
                         "rel_residual": inf["rel_residual"]}
            log(f"{name} to 1e-6: {ttr[name]['seconds']:.1f} s, {inf['iterations']} iterations")
        p.set_solve_options(translation=P.CELES_TRANSLATION_DIRECT)
        ttr["speedup_mixed_vs_fp64"] = ttr["fp64"]["seconds"] / ttr["mixed"]["seconds"]
        ttr["speedup_mixed_rotate_vs_fp64"] = ttr["fp64"]["seconds"] / ttr["mixed_rotate"]["seconds"]
        ttr["solve_seconds_exclude"] = "preconditioner set-up (preconditioner_setup_s)"

    # ---- the 2,000-sphere slab: preconditioned FP64 GMRES to 1e-8 ----
    small = None
    if a.small_workload:
        ws = workload(a.small_workload)
        ps = problem(ws, tol=ws.tol, restart=100, maxiter=3000)
        t0 = time.perf_counter()
        ps.build_preconditioner(1500.0)
        torch.cuda.synchronize()
        tps = time.perf_counter() - t0
        ps.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, inf = ps.solve()
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        xs_ = torch.from_numpy(random_coefficients(1, 1, ws.N, ws.nmax)[0]).to("cuda")
        ys_ = torch.empty_like(xs_)
        ps.apply_W(xs_, ys_, P.CELES_FP64, stream=stream)
        ps.kernel_timing(True)
        for _ in range(a.matvec_reps):
            ps.apply_W(xs_, ys_, P.CELES_FP64, stream=stream)
        torch.cuda.synchronize()
        kms, _ = ps.kernel_timing(False)
        upd = ws.N * (ws.N - 1) * ws.nmax ** 2
        small = {"workload": f"{ws.name}: N={ws.N}, lmax {ws.lmax}, Gaussian beam, cuboid edge 1500 nm",
                 "solve_to_1e-8_seconds": ts, "iterations": inf["iterations"], "matvecs": inf["matvecs"],
                 "rel_residual": inf["rel_residual"], "preconditioner_setup_s": tps,
                 "solve_updates_per_s": inf["matvecs"] * upd / ts, "kernel_ms": kms,
                 "kernel_frac": flops_per_pair(ws.lmax, a.hankel == "lut") * ws.N * (ws.N - 1) / (kms * 1e-3) / 1e12 /
                                PEAK_FP64_VALU_TFLOPS}
        ps.close()
        log(f"{ws.name} solve to 1e-8: {ts:.2f} s")

    # ---- CPU oracle on a bounded sample of receiver rows ----
    cpu = None
    if not a.no_cpu_baseline:
        k = 2 * math.pi * w.n0 / w.wavelength
        # one process per host core (the box's share: 16), each timing the
        # plain oracle on its own receiver rows for the same wall window
        ncore = min(16, os.cpu_count() or 1)
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(ncore) as ex:
            parts = list(ex.map(_oracle_rows_worker, [(w.positions, w.radii, k, L, w.lut_dr, r, ncore, a.cpu_seconds)
                                                      for r in range(ncore)]))
        rows = sum(r for r, _ in parts)
        t_cpu = max(t for _, t in parts)
        cpu = {"value": rows * (N - 1) * nm * nm / t_cpu, "unit": "updates/s", "cores": ncore, "kind": "oracle",
               "sample": f"{rows} of {N} receiver rows of one W.b (same geometry, LUT mode) in {t_cpu:.1f} s "
                         f"on {ncore} processes (numpy BLAS 1 thread each)"}
        log(f"CPU oracle: {rows} rows in {t_cpu:.1f} s")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * t_steps / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: N={N} RSA slab, radii lognormal(150 nm, 10%), n=1.52, vf 0.3, "
                               f"t={w.box[2] / 1000:g} um, lmax={L}, Gaussian beam w=2 um, lambda=550 nm, "
                               f"LUT dr=1 nm; step = one FP64 W.b (complex128)",
                   "N": N, "lmax": L, "hankel": a.hankel},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VALU_TFLOPS, "traffic": traffic},
        "cpu_baseline": cpu,
        "kernel": f"wx_fused_kernel<double, {L}, 1, {hmode}> (one launch = one W.b over all N(N-1) pairs)",
        "kernel_ms": kernel_ms, "kernel_launches_timed": kernel_launches,
        "flops_per_pair": fpp, "flops_per_pair_executed": fpp_exec,
        "kernel_tflops_executed": fpp_exec * N * (N - 1) / (kernel_ms * 1e-3) / 1e12,
        "fp32_kernel": {"kernel": f"wx_fused_kernel<float, {L}, 1, {hmode}> (complex64, the inner solves of the "
                                  "mixed path)", "kernel_ms": k32_ms,
                        "tflops": mv_flops / (k32_ms * 1e-3) / 1e12, "peak": PEAK_FP32_VALU_TFLOPS,
                        "frac": mv_flops / (k32_ms * 1e-3) / 1e12 / PEAK_FP32_VALU_TFLOPS,
                        "updates_per_s": updates_per_mv / (k32_ms * 1e-3)},
        "kernel_other_hankel": {"hankel": other, "kernel_ms": other_kernel_ms,
                                "frac": other_fpp * N * (N - 1) / (other_kernel_ms * 1e-3) / 1e12 /
                                        PEAK_FP64_VALU_TFLOPS},
        "rotate_scheme": rotate,
        "setup_s": t_setup,
        "preconditioner": None if pre_info is None else {"edge_nm": pre_info[0], "cuboids": pre_info[1],
                                                         "bytes": pre_info[2], "setup_s": t_pre},
        "time_to_residual_1e-6": ttr,
        "small_workload": small,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

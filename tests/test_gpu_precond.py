"""Block-diagonal preconditioner (Section 3.2.1) through the C ABI: y = P^{-1} x
element by element against the oracle's block LU solves, on a problem with
many cuboids of uneven size (all blocks), and on the 2,000-sphere benchmark
slab for sampled blocks (each block's master matrix built by the oracle from
the block's spheres alone); FP64 and the complex64 copy; state errors."""
import numpy as np
import pytest
import torch

import paper_1706_02145_amd as P
from celes_inputs import random_coefficients, workload
from oracle.solve import BlockDiagonalPreconditioner, master_matrix, partition, solve_dense
from tests.gpu_helpers import make_problem, rel

pytestmark = pytest.mark.gpu


def _apply(p, x, precision):
    dt = torch.complex128 if precision == P.CELES_FP64 else torch.complex64
    xd = torch.from_numpy(x).to("cuda", dt)
    yd = torch.empty_like(xd)
    p.apply_preconditioner(xd, yd, precision)
    torch.cuda.synchronize()
    return yd.cpu().numpy().astype(np.complex128)


def test_apply_matches_oracle_all_blocks():
    w = workload("slab300_l3")
    edge = 700.0
    perm, off = partition(w.positions, edge)
    sizes = np.diff(off)
    print(f"[precond] slab300_l3 edge {edge}: {sizes.size} blocks, sizes {sizes.min()}..{sizes.max()}", flush=True)
    assert sizes.size >= 8 and sizes.min() < sizes.max()
    M, W, t = master_matrix(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax)
    pre = BlockDiagonalPreconditioner(M, w.nmax, perm, off)
    x = random_coefficients(11, 1, w.N, w.nmax)[0]
    yref = pre(x.reshape(-1)).reshape(w.N, -1)
    p = make_problem(w, hankel=1)
    with pytest.raises(P.CelesError) as e:
        _apply(p, x, P.CELES_FP64)
    assert e.value.name == "CELES_E_STATE"
    p.build_preconditioner(edge)
    assert rel(_apply(p, x, P.CELES_FP64), yref) <= 1e-11
    assert rel(_apply(p, x, P.CELES_MIXED), yref) <= 1e-5


def test_apply_full_size_sampled_blocks():
    w = workload("slab2000_l4")
    edge = 1500.0
    perm, off = partition(w.positions, edge)
    sizes = np.diff(off)
    order = np.argsort(sizes, kind="stable")
    pick = [int(order[0]), int(order[1]), int(order[len(order) // 2])]
    print(f"[precond] slab2000_l4 edge {edge}: {sizes.size} blocks, sampled sizes {sizes[pick].tolist()}", flush=True)
    x = random_coefficients(12, 1, w.N, w.nmax)[0]
    p = make_problem(w, hankel=1)
    p.build_preconditioner(edge)
    y = _apply(p, x, P.CELES_FP64)
    for j in pick:
        sph = perm[off[j]:off[j + 1]]
        Mj, _, _ = master_matrix(w.positions[sph], w.radii[sph], w.n_sphere[sph], w.n0, w.wavelength, w.lmax)
        yj = solve_dense(Mj, x[sph].reshape(-1)).reshape(len(sph), -1)
        assert rel(y[sph], yj) <= 1e-11


def test_single_cuboid_preconditioner_is_the_exact_inverse():
    # one cuboid holds every sphere: P^{-1} = M^{-1}, so right-preconditioned
    # GMRES converges in one iteration; also fewer blocks than set-up streams
    w = workload("slab64_l3")
    print("[precond] slab64_l3 single cuboid", flush=True)
    p = make_problem(w, hankel=1, tol=1e-10)
    p.build_preconditioner(1e6)
    b, info = p.solve()
    assert info["status"] == 0 and info["iterations"] == 1
    M, W, t = master_matrix(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax)
    from tests.gpu_helpers import oracle_incident
    bref = solve_dense(M, t * oracle_incident(w).reshape(-1)).reshape(w.N, -1)
    assert rel(b[0], bref) <= 1e-10


@pytest.mark.timeout(400)
def test_complex64_copy_beyond_2_to_32_entries():
    # Regression: the complex64 copy of the inverses was written by a launch
    # with one work-item per entry; above 2^32 entries that exceeds what one
    # dispatch can address and most cuboids kept zero inverses.  The budgeted
    # edge for 100 spheres per cuboid on the 20,000-sphere slab gives 5.4e9
    # entries: every cuboid of the complex64 apply must match the FP64 apply.
    w = workload("slab20000_l4")
    p = make_problem(w, hankel=0, target_Nj=100.0)
    edge, nb, by = p.build_preconditioner()
    print(f"[precond] slab20000_l4 auto edge {edge:.0f} nm: {nb} cuboids, {by / 2**30:.1f} GiB", flush=True)
    perm, off = partition(w.positions, edge)
    sizes = np.diff(off).astype(np.float64)
    assert float(np.sum((sizes * w.nmax) ** 2)) > 2.0 ** 32
    x = random_coefficients(13, 1, w.N, w.nmax)[0]
    y64 = _apply(p, x, P.CELES_FP64)
    y32 = _apply(p, x, P.CELES_MIXED)
    # per cuboid: the last cuboids are the ones a wrapped launch would miss
    for j in (0, nb // 2, nb - 1):
        sph = perm[off[j]:off[j + 1]]
        assert rel(y32[sph], y64[sph]) <= 1e-5, j
    assert rel(y32, y64) <= 1e-5


@pytest.mark.parametrize("K", [3, 8, 11])
def test_apply_several_rhs_matches_oracle_and_single(K):
    # K right-hand sides through the grouped apply (each inverse tile read once
    # per group of eight): every column against the oracle's block LU solve and
    # against the one-right-hand-side apply; a ragged last group (K = 3, 11)
    w = workload("slab300_l3")
    edge = 700.0
    perm, off = partition(w.positions, edge)
    M, W, t = master_matrix(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax)
    pre = BlockDiagonalPreconditioner(M, w.nmax, perm, off)
    X = random_coefficients(30 + K, K, w.N, w.nmax)
    p = make_problem(w, hankel=1)
    p.build_preconditioner(edge)
    for prec, dt, bar in ((P.CELES_FP64, torch.complex128, 1e-11), (P.CELES_MIXED, torch.complex64, 1e-5)):
        xd = torch.from_numpy(X).to("cuda", dt)
        yd = torch.empty_like(xd)
        p.apply_preconditioner(xd, yd, prec, K=K)
        torch.cuda.synchronize()
        Y = yd.cpu().numpy().astype(np.complex128)
        for k in range(K):
            yref = pre(X[k].reshape(-1)).reshape(w.N, -1)
            assert rel(Y[k], yref) <= bar, (prec, k)
            assert rel(Y[k], _apply(p, X[k], prec)) <= (1e-13 if prec == P.CELES_FP64 else 1e-6)

"""Pins for the assembled problem: the single-sphere case reduces to the
textbook Mie series, the optical theorem holds with C_sca from an
independent far-field quadrature, lossless spheres absorb nothing, and the
reference GMRES (with and without the block-diagonal preconditioner) reaches
the LU solution."""
import math

import numpy as np

from celes_inputs import workload
from oracle.incident import plane_wave_coefficients, gaussian_beam_coefficients
from oracle.mie import bohren_huffman_ab
from oracle.observables import absorption, extinction, scattering_cross_section
from oracle.solve import (BlockDiagonalPreconditioner, gmres, master_matrix, partition,
                          solve_dense, wavenumber)


def _problem(w, hankel=None):
    k = wavenumber(w.n0, w.wavelength)
    M, W, t = master_matrix(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, hankel)
    il = w.illumination
    if il["kind"] == "plane":
        a = plane_wave_coefficients(w.positions, k, w.lmax, il["beta"], il["alpha"], il["pol"])
    else:
        a = gaussian_beam_coefficients(w.positions, k, w.lmax, il["waist"], il["focus"], il["alpha_G"])
    return k, M, W, t, a


def test_single_sphere_is_textbook_mie():
    k = 2 * math.pi / 550
    R, m, L = 100.0, 1.5 + 0.01j, 6
    pos = np.zeros((1, 3))
    M, W, t = master_matrix(pos, [R], [m], 1.0, 550.0, L)
    a = plane_wave_coefficients(pos, k, L, 0.0, 0.0, 2)
    b = solve_dense(M, t * a.reshape(-1))
    assert np.allclose(b, t * a.reshape(-1), atol=1e-15)
    an, bn = bohren_huffman_ab(L, k * R, m)
    n = np.arange(1, L + 1)
    cext = 2 * math.pi / k ** 2 * np.sum((2 * n + 1) * np.real(an + bn))
    csca = 2 * math.pi / k ** 2 * np.sum((2 * n + 1) * (np.abs(an) ** 2 + np.abs(bn) ** 2))
    assert abs(extinction(k, a, b) - cext) < 1e-12 * cext
    assert abs(scattering_cross_section(k, pos, b.reshape(1, -1), L) - csca) < 1e-12 * csca


def test_optical_theorem_cube8():
    w = workload("cube8_l3")
    k, M, W, t, a = _problem(w)
    rhs = t * a.reshape(-1)
    b = solve_dense(M, rhs)
    assert np.linalg.norm(M @ b - rhs) <= 1e-13 * np.linalg.norm(rhs)
    ce = extinction(k, a, b)
    ca = absorption(k, b, t)
    cs = scattering_cross_section(k, w.positions, b.reshape(w.N, -1), w.lmax)
    assert ca > 0
    assert abs(ce - cs - ca) <= 1e-10 * ce


def test_lossless_cluster_absorbs_nothing():
    rng = np.random.default_rng(2)
    pos = np.array([[0, 0, 0], [0, 0, 400.0], [350.0, 0, 100.0]])
    k = 2 * math.pi / 550
    M, W, t = master_matrix(pos, [100.0, 120.0, 90.0], [1.52] * 3, 1.0, 550.0, 3)
    a = plane_wave_coefficients(pos, k, 3, 0.4, 0.2, 1)
    b = solve_dense(M, t * a.reshape(-1))
    ce = extinction(k, a, b)
    assert abs(absorption(k, b, t)) < 1e-12 * ce
    cs = scattering_cross_section(k, pos, b.reshape(3, -1), 3)
    assert abs(ce - cs) < 1e-10 * ce


def test_gmres_and_preconditioner_reach_lu_solution():
    w = workload("slab64_l3")
    k, M, W, t, a = _problem(w)
    rhs = t * a.reshape(-1)
    b = solve_dense(M, rhs)
    x, its, _ = gmres(lambda v: M @ v, rhs, tol=1e-11, restart=60)
    assert np.linalg.norm(x - b) <= 1e-9 * np.linalg.norm(b)
    perm, off = partition(w.positions, 700.0)
    assert sorted(perm.tolist()) == list(range(w.N))
    P = BlockDiagonalPreconditioner(M, w.nmax, perm, off)
    xp, itp, _ = gmres(lambda v: M @ v, rhs, tol=1e-11, restart=60, precond=P)
    assert np.linalg.norm(xp - b) <= 1e-9 * np.linalg.norm(b)
    assert itp < its


def test_partition_blocks_are_cells():
    w = workload("slab64_l3")
    edge = 500.0
    perm, off = partition(w.positions, edge)
    lo = w.positions.min(axis=0)
    cells = np.floor((w.positions - lo) / edge).astype(int)
    for j in range(len(off) - 1):
        c = cells[perm[off[j]:off[j + 1]]]
        assert (c == c[0]).all()
        assert list(perm[off[j]:off[j + 1]]) == sorted(perm[off[j]:off[j + 1]])


def test_gmres_exact_in_n_steps_and_monotone_restarts():
    # GMRES minimises the residual over x0 + Krylov space: without restart it
    # is exact after n steps (up to rounding), and across restarts the true
    # residual can never increase (the previous iterate is in the search space).
    rng = np.random.default_rng(11)
    n = 40
    A = np.eye(n) + 0.4 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, its, _ = gmres(lambda v: A @ v, b, tol=1e-13, restart=n + 5)
    assert its <= n and np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    x, its, hist = gmres(lambda v: A @ v, b, tol=1e-12, restart=5, maxiter=2000)
    assert all(h2 <= h1 * (1 + 1e-12) for h1, h2 in zip(hist, hist[1:]))
    assert hist[-1] <= 1e-12

"""Pins for the oracle's BiCGSTAB (the alternative solver of Section 3.2),
each one fixed by mathematics other than the solver's own update formulas:

- Krylov termination: for a Hermitian positive definite matrix with d
  distinct eigenvalues and the shadow residual equal to the initial residual,
  BiCG coincides with CG and ends in d steps; BiCGSTAB's intermediate residual
  s carries BiCG's residual polynomial, so it vanishes at iteration d.  A wrong
  alpha or beta breaks this.
- omega minimises ||s - omega t|| over complex omega, so the squared updated
  residual equals ||s||^2 - |t^H s|^2 / ||t||^2 (Pythagoras).  A conjugated
  omega or a dropped term breaks it.
- Petrov-Galerkin condition of BiCG: s = psi_{i-1}(A) phi_i(A) r_0 with
  psi of degree i - 1 and phi_i orthogonal to the shadow Krylov space of
  dimension i, so r_tilde^H s = 0 at every iteration.  A conjugated rho or
  alpha breaks it.
- the updated residual equals the true residual rhs - M x after every
  iteration (up to rounding), which fixes the x update against the r update.
- on the master equation of a sphere cluster, with and without the
  block-diagonal preconditioner, the solution is the dense LU solution.
"""
import numpy as np
import pytest

from celes_inputs import workload
from oracle.incident import plane_wave_coefficients
from oracle.solve import (BlockDiagonalPreconditioner, bicgstab, master_matrix, partition, solve_dense,
                          wavenumber)


def _hpd_with_eigenvalues(lams, n, seed):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Q, _ = np.linalg.qr(Z)
    lam = np.resize(np.asarray(lams, dtype=float), n)
    return (Q * lam) @ Q.conj().T, rng


@pytest.mark.parametrize("lams", [[2.0], [1.0, 3.0], [1.0, 2.5, 6.0], [0.5, 1.0, 2.0, 4.0]])
def test_terminates_in_number_of_distinct_eigenvalues(lams):
    A, rng = _hpd_with_eigenvalues(lams, 24, seed=len(lams))
    rhs = rng.standard_normal(24) + 1j * rng.standard_normal(24)
    x, its, hist = bicgstab(lambda v: A @ v, rhs, tol=1e-11, maxiter=50)
    assert its <= len(lams)
    assert hist[-1] <= 1e-11
    assert np.linalg.norm(x - np.linalg.solve(A, rhs)) <= 1e-9 * np.linalg.norm(x)


def _master(name):
    w = workload(name)
    k = wavenumber(w.n0, w.wavelength)
    M, W, t = master_matrix(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax)
    il = w.illumination
    a = plane_wave_coefficients(w.positions, k, w.lmax, il["beta"], il["alpha"], il["pol"])
    return w, M, t * a.reshape(-1)


def test_omega_minimises_and_residual_recursion_is_true_residual():
    w, M, rhs = _master("cube8_l3")
    trace = []
    x, its, hist = bicgstab(lambda v: M @ v, rhs, tol=1e-12, maxiter=200, trace=trace)
    assert hist[-1] <= 1e-12 and len(trace) == its >= 3
    nb = np.linalg.norm(rhs)
    for st in trace:
        s, t, r = st["s"], st["t"], st["r"]
        if t is not None:
            ts = np.vdot(t, s)
            expect = np.linalg.norm(s) ** 2 - abs(ts) ** 2 / np.vdot(t, t).real
            assert abs(np.linalg.norm(r) ** 2 - expect) <= 1e-10 * np.linalg.norm(s) ** 2
            assert np.linalg.norm(r) <= np.linalg.norm(s) * (1 + 1e-12)
        rt = st["r_tilde"]
        assert abs(np.vdot(rt, s)) <= 1e-10 * np.linalg.norm(rt) * np.linalg.norm(s) + 1e-13 * nb ** 2
        true_r = rhs - M @ st["x"]
        assert np.linalg.norm(true_r - r) <= 1e-11 * nb


def test_matches_dense_lu_with_and_without_preconditioner():
    w, M, rhs = _master("slab64_l3")
    bref = solve_dense(M, rhs)
    x0, its0, h0 = bicgstab(lambda v: M @ v, rhs, tol=1e-11, maxiter=2000)
    perm, off = partition(w.positions, 700.0)
    pre = BlockDiagonalPreconditioner(M, M.shape[0] // w.N, perm, off)
    x1, its1, h1 = bicgstab(lambda v: M @ v, rhs, tol=1e-11, maxiter=2000, precond=pre)
    for x, h in ((x0, h0), (x1, h1)):
        assert h[-1] <= 1e-11
        assert np.linalg.norm(x - bref) <= 1e-9 * np.linalg.norm(bref)
    assert its1 < its0


def test_zero_rhs_and_exact_initial_guess():
    w, M, rhs = _master("cube8_l3")
    x, its, hist = bicgstab(lambda v: M @ v, np.zeros_like(rhs))
    assert its == 0 and not np.any(x)
    b = solve_dense(M, rhs)
    x, its, hist = bicgstab(lambda v: M @ v, rhs, tol=1e-10, x0=b)
    assert its == 0 and hist[0] <= 1e-12

"""Pins for the sub-ensemble initial guess (Section 4.2's custom initial
condition): the whole ensemble as sub-ensemble gives the exact solution; the
sub-ensemble's master matrix is the principal sub-matrix of the full one
(couplings depend on sphere pairs only); for two clusters far apart, the
guess from one cluster matches the full solution there with an error that
falls like the inverse separation (the far-field decay of the coupling)."""
import numpy as np

from celes_inputs import workload
from oracle.incident import plane_wave_coefficients
from oracle.solve import master_matrix, solve_dense, subsystem_initial_guess, wavenumber


def _full(pos, radii, ns, w):
    k = wavenumber(w.n0, w.wavelength)
    M, W, t = master_matrix(pos, radii, ns, w.n0, w.wavelength, w.lmax)
    a = plane_wave_coefficients(pos, k, w.lmax, 0.3, 0.2, 2)
    return M, t, a, solve_dense(M, t * a.reshape(-1)).reshape(len(pos), -1)


def test_whole_ensemble_gives_the_solution():
    w = workload("cube8_l3")
    M, t, a, b = _full(w.positions, w.radii, w.n_sphere, w)
    x0 = subsystem_initial_guess(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, a, np.arange(w.N))
    assert np.linalg.norm(x0 - b) <= 1e-12 * np.linalg.norm(b)


def test_sub_master_matrix_is_principal_submatrix():
    w = workload("cube8_l3")
    idx = np.array([6, 1, 3])
    M, _, _ = master_matrix(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax)
    Ms, _, _ = master_matrix(w.positions[idx], w.radii[idx], w.n_sphere[idx], w.n0, w.wavelength, w.lmax)
    nm = w.nmax
    ix = (idx[:, None] * nm + np.arange(nm)[None, :]).reshape(-1)
    assert np.array_equal(Ms, M[np.ix_(ix, ix)])


def test_distant_cluster_error_falls_with_separation():
    w = workload("cube8_l3")
    errs = []
    for sep in (2e5, 2e6):
        pos = np.concatenate([w.positions, w.positions + np.array([sep, 0.0, 0.0])])
        radii = np.concatenate([w.radii, w.radii])
        ns = np.concatenate([w.n_sphere, w.n_sphere])
        M, t, a, b = _full(pos, radii, ns, w)
        idx = np.arange(w.N, 2 * w.N)     # the displaced cluster: its own rows of a_in
        x0 = subsystem_initial_guess(pos, radii, ns, w.n0, w.wavelength, w.lmax, a, idx)
        assert not np.any(x0[:w.N])
        errs.append(np.linalg.norm(x0[idx] - b[idx]) / np.linalg.norm(b[idx]))
    assert errs[0] < 1e-3
    assert 5.0 < errs[0] / errs[1] < 20.0

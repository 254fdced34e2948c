"""Phase-function element S11 (TE/TM-averaged far-field intensity, the
paper's validation observable) through the C ABI: one sphere against the
textbook Mie amplitudes, a cluster against the oracle evaluated on the
oracle's own dense-LU solutions, one two-wave problem against two one-wave
problems, and the missing-solution error."""
import math

import numpy as np
import pytest

import paper_1706_02145_amd as P
from celes_inputs import workload
from oracle.incident import plane_wave_coefficients
from oracle.mie import bohren_huffman_S1_S2
from oracle.observables import phase_function_s11
from oracle.solve import master_matrix, solve_dense
from tests.gpu_helpers import k_of

pytestmark = pytest.mark.gpu


def test_single_sphere_s11_is_textbook_mie():
    print("[s11] single sphere", flush=True)
    R, m, L, lam = 250.0, 1.5 + 0.02j, 6, 550.0
    p = P.Problem(np.zeros((1, 3)), [R], m, 1.0, lam, L, hankel=P.CELES_HANKEL_DIRECT, tol=1e-12)
    p.set_plane_waves([0.0, 0.0], [0.0, 0.0], [1, 2])
    p.solve()
    theta = np.linspace(0.0, math.pi, 61)
    s = P.s11([p], theta, n_phi=4)
    S1, S2 = bohren_huffman_S1_S2(L, 2 * math.pi / lam * R, m, theta)
    ref = 0.5 * (np.abs(S1) ** 2 + np.abs(S2) ** 2)
    assert np.allclose(s, ref, rtol=1e-9, atol=1e-13 * ref.max())


def test_cluster_s11_matches_oracle_and_run_split():
    w = workload("slab64_l3")
    print("[s11] slab64_l3 TE/TM", flush=True)
    k = k_of(w)
    beta, alpha = 0.3, 0.7
    M, W, t = master_matrix(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax)
    runs = [solve_dense(M, t * plane_wave_coefficients(w.positions, k, w.lmax, beta, alpha, pol).reshape(-1))
            .reshape(w.N, -1) for pol in (1, 2)]
    theta = np.linspace(0.0, math.pi, 25)
    ref = phase_function_s11(k, w.positions, runs, w.lmax, theta, n_phi=16)
    both = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, hankel=P.CELES_HANKEL_DIRECT,
                     tol=1e-11)
    both.set_plane_waves([beta, beta], [alpha, alpha], [1, 2])
    both.solve()
    s_both = P.s11([both], theta, n_phi=16)
    assert np.max(np.abs(s_both - ref) / ref.max()) <= 1e-9
    single = []
    for pol in (1, 2):
        q = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, hankel=P.CELES_HANKEL_DIRECT,
                      tol=1e-11)
        q.set_plane_waves([beta], [alpha], [pol])
        q.solve()
        single.append(q)
    s_split = P.s11(single, theta, n_phi=16)
    assert np.max(np.abs(s_split - s_both) / s_both.max()) <= 1e-9
    fresh = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax)
    fresh.set_plane_waves([beta], [alpha], [1])
    with pytest.raises(P.CelesError) as e:
        P.s11([both, fresh], theta)
    assert e.value.name == "CELES_E_STATE"


def test_far_field_sums_many_spheres_sampled_directions():
    # the device sphere sums against the oracle's far field on the same
    # coefficients (the library's own solution), 2,000 spheres, lmax 4
    from oracle.observables import far_field
    from tests.gpu_helpers import make_problem
    w = workload("slab2000_l4")
    print("[s11] slab2000_l4 far field, sampled directions", flush=True)
    p = make_problem(w, tol=1e-4)
    b, _ = p.solve()
    rng = np.random.default_rng(5)
    theta = np.concatenate([[0.0, math.pi, math.pi / 2], np.arccos(rng.uniform(-1, 1, 21))])
    phi = rng.uniform(0, 2 * math.pi, theta.size)
    F = p.far_field(theta, phi)[0]
    ref = far_field(k_of(w), w.positions, b[0], w.lmax, theta, phi)
    assert np.max(np.abs(F - ref)) <= 1e-11 * np.max(np.abs(ref))

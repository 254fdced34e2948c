"""Pins for the phase-function element S11 (far-field intensity averaged over
TE and TM incidence, the paper's validation observable).  For one sphere
under x- and y-polarised plane waves along +z the average is the textbook
unpolarised result (|S1|^2 + |S2|^2) / 2 of Bohren & Huffman at every
direction, computed from an independent series (their angular functions and
Mie coefficients); integrating it over the sphere gives k^2 times the mean
scattering cross section."""
import math

import numpy as np
import pytest

from oracle.incident import plane_wave_coefficients
from oracle.mie import T_vector, bohren_huffman_S1_S2
from oracle.observables import phase_function_s11, scattering_cross_section


@pytest.mark.parametrize("R,m", [(80.0, 1.5), (200.0, 1.33 + 0.05j), (350.0, 2.0 + 0.1j)])
def test_single_sphere_s11_is_textbook(R, m):
    lam, L = 550.0, 12
    k = 2 * math.pi / lam
    pos = np.zeros((1, 3))
    t = T_vector(L, k, [R], [m])
    runs = [t * plane_wave_coefficients(pos, k, L, 0.0, 0.0, pol) for pol in (1, 2)]
    theta = np.linspace(0.0, math.pi, 37)
    s11 = phase_function_s11(k, pos, runs, L, theta, n_phi=5)
    S1, S2 = bohren_huffman_S1_S2(L, k * R, m, theta)
    ref = 0.5 * (np.abs(S1) ** 2 + np.abs(S2) ** 2)
    assert np.allclose(s11, ref, rtol=1e-10, atol=1e-14 * ref.max())


def test_cluster_s11_integrates_to_scattering_cross_section():
    from celes_inputs import workload
    from oracle.solve import master_matrix, solve_dense
    w = workload("cube8_l3")
    k = 2 * math.pi * w.n0 / w.wavelength
    M, W, t = master_matrix(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax)
    runs = []
    for pol in (1, 2):
        a = plane_wave_coefficients(w.positions, k, w.lmax, 0.4, 1.0, pol)
        runs.append(solve_dense(M, t * a.reshape(-1)).reshape(w.N, -1))
    x, wq = np.polynomial.legendre.leggauss(40)
    s11 = phase_function_s11(k, w.positions, runs, w.lmax, np.arccos(x), n_phi=48)
    integral = 2 * math.pi * np.sum(wq * s11) / k ** 2
    csca = np.mean([scattering_cross_section(k, w.positions, b, w.lmax) for b in runs])
    assert abs(integral - csca) <= 1e-9 * csca

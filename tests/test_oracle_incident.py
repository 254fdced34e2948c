"""Pins for the initial-field coefficients: the expanded field must reproduce
the plane wave itself, and the Gaussian-beam coefficients must reproduce a
direct angular-spectrum quadrature of the beam (no Bessel identity)."""
import math

import numpy as np
import pytest

from oracle.incident import gaussian_beam_coefficients, gaussian_beam_field, plane_wave_coefficients
from oracle.svwf import pvwf, svwf
from oracle.translation import multi_indices


@pytest.mark.parametrize("beta,alpha,pol", [(0.0, 0.0, 2), (0.0, 0.0, 1), (0.7, 1.1, 1),
                                            (2.0, -0.4, 2), (math.pi, 0.3, 1)])
def test_plane_wave_expansion_reproduces_field(beta, alpha, pol):
    k = 2 * math.pi / 550
    L = 22
    ri = np.array([[120.0, -80.0, 300.0]])
    pts = ri + np.random.default_rng(0).uniform(-60, 60, (6, 3))
    a = plane_wave_coefficients(ri, k, L, beta, alpha, pol)[0]
    E = sum(a[c] * svwf(1, t, l, m, pts - ri, k) for c, (t, l, m) in enumerate(multi_indices(L)))
    assert np.abs(E - pvwf(pol, alpha, beta, pts, k)).max() < 1e-12


def test_normal_incidence_coefficient_magnitudes():
    k = 2 * math.pi / 550
    a = plane_wave_coefficients(np.zeros((1, 3)), k, 4, 0.0, 0.0, 2)[0]
    for c, (t, l, m) in enumerate(multi_indices(4)):
        want = 2 * l + 1 if abs(m) == 1 else 0.0
        assert abs(abs(a[c]) ** 2 - want) < 1e-12


def test_gaussian_coefficients_reproduce_angular_spectrum():
    k = 2 * math.pi / 550
    L = 14
    w = 1000.0
    focus = np.array([30.0, -20.0, -100.0])
    aG = -math.pi / 2
    ri = np.array([[400.0, -250.0, 300.0]])
    pts = ri + np.random.default_rng(0).uniform(-50, 50, (3, 3))
    a = gaussian_beam_coefficients(ri, k, L, w, focus, aG, n_beta=256)[0]
    E = sum(a[c] * svwf(1, t, l, m, pts - ri, k) for c, (t, l, m) in enumerate(multi_indices(L)))
    Ed = gaussian_beam_field(pts, k, w, focus, aG, n_beta=200, n_alpha=96)
    assert np.abs(E - Ed).max() < 1e-11 * np.abs(Ed).max()

"""Pins for oracle.special: normalization, parity, closed forms, pole limits,
and the spherical Hankel function against mpmath at 30 digits."""
import math

import mpmath
import numpy as np
import pytest

from oracle.special import legendre, pi_tau, sph_h1


def test_legendre_normalized_orthonormal():
    x, w = np.polynomial.legendre.leggauss(64)
    for m in range(0, 7):
        for l in range(m, 9):
            for l2 in range(m, 9):
                v = np.sum(w * legendre(l, m, x) * legendre(l2, m, x))
                assert abs(v - (1.0 if l == l2 else 0.0)) < 1e-13


def test_legendre_closed_forms_and_parity():
    x = np.linspace(-0.99, 0.99, 17)
    s = np.sqrt(1 - x * x)
    assert np.allclose(legendre(0, 0, x), 1 / math.sqrt(2), atol=1e-15)
    assert np.allclose(legendre(1, 1, x), math.sqrt(3) / 2 * s, atol=1e-15)   # no CS phase
    assert np.allclose(legendre(2, 0, x), math.sqrt(5 / 2) * (3 * x * x - 1) / 2, atol=1e-15)
    assert np.allclose(legendre(2, 2, x), math.sqrt(15) / 4 * s * s, atol=1e-15)
    for l in range(0, 8):
        for m in range(0, l + 1):
            assert np.allclose(legendre(l, m, -x), (-1) ** (l + m) * legendre(l, m, x), atol=1e-13)


def test_pi_tau_against_definitions():
    th = np.linspace(0.05, math.pi - 0.05, 23)
    h = 1e-6
    for l in range(1, 7):
        for m in range(0, l + 1):
            pi, tau = pi_tau(l, m, th)
            if m > 0:   # pi_l^0 is only ever used multiplied by m = 0
                assert np.allclose(pi * np.sin(th), legendre(l, m, np.cos(th)), atol=1e-13)
            fd = (legendre(l, m, np.cos(th + h)) - legendre(l, m, np.cos(th - h))) / (2 * h)
            assert np.allclose(tau, fd, atol=1e-7)


@pytest.mark.parametrize("pole", [0.0, math.pi])
def test_pi_tau_pole_limits(pole):
    eps = 1e-7
    th = eps if pole == 0.0 else math.pi - eps
    for l in range(1, 7):
        for m in range(0, l + 1):
            p0, t0 = pi_tau(l, m, pole)
            p1, t1 = pi_tau(l, m, th)
            # pi_l^0 diverges at the poles but only ever appears multiplied by m = 0
            assert m == 0 or abs(p0 - p1) < 1e-5
            assert abs(t0 - t1) < 1e-5


def test_hankel_against_mpmath():
    mpmath.mp.dps = 30
    for l in range(0, 10):
        for x in (0.3, 1.7, 5.0, 33.3):
            j = mpmath.sqrt(mpmath.pi / (2 * x)) * mpmath.besselj(l + 0.5, x)
            y = mpmath.sqrt(mpmath.pi / (2 * x)) * mpmath.bessely(l + 0.5, x)
            ref = complex(j, y)
            got = sph_h1(l, x)
            assert abs(got - ref) <= 1e-13 * abs(ref)

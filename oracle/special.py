"""Special functions used by the vector wave functions (paper, Appendix A.1).

Conventions (pinned by the SVWF addition theorem test):
  * P_l^m denotes the *normalized* associated Legendre function
        P_l^m(x) = sqrt((2l+1)/2 * (l-m)!/(l+m)!) (1-x^2)^{m/2} d^m/dx^m P_l(x),
    m >= 0, without the Condon-Shortley phase (so that int_{-1}^{1} P^2 = 1).
  * pi_l^m(theta) = P_l^m(cos theta) / sin theta,
    tau_l^m(theta) = d/dtheta P_l^m(cos theta)   (Appendix A.1).
  * z_l^(1) = j_l, z_l^(3) = h_l^(1) = j_l + i y_l.
"""
from math import factorial, sqrt

import numpy as np
from numpy.polynomial.legendre import Legendre
from scipy.special import spherical_jn, spherical_yn


def norm_lm(l, m):
    """Normalization factor sqrt((2l+1)/2 (l-m)!/(l+m)!)."""
    return sqrt((2 * l + 1) / 2.0 * factorial(l - m) / factorial(l + m))


def _dmPl(l, m, x):
    """d^m P_l(x) / dx^m (a polynomial; numpy's Legendre series derivative)."""
    if m > l:
        return np.zeros_like(x)
    return Legendre.basis(l).deriv(m)(x) if m > 0 else Legendre.basis(l)(x)


def legendre(l, m, x, s=None):
    """Normalized associated Legendre function P_l^m(x), m >= 0, without the
    Condon-Shortley phase: N_lm (1-x^2)^{m/2} d^m P_l/dx^m.  Pass s = sin(theta)
    (>= 0) when it is known, so that (1-x^2)^{1/2} is not recomputed from x
    (which loses accuracy near the poles)."""
    m = abs(m)
    x = np.asarray(x, dtype=np.float64)
    if m > l:
        return np.zeros_like(x)
    if s is None:
        s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    return norm_lm(l, m) * s ** m * _dmPl(l, m, x)


def pi_tau(l, m, theta):
    """pi_l^m(theta) = P_l^m(cos theta)/sin theta and tau_l^m(theta) =
    d/dtheta P_l^m(cos theta) for m >= 0 (Appendix A.1).  Written with
    P_l^m(cos t) = N sin^m(t) Q(cos t), Q = d^m P_l/dx^m:
        pi  = N sin^{m-1}(t) Q(cos t)                        (m >= 1; 0 for m = 0)
        tau = N [m sin^{m-1}(t) cos(t) Q(cos t) - sin^{m+1}(t) Q'(cos t)]
    which are exact at the poles as well."""
    m = abs(m)
    th = np.asarray(theta, dtype=np.float64)
    x, s = np.cos(th), np.abs(np.sin(th))
    N = norm_lm(l, m)
    Q = _dmPl(l, m, x)
    Qd = _dmPl(l, m + 1, x)
    if m == 0:
        pi = np.zeros_like(x)
        tau = -N * s * Qd
    else:
        pi = N * s ** (m - 1) * Q
        tau = N * (m * s ** (m - 1) * x * Q - s ** (m + 1) * Qd)
    return pi, tau


def sph_jn(l, z):
    return spherical_jn(l, z)


def sph_yn(l, z):
    return spherical_yn(l, z)


def sph_h1(l, x):
    """Spherical Hankel function of the first kind, h_l = j_l + i y_l."""
    return spherical_jn(l, x) + 1j * spherical_yn(l, x)


def sph_h1_deriv(l, x):
    return spherical_jn(l, x, derivative=True) + 1j * spherical_yn(l, x, derivative=True)


def radial(nu, l, x):
    """z_l^(nu)(x) and d/dx [x z_l^(nu)(x)] for nu = 1 (j_l) or 3 (h_l)."""
    if nu == 1:
        z = spherical_jn(l, x)
        dz = spherical_jn(l, x, derivative=True)
    elif nu == 3:
        z = sph_h1(l, x)
        dz = sph_h1_deriv(l, x)
    else:
        raise ValueError("nu must be 1 or 3")
    return z, z + x * dz

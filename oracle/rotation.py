"""Rotation of the SVWF basis and the rotation-translation-rotation form of
the translation operator.

Test infrastructure: the plain reference the library is checked against,
never called by the library.

The paper's Discussion (Section 5) names rotating the coordinate frame so
that the translation runs along z as the way to bring the translation cost
from O(lmax^4) down to O(lmax^3).  This module states that factorisation for
this oracle's normalisation (reading R1: angular functions
e^{i m phi} P_l^{|m|}(cos theta) with the normalised Legendre functions of
Appendix A.1, no Condon-Shortley phase).

Wigner's small-d function (the definition, Wigner's explicit sum),
  d^l_{m m'}(beta) = sum_k (-1)^{m'-m+k} sqrt((l+m')!(l-m')!(l+m)!(l-m)!)
                     / ((l+m-k)! k! (m'-m+k)! (l-m'-k)!)
                     cos(beta/2)^{2l+m-m'-2k} sin(beta/2)^{m'-m+2k},
is evaluated in 40-digit arithmetic: the alternating sum cancels badly in
double precision once l exceeds about 10.

Basis rotation.  For the rotation R = R_z(phi) R_y(theta), which takes the z
axis to the direction (theta, phi),
  U^l_{m m''}(phi, theta) = e^{i m phi} c_m c_{m''} d^l_{m m''}(theta),
  c_m = (-1)^m for m > 0 and 1 otherwise
(c_m converts the Condon-Shortley harmonics, for which the d-matrix is the
standard one, to the normalisation used here).  The angular functions obey
f_l(R u) = U^l f_l(u), f_l = (f_{l,-l}, ..., f_{l,l}): the rotation theorem
that the tests check point by point.  U acts within each (tau, l) block.

Translation.  With d = |d| (sin theta cos phi, sin theta sin phi, cos theta),
  A(d) = U(phi, theta) A(|d| z) U(phi, theta)^H,
where A(|d| z) is the translation along +z, which couples only equal m
(Appendix A.2 at theta = 0, where P_p^mu(1) = 0 for mu > 0).
"""
from functools import lru_cache
from math import factorial

import mpmath
import numpy as np

from .translation import idx, nmax_of, translation_matrix

mpmath.mp.dps = 40


@lru_cache(maxsize=None)
def _d_terms(l, m, mp):
    """(coefficient, power of cos, power of sin) of Wigner's sum, exact."""
    out = []
    pre = factorial(l + mp) * factorial(l - mp) * factorial(l + m) * factorial(l - m)
    for k in range(0, 2 * l + 1):
        a, b, c = l + m - k, mp - m + k, l - mp - k
        if a < 0 or b < 0 or c < 0:
            continue
        den = factorial(a) * factorial(k) * factorial(b) * factorial(c)
        out.append(((-1) ** (mp - m + k), pre, den, 2 * l + m - mp - 2 * k, mp - m + 2 * k))
    return tuple(out)


def wigner_small_d(l, mp, m, beta):
    """d^l_{m' m}(beta), Wigner's explicit sum in 40-digit arithmetic."""
    c = mpmath.cos(mpmath.mpf(beta) / 2)
    s = mpmath.sin(mpmath.mpf(beta) / 2)
    tot = mpmath.mpf(0)
    for sign, pre, den, pc, ps in _d_terms(l, m, mp):
        tot += sign * mpmath.sqrt(mpmath.mpf(pre)) / den * c ** pc * s ** ps
    return float(tot)


def _c(m):
    return -1.0 if (m > 0 and m % 2) else 1.0


def basis_rotation_l(l, phi, theta):
    """U^l(phi, theta), [2l+1, 2l+1], rows and columns m = -l..l."""
    ms = range(-l, l + 1)
    return np.array([[np.exp(1j * m * phi) * _c(m) * _c(m2) * wigner_small_d(l, m, m2, theta) for m2 in ms]
                     for m in ms])


def basis_rotation(L, phi, theta):
    """Block-diagonal U over (tau, l) in the multi-index order, [nmax, nmax]."""
    nm = nmax_of(L)
    U = np.zeros((nm, nm), dtype=np.complex128)
    for l in range(1, L + 1):
        block = basis_rotation_l(l, phi, theta)
        for tau in (1, 2):
            s = idx(tau, l, -l, L)          # the (tau, l) block is contiguous, m = -l..l
            U[s:s + 2 * l + 1, s:s + 2 * l + 1] = block
    return U


def pair_angles(d):
    """(|d|, theta, phi) of a displacement; phi = 0 on the z axis."""
    d = np.asarray(d, dtype=np.float64)
    r = float(np.sqrt(np.sum(d * d)))
    rho = float(np.hypot(d[0], d[1]))
    theta = float(np.arctan2(rho, d[2]))
    phi = float(np.arctan2(d[1], d[0])) if rho > 0 else 0.0
    return r, theta, phi


def translation_matrix_rtr(d, k, L, hankel=None, Lrow=None):
    """A(d) as rotation, translation along z, rotation back:
    U(phi, theta) A(|d| z) U(phi, theta)^H (rows l > Lrow zero when Lrow < L)."""
    r, theta, phi = pair_angles(d)
    Az = translation_matrix(np.array([0.0, 0.0, r]), k, L, hankel, Lrow)
    U = basis_rotation(L, phi, theta)
    return U @ Az @ U.conj().T

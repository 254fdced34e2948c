"""Observables from the scattered-field coefficients (paper, Appendix D and
the SVWF definitions of Appendix A.1).

With unit incident amplitude (E0 = 1) and background wavenumber k:
  extinction   C_ext = -(pi/k^2) Re sum_{i,n} conj(a_in) b
  absorption   C_abs = -(pi/k^2) sum_{i,n} |b|^2 (Re(1/Q) + 1)
  scattering   C_sca = (1/k^2) oint |F|^2 dOmega, E_sca -> e^{ikr}/(kr) F(theta, phi),
  F = sum_i e^{-ik rhat.r_i} sum_n b_n^i f_n,
  f_{1lm} = (-i)^{l+1} (2l(l+1))^{-1/2} e^{im phi} (i m pi e_theta - tau e_phi)
  f_{2lm} = (-i)^{l}   (2l(l+1))^{-1/2} e^{im phi} (tau e_theta + i m pi e_phi)
(the large-argument limits h_l(x) -> (-i)^{l+1} e^{ix}/x and
d(x h_l)/dx / x -> (-i)^l e^{ix}/x applied to the SVWFs).
C_sca is evaluated by quadrature, independently of W, so that the optical
theorem C_ext = C_sca + C_abs checks the whole solve.
"""
import numpy as np

from .special import pi_tau
from .svwf import svwf
from .translation import multi_indices


def extinction(k, a_in, b):
    return -np.pi / k ** 2 * np.real(np.vdot(a_in.reshape(-1), b.reshape(-1)))


def absorption(k, b, tvec):
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(tvec != 0, np.real(1.0 / tvec) + 1.0, 0.0)
    return -np.pi / k ** 2 * float(np.sum(np.abs(b) ** 2 * f))


def far_field(k, pos, b, L, theta, phi):
    """F(theta, phi) as cartesian 3-vectors [ndir, 3] for coefficients b [N, nmax]."""
    theta = np.atleast_1d(theta)
    phi = np.atleast_1d(phi)
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    rhat = np.stack([st * cp, st * sp, ct], -1)
    et = np.stack([ct * cp, ct * sp, -st], -1)
    ep = np.stack([-sp, cp, np.zeros_like(phi)], -1)
    ph = np.exp(-1j * k * (rhat @ np.asarray(pos).T))          # [ndir, N]
    coef = ph @ b                                               # [ndir, nmax]
    F = np.zeros((theta.size, 3), dtype=np.complex128)
    for c, (tau, l, m) in enumerate(multi_indices(L)):
        pi, ta = pi_tau(l, abs(m), theta)
        e = np.exp(1j * m * phi) / np.sqrt(2.0 * l * (l + 1))
        if tau == 1:
            v = (-1j) ** (l + 1) * e[:, None] * ((1j * m * pi)[:, None] * et - ta[:, None] * ep)
        else:
            v = (-1j) ** l * e[:, None] * (ta[:, None] * et + (1j * m * pi)[:, None] * ep)
        F += coef[:, c][:, None] * v
    return F


def scattering_cross_section(k, pos, b, L, n_theta=None, n_phi=None):
    """C_sca by Gauss-Legendre quadrature in cos(theta) and the trapezoid rule
    in phi, sized from the band limit L + k D (D = cluster diameter)."""
    pos = np.asarray(pos)
    D = 2.0 * np.max(np.linalg.norm(pos - pos.mean(axis=0), axis=1)) if pos.shape[0] > 1 else 0.0
    band = int(L + k * D) + 10
    nt = n_theta or band + 1
    nph = n_phi or 2 * band + 2
    x, w = np.polynomial.legendre.leggauss(nt)
    theta = np.arccos(x)
    phi = 2 * np.pi * np.arange(nph) / nph
    TT, PP = np.meshgrid(theta, phi, indexing="ij")
    WW = np.repeat(w[:, None], nph, axis=1) * (2 * np.pi / nph)
    F = far_field(k, pos - pos.mean(axis=0), b, L, TT.reshape(-1), PP.reshape(-1))
    return float(np.sum(WW.reshape(-1) * np.sum(np.abs(F) ** 2, axis=1))) / k ** 2


def scattered_field(k, pos, b, L, points):
    """Near field sum_i sum_n b_n^i Psi^(3)_n(r - r_i) at points outside all spheres."""
    pts = np.atleast_2d(points)
    E = np.zeros((pts.shape[0], 3), dtype=np.complex128)
    for i in range(np.asarray(pos).shape[0]):
        for c, (tau, l, m) in enumerate(multi_indices(L)):
            if b[i, c] != 0:
                E += b[i, c] * svwf(3, tau, l, m, pts - pos[i], k)
    return E

"""Spherical and plane vector wave functions (paper, Appendix A.1).

  Psi_{1lm}^(nu)(r) = e^{im phi}/sqrt(2l(l+1)) z_l(kr)
                      (i m pi_l^{|m|}(theta) e_theta - tau_l^{|m|}(theta) e_phi)
  Psi_{2lm}^(nu)(r) = e^{im phi}/sqrt(2l(l+1)) ( l(l+1) z_l(kr)/(kr) P_l^{|m|} e_r
                      + [d(kr z_l)/d(kr)]/(kr) (tau e_theta + i m pi e_phi) )
  Phi_1(alpha, beta; r) = e^{i k.r} e_alpha,  Phi_2 = e^{i k.r} e_beta
Fields are returned as cartesian complex 3-vectors.
"""
import numpy as np

from .special import legendre, pi_tau, radial


def _sph(r):
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    rr = np.sqrt(np.sum(r * r, axis=1))
    th = np.arccos(np.clip(r[:, 2] / rr, -1.0, 1.0))
    ph = np.arctan2(r[:, 1], r[:, 0])
    return rr, th, ph


def _unit_vectors(th, ph):
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    er = np.stack([st * cp, st * sp, ct], axis=-1)
    et = np.stack([ct * cp, ct * sp, -st], axis=-1)
    ep = np.stack([-sp, cp, np.zeros_like(ph)], axis=-1)
    return er, et, ep


def svwf(nu, tau, l, m, r, k):
    """Psi_{tau l m}^(nu)(r) at points r [P, 3]; returns [P, 3] complex."""
    rr, th, ph = _sph(r)
    kr = k * rr
    z, dkrz = radial(nu, l, kr)
    P = legendre(l, abs(m), np.cos(th), np.sin(th))
    pi, ta = pi_tau(l, abs(m), th)
    er, et, ep = _unit_vectors(th, ph)
    e = np.exp(1j * m * ph) / np.sqrt(2.0 * l * (l + 1))
    if tau == 1:
        v = (1j * m * pi)[:, None] * et - ta[:, None] * ep
        return (e * z)[:, None] * v
    v = (l * (l + 1) * z / kr * P)[:, None] * er \
        + (dkrz / kr)[:, None] * (ta[:, None] * et + (1j * m * pi)[:, None] * ep)
    return e[:, None] * v


def pvwf(j, alpha, beta, r, k):
    """Phi_j(alpha, beta; r) = exp(i k.r) e_j with e_1 = e_alpha, e_2 = e_beta."""
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    kv = k * np.array([np.sin(beta) * np.cos(alpha), np.sin(beta) * np.sin(alpha), np.cos(beta)])
    ph = np.exp(1j * (r @ kv))
    if j == 1:
        e = np.array([-np.sin(alpha), np.cos(alpha), 0.0])
    else:
        e = np.array([np.cos(beta) * np.cos(alpha), np.cos(beta) * np.sin(alpha), -np.sin(beta)])
    return ph[:, None] * e[None, :]

"""Initial-field coefficients a_in (paper, Appendix A.2 "PVWF to SVWF" and
Appendix C).

Transformation operator (eq. B), for n = (tau, l, m), polarisation j:
  B_{nj}(beta)  = -1/i^{l+1} / sqrt(2l(l+1)) (i delta_{j1} + delta_{j2})
                  (delta_{tau j} tau_l^{|m|}(beta) + (1-delta_{tau j}) m pi_l^{|m|}(beta))
  B^dagger_{nj} = the same with every explicit i replaced by -i.
PVWF expansion:  Phi_j(alpha, beta; r) = 4 sum_n e^{-i m alpha} B^dagger_{nj}(beta) Psi^(1)_n(r).
"""
import numpy as np
from scipy.special import jv

from .special import pi_tau
from .translation import multi_indices, nmax_of


def B_dagger(tau, l, m, j, beta):
    pi, ta = pi_tau(l, abs(m), beta)
    pol = (-1j if j == 1 else 1.0)
    ang = ta if tau == j else m * pi
    return -(1.0 / (-1j) ** (l + 1)) / np.sqrt(2.0 * l * (l + 1)) * pol * ang


def B_op(tau, l, m, j, beta):
    pi, ta = pi_tau(l, abs(m), beta)
    pol = (1j if j == 1 else 1.0)
    ang = ta if tau == j else m * pi
    return -(1.0 / (1j) ** (l + 1)) / np.sqrt(2.0 * l * (l + 1)) * pol * ang


def plane_wave_coefficients(pos, k, L, beta, alpha, pol, E0=1.0):
    """a_in for E0 Phi_pol(alpha, beta; r): expanding about each centre r_i,
    Phi_j(r) = e^{i k.r_i} Phi_j(r - r_i), then the PVWF expansion gives
    a_{in,n}^i = 4 E0 e^{i k.r_i} e^{-i m alpha} B^dagger_{nj}(beta).
    Returns [N, nmax]."""
    pos = np.atleast_2d(np.asarray(pos, dtype=np.float64))
    kv = k * np.array([np.sin(beta) * np.cos(alpha), np.sin(beta) * np.sin(alpha), np.cos(beta)])
    ph = np.exp(1j * (pos @ kv))
    v = np.array([4.0 * E0 * np.exp(-1j * m * alpha) * B_dagger(tau, l, m, pol, beta)
                  for (tau, l, m) in multi_indices(L)])
    return ph[:, None] * v[None, :]


def gaussian_beam_coefficients(pos, k, L, waist, focus, alpha_G, E0=1.0, n_beta=512):
    """a_in for the Gaussian beam of Appendix C:

      a_{in,n}^i = E0 k^2 w^2/pi sum_j int_0^{pi/2} dbeta sin(beta) cos(beta)
                   B^dagger_{nj}(beta) I_{jn}(beta)
                   exp(-w^2 k^2 sin^2(beta)/4 + i k z_{G,i} cos(beta)),
      I_{jn} = 2 pi e^{-i alpha_G} i^{|m-1|} e^{-i(m-1) phi_{G,i}} J_{|m-1|}(k rho sin beta) (d_{j1} - i d_{j2})/2
             + 2 pi e^{+i alpha_G} i^{|m+1|} e^{-i(m+1) phi_{G,i}} J_{|m+1|}(k rho sin beta) (d_{j1} + i d_{j2})/2,
    with (rho_{G,i}, phi_{G,i}, z_{G,i}) the cylindrical coordinates of r_i - r_G.
    The plane-wave phase e^{i k.(r_i - r_G)} is the product of its lateral and
    axial factors (the sum printed in Appendix C is read as a product).  The
    beta integral uses n_beta-point Gauss-Legendre quadrature on [0, pi/2].
    Returns [N, nmax]."""
    pos = np.atleast_2d(np.asarray(pos, dtype=np.float64))
    rel = pos - np.asarray(focus, dtype=np.float64)[None, :]
    rho = np.hypot(rel[:, 0], rel[:, 1])
    phG = np.arctan2(rel[:, 1], rel[:, 0])
    zG = rel[:, 2]
    xg, wg = np.polynomial.legendre.leggauss(n_beta)
    beta = 0.25 * np.pi * (xg + 1.0)
    wb = 0.25 * np.pi * wg
    sb, cb = np.sin(beta), np.cos(beta)
    gauss = np.exp(-(waist * k * sb) ** 2 / 4.0)
    axial = np.exp(1j * k * np.outer(zG, cb))                     # [N, nb]
    arg = k * np.outer(rho, sb)                                   # [N, nb]
    base = (wb * sb * cb * gauss)[None, :] * axial                # [N, nb]
    idx = multi_indices(L)
    out = np.zeros((pos.shape[0], nmax_of(L)), dtype=np.complex128)
    for c, (tau, l, m) in enumerate(idx):
        acc = np.zeros(pos.shape[0], dtype=np.complex128)
        for j in (1, 2):
            Bd = B_dagger(tau, l, m, j, beta)                            # [nb]
            t1 = (2 * np.pi * np.exp(-1j * alpha_G) * (1j) ** abs(m - 1)
                  * np.exp(-1j * (m - 1) * phG)[:, None] * jv(abs(m - 1), arg)
                  * ((1.0 if j == 1 else 0.0) - 1j * (1.0 if j == 2 else 0.0)) / 2.0)
            t2 = (2 * np.pi * np.exp(1j * alpha_G) * (1j) ** abs(m + 1)
                  * np.exp(-1j * (m + 1) * phG)[:, None] * jv(abs(m + 1), arg)
                  * ((1.0 if j == 1 else 0.0) + 1j * (1.0 if j == 2 else 0.0)) / 2.0)
            acc += np.sum(base * Bd[None, :] * (t1 + t2), axis=1)
        out[:, c] = E0 * k * k * waist * waist / np.pi * acc
    return out


def gaussian_beam_field(r, k, waist, focus, alpha_G, E0=1.0, n_beta=256, n_alpha=256):
    """Initial field of Appendix C (eq. "E_in Gauss") evaluated by direct 2D
    quadrature of the angular-spectrum integral, with the small-beta
    polarisation approximation of that appendix.  Independent of the
    coefficient formula above (no Bessel identity, no PVWF expansion)."""
    r = np.atleast_2d(np.asarray(r, dtype=np.float64)) - np.asarray(focus)[None, :]
    xg, wg = np.polynomial.legendre.leggauss(n_beta)
    beta = 0.25 * np.pi * (xg + 1.0)
    wb = 0.25 * np.pi * wg
    alpha = 2 * np.pi * np.arange(n_alpha) / n_alpha
    wa = 2 * np.pi / n_alpha
    E = np.zeros((r.shape[0], 3), dtype=np.complex128)
    ca, sa = np.cos(alpha), np.sin(alpha)
    pa, qa = np.cos(alpha - alpha_G), np.sin(alpha - alpha_G)
    for b, w_b in zip(beta, wb):
        sb, cb = np.sin(b), np.cos(b)
        g = E0 * k * k * waist * waist / (4 * np.pi) * sb * cb * np.exp(-(waist * k * sb) ** 2 / 4)
        kv = k * np.stack([sb * ca, sb * sa, np.full_like(ca, cb)], -1)        # [na, 3]
        ph = np.exp(1j * (r @ kv.T))                                          # [P, na]
        ea = np.stack([-sa, ca, np.zeros_like(ca)], -1)
        eb = np.stack([cb * ca, cb * sa, np.full_like(ca, -sb)], -1)
        pol = pa[:, None] * ea + qa[:, None] * eb                             # [na, 3]
        E += (w_b * wa * g) * (ph @ pol)
    return E

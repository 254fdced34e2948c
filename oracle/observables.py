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


def phase_function_s11(k, pos, b_runs, L, theta, n_phi=64):
    """(1,1) element of the phase matrix as the paper obtains it (Section 4,
    validation): the far-field intensity |F(theta, phi)|^2 averaged over
    runs with different incident polarisations (b_runs: list of [N, nmax]
    coefficient arrays, e.g. TE and TM) and over n_phi equally spaced
    azimuths phi_j = 2 pi j / n_phi.  Not normalised: k^2 times the
    polarisation-averaged differential scattering cross section; divide by
    the value at theta = 0 for the S11(0) = 1 convention."""
    theta = np.atleast_1d(np.asarray(theta, dtype=float))
    out = np.zeros(theta.size)
    phis = 2.0 * np.pi * np.arange(n_phi) / n_phi
    for b in b_runs:
        for ph in phis:
            F = far_field(k, pos, b, L, theta, np.full(theta.size, ph))
            out += np.sum(np.abs(F) ** 2, axis=1)
    return out / (len(b_runs) * n_phi)


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


def gaussian_spectrum(k, waist, focus, alpha_G, E0, beta, alpha):
    """Plane-wave pattern (g_alpha, g_beta) of the Gaussian beam of Appendix C
    in direction (beta, alpha), beta < pi/2: the amplitude
    E0 k^2 w^2/(4 pi) cos(beta) exp(-(w k sin(beta))^2 / 4), polarisation
    cos(alpha - alpha_G) e_alpha + sin(alpha - alpha_G) e_beta, and the phase
    exp(-i k.r_G) of the focus (the same spectrum as gaussian_beam_field)."""
    sb, cb = np.sin(beta), np.cos(beta)
    g = E0 * k * k * waist * waist / (4 * np.pi) * cb * np.exp(-(waist * k * sb) ** 2 / 4)
    kr = k * (sb * np.cos(alpha) * focus[0] + sb * np.sin(alpha) * focus[1] + cb * focus[2])
    ph = np.exp(-1j * kr)
    return g * np.cos(alpha - alpha_G) * ph, g * np.sin(alpha - alpha_G) * ph


def power_flux(k, pos, b, L, tvec, waist, focus, alpha_G, E0=1.0, n_beam=64, n_beta=None, n_alpha=None):
    """Reflected, transmitted and absorbed fractions of a Gaussian beam's power
    (Appendix D).  A field sum_j int dalpha int dbeta sin(beta) g_j Phi_j
    carries the power P = 2 pi^2/(omega k mu0) sum_j oint |g_j|^2 dOmega.  At
    large r a plane-wave superposition tends to -2 pi i e^{ikr}/(kr) g(rhat)
    (stationary phase), so the scattered field E -> e^{ikr}/(kr) F has the
    pattern g_sca = (i / 2 pi) F.  Upper hemisphere: g_in + g_sca (transmitted),
    lower hemisphere: g_sca (reflected).  Absorbed power from the Mie
    coefficients as in `absorption`.  Returns (P_inc / I_0 with I_0 the
    intensity of a unit plane wave, R, T, A)."""
    pos = np.asarray(pos, dtype=np.float64)
    D = 2.0 * float(np.max(np.linalg.norm(pos, axis=1)))
    band = int(L + k * D) + 10
    nb = n_beta or band + 1
    na = n_alpha or 2 * band + 2
    b1 = min(np.pi / 2, float(np.arcsin(min(1.0, 8.0 / (k * waist)))))

    def gl(a, c, n):
        x, w = np.polynomial.legendre.leggauss(n)
        return 0.5 * (c - a) * (x + 1) + a, 0.5 * (c - a) * w

    parts = [gl(0.0, b1, n_beam)]
    if b1 < np.pi / 2:
        parts.append(gl(b1, np.pi / 2, nb))
    bf = np.concatenate([p[0] for p in parts])
    wf = np.concatenate([p[1] for p in parts])
    bb, wb = gl(np.pi / 2, np.pi, nb)
    alpha = 2 * np.pi * np.arange(na) / na
    wa = 2 * np.pi / na

    def pattern(beta):
        BB, AA = np.meshgrid(beta, alpha, indexing="ij")
        F = far_field(k, pos, b, L, BB.reshape(-1), AA.reshape(-1)).reshape(BB.shape + (3,))
        ea = np.stack([-np.sin(AA), np.cos(AA), np.zeros_like(AA)], -1)
        eb = np.stack([np.cos(BB) * np.cos(AA), np.cos(BB) * np.sin(AA), -np.sin(BB)], -1)
        return BB, AA, 1j / (2 * np.pi) * np.sum(F * ea, -1), 1j / (2 * np.pi) * np.sum(F * eb, -1)

    BB, AA, sa, sb_ = pattern(bf)
    ga, gb = gaussian_spectrum(k, waist, focus, alpha_G, E0, BB, AA)
    wf2 = (wf * np.sin(bf))[:, None] * wa
    P0 = float(np.sum(wf2 * (np.abs(ga) ** 2 + np.abs(gb) ** 2)))
    T = float(np.sum(wf2 * (np.abs(ga + sa) ** 2 + np.abs(gb + sb_) ** 2))) / P0
    _, _, ra, rb = pattern(bb)
    R = float(np.sum((wb * np.sin(bb))[:, None] * wa * (np.abs(ra) ** 2 + np.abs(rb) ** 2))) / P0
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(tvec != 0, np.real(1.0 / tvec) + 1.0, 0.0)
    A = -float(np.sum(np.abs(b) ** 2 * f)) / (4 * np.pi) / P0
    return 4 * np.pi ** 2 / k ** 2 * P0, R, T, A

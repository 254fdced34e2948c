"""SVWF translation operator and the coupling matrix W (paper, Section 2.2 and
Appendix A.2).

Multi-index n = (tau, l, m), tau in {1, 2}, l = 1..L, m = -l..l.  The paper
fixes no linear order; this oracle uses (0-based)
    idx(tau, l, m) = (tau-1) L(L+2) + l(l+1) + m - 1,      nmax = 2 L (L+2).

Translation operator (Appendix A.2, eqs. "A operator" / "B operator"):
    A_{tau l m, tau' l' m'}(d) = delta_{tau tau'} A_{ml,m'l'}(d)
                                 + (1 - delta_{tau tau'}) B_{ml,m'l'}(d),
    A_{ml,m'l'}(d) = e^{i(m-m') phi_d} sum_{p=|l-l'|}^{l+l'} a5(l,m|l',m'|p)
                     h_p(kd) P_p^{|m-m'|}(cos theta_d),
    B_{ml,m'l'}(d) = same with b5 and p from |l-l'|+1.
Coupling matrix (Section 2.2): W^{ii'}_{nn'} = A_{n'n}(r_i - r_{i'}), i != i'.
"""
from functools import lru_cache
from fractions import Fraction
from math import sqrt

import numpy as np

from .special import legendre, sph_h1
from .wigner import wigner3j_exact, frac_sqrt_float


def nmax_of(L):
    return 2 * L * (L + 2)


def idx(tau, l, m, L):
    """Linear index of n = (tau, l, m)."""
    return (tau - 1) * L * (L + 2) + l * (l + 1) + m - 1


def multi_indices(L):
    """List of (tau, l, m) in index order."""
    out = []
    for tau in (1, 2):
        for l in range(1, L + 1):
            for m in range(-l, l + 1):
                out.append((tau, l, m))
    return out


_IPOW = (1, 1j, -1, -1j)


def _ipow(e):
    # i^e for any integer e (mathematical modulo, so negative e is allowed)
    return _IPOW[e % 4]


@lru_cache(maxsize=None)
def a5(l, m, lp, mp, p):
    """a5(l,m|l',m'|p) exactly as printed in Appendix A.2 (real-valued)."""
    s1, q1 = wigner3j_exact(l, lp, p, m, -mp, mp - m)
    s2, q2 = wigner3j_exact(l, lp, p, 0, 0, 0)
    if s1 == 0 or s2 == 0:
        return 0.0
    c = l * (l + 1) + lp * (lp + 1) - p * (p + 1)
    if c == 0:
        return 0.0
    sq = Fraction(c * c * (2 * p + 1) * (2 * l + 1) * (2 * lp + 1),
                  2 * l * (l + 1) * lp * (lp + 1)) * q1 * q2
    sign = s1 * s2 * (1 if c > 0 else -1) * (-1) ** ((m - mp) % 2)
    ph = _ipow(abs(m - mp) - abs(m) - abs(mp) + lp - l + p)
    return ph * sign * frac_sqrt_float(sq)


@lru_cache(maxsize=None)
def b5(l, m, lp, mp, p):
    """b5(l,m|l',m'|p) exactly as printed in Appendix A.2 (imaginary-valued)."""
    if p - 1 < abs(l - lp):
        return 0.0
    s1, q1 = wigner3j_exact(l, lp, p, m, -mp, mp - m)
    s2, q2 = wigner3j_exact(l, lp, p - 1, 0, 0, 0)
    if s1 == 0 or s2 == 0:
        return 0.0
    rad = (l + lp + 1 + p) * (l + lp + 1 - p) * (p + l - lp) * (p - l + lp) * (2 * p + 1)
    if rad <= 0:
        return 0.0
    sq = Fraction(rad * (2 * l + 1) * (2 * lp + 1), 2 * l * (l + 1) * lp * (lp + 1)) * q1 * q2
    sign = s1 * s2 * (-1) ** ((m - mp) % 2)
    ph = _ipow(abs(m - mp) - abs(m) - abs(mp) + lp - l + p)
    return ph * sign * frac_sqrt_float(sq)


def _pair_geometry(d):
    d = np.atleast_2d(np.asarray(d, dtype=np.float64))
    r = np.sqrt(np.sum(d * d, axis=1))
    rho = np.hypot(d[:, 0], d[:, 1])
    ct = d[:, 2] / r
    st = rho / r
    ph = np.where(rho > 0, np.arctan2(d[:, 1], d[:, 0]), 0.0)
    return r, ct, st, ph


def translation_blocks(d, k, L, hankel=None, Lrow=None):
    """A_{nn'}(d) for an array of displacement vectors d [P, 3].

    Returns complex array [P, nmax, nmax] with A[:, n, n'] = A_{nn'}(d).
    `hankel(p, x)` overrides h_p^(1)(x) (used for the lookup-table mode);
    default is the exact spherical Hankel function.  With Lrow < L only the
    rows with l <= Lrow are filled (the rest stay zero).
    """
    Lrow = L if Lrow is None else Lrow
    hk = hankel if hankel is not None else sph_h1
    r, ct, st, ph = _pair_geometry(d)
    P = r.size
    kd = k * r
    hp = [hk(p, kd) for p in range(2 * L + 1)]
    Pl = {}
    for p in range(2 * L + 1):
        for mu in range(p + 1):
            Pl[(p, mu)] = legendre(p, mu, ct, st)
    nm = nmax_of(L)
    half = L * (L + 2)
    out = np.zeros((P, nm, nm), dtype=np.complex128)
    for l in range(1, Lrow + 1):
        for m in range(-l, l + 1):
            for lp in range(1, L + 1):
                for mp in range(-lp, lp + 1):
                    mu = abs(m - mp)
                    Asum = np.zeros(P, dtype=np.complex128)
                    Bsum = np.zeros(P, dtype=np.complex128)
                    for p in range(abs(l - lp), l + lp + 1):
                        if p < mu:
                            continue
                        c = a5(l, m, lp, mp, p)
                        if c != 0:
                            Asum += c * hp[p] * Pl[(p, mu)]
                        if p >= abs(l - lp) + 1:
                            c = b5(l, m, lp, mp, p)
                            if c != 0:
                                Bsum += c * hp[p] * Pl[(p, mu)]
                    e = np.exp(1j * (m - mp) * ph)
                    Av = e * Asum
                    Bv = e * Bsum
                    i0 = l * (l + 1) + m - 1
                    j0 = lp * (lp + 1) + mp - 1
                    out[:, i0, j0] = Av
                    out[:, half + i0, half + j0] = Av
                    out[:, i0, half + j0] = Bv
                    out[:, half + i0, j0] = Bv
    return out


def translation_matrix(d, k, L, hankel=None, Lrow=None):
    """A_{nn'}(d) for a single displacement vector d."""
    return translation_blocks(np.asarray(d)[None, :], k, L, hankel, Lrow)[0]


def coupling_matrix(pos, k, L, hankel=None):
    """Dense W with W[(i,n),(i',n')] = A_{n'n}(r_i - r_{i'}) for i != i' and
    zero diagonal blocks (Section 2.2).  Shape [N nmax, N nmax]."""
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[0]
    nm = nmax_of(L)
    ii, jj = np.nonzero(~np.eye(N, dtype=bool))
    blocks = translation_blocks(pos[ii] - pos[jj], k, L, hankel)
    W = np.zeros((N, nm, N, nm), dtype=np.complex128)
    W[ii, :, jj, :] = np.transpose(blocks, (0, 2, 1))
    return W.reshape(N * nm, N * nm)


def apply_W_rows(pos, x, k, L, rows, hankel=None):
    """(W x)^i for the receiving spheres i in `rows`, computed on the fly
    (W is never formed).  x: [N, nmax] complex, or [K, N, nmax] for K
    right-hand sides sharing the geometry.  Returns [len(rows), nmax], or
    [K, len(rows), nmax]."""
    pos = np.asarray(pos, dtype=np.float64)
    x = np.asarray(x)
    single = x.ndim == 2
    xs = x[None] if single else x
    K, N = xs.shape[0], pos.shape[0]
    out = np.zeros((K, len(rows), nmax_of(L)), dtype=np.complex128)
    for a, i in enumerate(rows):
        src = np.array([j for j in range(N) if j != i], dtype=np.int64)
        blocks = translation_blocks(pos[i] - pos[src], k, L, hankel)
        # y_n = sum_{i', n'} A_{n'n}(r_i - r_i') x_{i' n'}, for every right-hand side
        out[:, a] = np.einsum("pab,kpa->kb", blocks, xs[:, src])
    return out[0] if single else out

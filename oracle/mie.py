"""Sphere T-matrix (paper, Appendix B) and an independent Mie series.

`mie_Q` follows the paper's closed form for Q_{1l}, Q_{2l} with x = kR and
k_i R = (n_i/n0) kR: the wavenumber inside the sphere is n_i omega/c and k is
the background wavenumber n0 omega/c, so the printed k_i = n_i k is read with
the relative index n_i/n0 (identical for n0 = 1).

`bohren_huffman_ab` is a separate implementation of the textbook Mie
coefficients a_n, b_n (Bohren & Huffman 1983, logarithmic-derivative method:
D_n(mx) by downward recurrence, Riccati-Bessel psi_n, chi_n by upward
recurrence).  It uses no scipy special functions, so comparing it with
`mie_Q` (a_l = -Q_{2l}, b_l = -Q_{1l}) checks the paper formula independently.
"""
import numpy as np
from scipy.special import spherical_jn, spherical_yn


def _psi_d(l, z):
    """j_l(z) and d/dz [z j_l(z)] (complex z allowed)."""
    j = spherical_jn(l, z)
    dj = spherical_jn(l, z, derivative=True)
    return j, j + z * dj


def _xi_d(l, x):
    h = spherical_jn(l, x) + 1j * spherical_yn(l, x)
    dh = spherical_jn(l, x, derivative=True) + 1j * spherical_yn(l, x, derivative=True)
    return h, h + x * dh


def mie_Q(L, k, R, n_sphere, n0=1.0):
    """Q[tau-1, l-1] for one sphere (Appendix B): T_{nn'} = Q_{tau l} delta."""
    m = complex(n_sphere) / n0
    x = k * R
    mx = m * x
    Q = np.zeros((2, L), dtype=np.complex128)
    for l in range(1, L + 1):
        jx, djx = _psi_d(l, x)
        jm, djm = _psi_d(l, mx)
        hx, dhx = _xi_d(l, x)
        Q[0, l - 1] = (jx * djm - jm * djx) / (jm * dhx - hx * djm)
        # multiply numerator and denominator of the printed Q_2l by 1/k^2
        Q[1, l - 1] = (jx * djm - m * m * jm * djx) / (m * m * jm * dhx - hx * djm)
    return Q


def bohren_huffman_ab(nmax, x, m):
    """Textbook Mie coefficients a_n, b_n, n = 1..nmax (e^{-i omega t})."""
    m = complex(m)
    mx = m * x
    nstop = nmax
    nmx = int(max(nstop, abs(mx)) + 16)
    D = np.zeros(nmx + 1, dtype=np.complex128)
    for n in range(nmx, 0, -1):
        D[n - 1] = n / mx - 1.0 / (D[n] + n / mx)
    psi0, psi1 = np.cos(x), np.sin(x)        # psi_{-1}, psi_0
    chi0, chi1 = -np.sin(x), np.cos(x)       # chi_{-1}, chi_0
    xi1 = complex(psi1, -chi1)
    a = np.zeros(nmax, dtype=np.complex128)
    b = np.zeros(nmax, dtype=np.complex128)
    for n in range(1, nmax + 1):
        psi = (2.0 * n - 1.0) * psi1 / x - psi0
        chi = (2.0 * n - 1.0) * chi1 / x - chi0
        xi = complex(psi, -chi)
        ta = D[n] / m + n / x
        tb = D[n] * m + n / x
        a[n - 1] = (ta * psi - psi1) / (ta * xi - xi1)
        b[n - 1] = (tb * psi - psi1) / (tb * xi - xi1)
        psi0, psi1 = psi1, psi
        chi0, chi1 = chi1, chi
        xi1 = complex(psi1, -chi1)
    # B&H define xi_n = psi_n - i chi_n with chi_n = -x y_n, i.e. xi = x h^(1).
    return a, b


def bohren_huffman_S1_S2(nmax, x, m, theta):
    """Textbook scattering amplitudes S1(theta), S2(theta) of a sphere
    (Bohren & Huffman): S1 = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n),
    S2 = sum (2n+1)/(n(n+1)) (a_n tau_n + b_n pi_n), with the angular
    functions pi_n, tau_n of cos(theta) from their upward recurrences (not
    the normalized Legendre functions the rest of the oracle uses)."""
    a, b = bohren_huffman_ab(nmax, x, m)
    mu = np.cos(np.atleast_1d(theta))
    S1 = np.zeros(mu.shape, dtype=np.complex128)
    S2 = np.zeros(mu.shape, dtype=np.complex128)
    pi_prev, pi_cur = np.zeros_like(mu), np.ones_like(mu)        # pi_0, pi_1
    for n in range(1, nmax + 1):
        tau = n * mu * pi_cur - (n + 1) * pi_prev
        f = (2.0 * n + 1.0) / (n * (n + 1.0))
        S1 += f * (a[n - 1] * pi_cur + b[n - 1] * tau)
        S2 += f * (a[n - 1] * tau + b[n - 1] * pi_cur)
        pi_prev, pi_cur = pi_cur, ((2.0 * n + 1.0) / n) * mu * pi_cur - ((n + 1.0) / n) * pi_prev
    return S1, S2


def T_vector(L, k, radii, n_sphere, n0=1.0):
    """Diagonal of the block T-matrix as [N, nmax] (Q_{tau l} repeated over m)."""
    radii = np.atleast_1d(radii)
    n_sphere = np.broadcast_to(np.asarray(n_sphere, dtype=np.complex128), radii.shape)
    nm = 2 * L * (L + 2)
    out = np.zeros((radii.size, nm), dtype=np.complex128)
    cache = {}
    for i, (R, ns) in enumerate(zip(radii, n_sphere)):
        key = (float(R), complex(ns))
        if key not in cache:
            Q = mie_Q(L, k, R, ns, n0)
            v = np.zeros(nm, dtype=np.complex128)
            c = 0
            for tau in (1, 2):
                for l in range(1, L + 1):
                    v[c:c + 2 * l + 1] = Q[tau - 1, l - 1]
                    c += 2 * l + 1
            cache[key] = v
        out[i] = cache[key]
    return out

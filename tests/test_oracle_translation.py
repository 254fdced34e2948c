"""Pins for the translation operator and W.

The decisive pin is the SVWF addition theorem (Appendix A.2): an outgoing
wave about one origin equals the regular-wave expansion about a displaced
origin with the translation coefficients.  It fixes the Legendre
normalization, the index roles of A, the powers of i in a5/b5 and the sign of
the azimuthal phase together.  The symmetry pins (reciprocity, axial
m-conservation, Hermitian part) are mathematical consequences that a dropped
term or a wrong sign would break.
"""
import math

import numpy as np
import pytest

from oracle.svwf import svwf
from oracle.translation import a5, b5, coupling_matrix, idx, multi_indices, translation_matrix
from oracle.lut import HankelLUT, lut_grid
from oracle.special import sph_h1
from scipy.special import spherical_jn, spherical_yn


@pytest.mark.parametrize("d", [
    (2.1, -3.2, 3.0),          # generic direction
    (0.0, 0.0, 4.5),           # along +z (phi undefined, theta = 0)
    (0.0, 0.0, -4.0),          # along -z (theta = pi)
    (-3.3, 1.2, -1.9),
])
def test_addition_theorem(d):
    k = 1.0
    d = np.array(d)
    Lp = 16    # truncation error of the expansion ~1e-12 for |r|/|d| < 0.1 here
    A = translation_matrix(d, k, Lp, Lrow=4)
    rng = np.random.default_rng(1)
    r = rng.uniform(-0.25, 0.25, (3, 3))
    for (tau, l, m) in multi_indices(4):
        lhs = svwf(3, tau, l, m, r + d, k)
        rhs = 0
        for (tp, lp, mp) in multi_indices(Lp):
            c = A[idx(tau, l, m, Lp), idx(tp, lp, mp, Lp)]
            if c != 0:
                rhs = rhs + c * svwf(1, tp, lp, mp, r, k)
        assert np.abs(lhs - rhs).max() <= 1e-10 * np.abs(lhs).max(), (tau, l, m)


def test_a5_real_b5_imaginary_and_selection_rules():
    L = 4
    for l in range(1, L + 1):
        for lp in range(1, L + 1):
            for m in range(-l, l + 1):
                for mp in range(-lp, lp + 1):
                    for p in range(0, l + lp + 2):
                        a = a5(l, m, lp, mp, p)
                        b = b5(l, m, lp, mp, p) if p >= 1 else 0.0
                        assert np.imag(a) == 0
                        assert np.real(b) == 0
                        if (l + lp + p) % 2 == 1 or p > l + lp or p < abs(l - lp):
                            assert a == 0
                        if (l + lp + p) % 2 == 0 or p > l + lp:
                            assert b == 0
                        if p < abs(m - mp):
                            assert a == 0 and b == 0
                        # m-mirror: a5 even, b5 odd under (m, m') -> (-m, -m')
                        assert abs(a5(l, -m, lp, -mp, p) - a) < 1e-15
                        if p >= 1:
                            assert abs(b5(l, -m, lp, -mp, p) + b) < 1e-15


def _flip_perm(L, N):
    ind = multi_indices(L)
    f = np.array([ind.index((t, l, -m)) for (t, l, m) in ind])
    nm = len(ind)
    return np.concatenate([i * nm + f for i in range(N)])


def test_reciprocity_of_W():
    rng = np.random.default_rng(3)
    pos = rng.uniform(-800, 800, (5, 3))
    k = 2 * math.pi / 550
    for L in (1, 2, 3):
        W = coupling_matrix(pos, k, L)
        Pi = _flip_perm(L, 5)
        assert np.abs(W[np.ix_(Pi, Pi)] - W.T).max() <= 1e-14 * np.abs(W).max()


def test_axial_pair_conserves_m():
    k = 2 * math.pi / 550
    L = 3
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 420.0]])
    W = coupling_matrix(pos, k, L)
    ind = multi_indices(L)
    nm = len(ind)
    blk = W[:nm, nm:]
    for a, (t, l, m) in enumerate(ind):
        for b, (tp, lp, mp) in enumerate(ind):
            if m != mp:
                assert abs(blk[a, b]) == 0.0
    assert np.abs(np.diag(blk)).min() > 0


def test_hermitian_part_uses_second_kind():
    # conj(W) = Pi W^(h2) Pi  =>  W^H = W^(h2), hence (W + W^H)/2 = W built with j_p.
    rng = np.random.default_rng(4)
    pos = rng.uniform(-600, 600, (4, 3))
    k = 2 * math.pi / 550
    L = 3
    W = coupling_matrix(pos, k, L)
    W2 = coupling_matrix(pos, k, L, hankel=lambda p, x: spherical_jn(p, x) - 1j * spherical_yn(p, x))
    WJ = coupling_matrix(pos, k, L, hankel=lambda p, x: spherical_jn(p, x) + 0j)
    s = np.abs(W).max()
    assert np.abs(W.conj().T - W2).max() <= 1e-14 * s
    assert np.abs((W + W.conj().T) / 2 - WJ).max() <= 1e-14 * s


def test_lut_error_within_hermite_bound():
    # cubic Hermite error <= (dr k)^4 / 384 max|h''''|; bound h'''' by finite differences
    k = 2 * math.pi / 550
    pos = np.array([[0, 0, 0], [3000.0, 0, 0], [0, 2500.0, 900.0]])
    radii = np.array([100.0, 100.0, 100.0])
    for dr in (1.0, 5.0):
        d_lo, n = lut_grid(pos, radii, dr)
        lut = HankelLUT(k, 8, d_lo, dr, n)
        d = np.linspace(d_lo + 0.01, d_lo + (n - 0.01) * dr, 4001)
        for p in range(0, 9):
            ex = sph_h1(p, k * d)
            got = lut(p, k * d)
            x = k * d
            hs = 1e-2
            d4 = (sph_h1(p, x + 2 * hs) - 4 * sph_h1(p, x + hs) + 6 * sph_h1(p, x)
                  - 4 * sph_h1(p, x - hs) + sph_h1(p, x - 2 * hs)) / hs ** 4
            bound = (dr * k) ** 4 / 384 * np.abs(d4)
            assert np.all(np.abs(got - ex) <= 1.5 * bound + 1e-13 * np.abs(ex))


def test_two_order_table_recurrence_keeps_relative_error():
    # h_0, h_1 interpolated (bounded by the test above); the upward recurrence
    # for p >= 2 follows the dominant y_p, so the relative error of h_p stays
    # at the level of h_0 and h_1.  A wrong recurrence coefficient gives an
    # O(1) error here.
    from oracle.lut import HankelLUT01
    k = 2 * math.pi / 550
    pos = np.array([[0, 0, 0], [3000.0, 0, 0], [0, 2500.0, 900.0]])
    radii = np.array([100.0, 100.0, 100.0])
    for dr in (1.0, 5.0):
        d_lo, n = lut_grid(pos, radii, dr)
        lut = HankelLUT01(k, 8, d_lo, dr, n)
        x = k * np.linspace(d_lo + 0.01, d_lo + (n - 0.01) * dr, 4001)
        base = max(np.max(np.abs(lut(p, x) - sph_h1(p, x)) / np.abs(sph_h1(p, x))) for p in (0, 1))
        assert base <= (1e-10 if dr == 1.0 else 1e-7)
        for p in range(2, 9):
            ex = sph_h1(p, x)
            assert np.max(np.abs(lut(p, x) - ex) / np.abs(ex)) <= 2 * base + 1e-14
        with pytest.raises(ValueError):
            lut(9, x)


def test_lut_matvec_close_to_exact():
    from oracle.lut import lut_for
    k = 2 * math.pi / 550
    rng = np.random.default_rng(9)
    pos = rng.uniform(-700, 700, (4, 3))
    radii = np.full(4, 100.0)
    L = 3
    lut = lut_for(pos, radii, k, L, 1.0)
    Wl = coupling_matrix(pos, k, L, hankel=lut)
    We = coupling_matrix(pos, k, L)
    assert np.linalg.norm(Wl - We) <= 1e-8 * np.linalg.norm(We)


def _two_sphere_z(L):
    return np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 430.0]]), np.array([100.0, 110.0])


@pytest.mark.parametrize("L", [1, 2, 3, 4])
@pytest.mark.parametrize("mode", ["direct", "lut"])
def test_apply_W_rows_equals_dense_coupling_matrix(L, mode):
    # The on-the-fly rows (Section 2.2, eq. a: (W x)^i = sum_{i' != i} A^T(r_i - r_i') x^{i'})
    # must equal the dense W times x.  The dense matrix is the one the reciprocity
    # and addition-theorem pins hold; the rows are assembled independently (a
    # per-receiver einsum over the source blocks), so a transposed contraction,
    # a wrong displacement sign or a self term included would fail here.
    from oracle.lut import lut_for
    from oracle.translation import apply_W_rows
    k = 2 * math.pi / 550
    rng = np.random.default_rng(100 + L)
    cases = []
    pos = rng.uniform(-900, 900, (6, 3))
    cases.append((pos, np.full(6, 100.0)))
    cases.append(_two_sphere_z(L))
    for pos, radii in cases:
        N = pos.shape[0]
        nm = 2 * L * (L + 2)
        hk = lut_for(pos, radii, k, L, 1.0) if mode == "lut" else None
        W = coupling_matrix(pos, k, L, hankel=hk)
        x = rng.standard_normal((N, nm)) + 1j * rng.standard_normal((N, nm))
        ref = (W @ x.reshape(-1)).reshape(N, nm)
        rows = list(range(N)) if N == 2 else [4, 0, 3]        # a non-contiguous, unsorted subset
        got = apply_W_rows(pos, x, k, L, rows, hankel=hk)
        assert np.abs(got - ref[rows]).max() <= 1e-14 * np.abs(ref).max(), (L, mode, N)


def test_apply_W_rows_z_pair_only_equal_m():
    # two spheres on the z axis: (W x)^i_n involves only the source entries with the
    # same m (axial pairs conserve m), so a unit source in one m leaves every other m
    # of the receiver at zero
    from oracle.translation import apply_W_rows
    k = 2 * math.pi / 550
    L = 3
    pos, _ = _two_sphere_z(L)
    ind = multi_indices(L)
    nm = len(ind)
    for col in (idx(1, 2, -1, L), idx(2, 3, 2, L)):
        x = np.zeros((2, nm), dtype=complex)
        x[1, col] = 1.0
        y = apply_W_rows(pos, x, k, L, [0])[0]
        m_src = ind[col][2]
        for a, (t, l, m) in enumerate(ind):
            if m != m_src:
                assert y[a] == 0
        assert np.abs(y).max() > 0


@pytest.mark.parametrize("mode", ["direct", "lut"])
def test_apply_W_rows_several_rhs_equals_dense(mode):
    # K right-hand sides at once ([K, N, nmax] in, [K, rows, nmax] out) against
    # the dense W applied to each column: a mixed-up right-hand-side axis or a
    # contraction over it would fail
    from oracle.lut import lut_for
    from oracle.translation import apply_W_rows
    k = 2 * math.pi / 550
    L = 2
    rng = np.random.default_rng(7)
    pos = rng.uniform(-800, 800, (5, 3))
    radii = np.full(5, 90.0)
    nm = 2 * L * (L + 2)
    hk = lut_for(pos, radii, k, L, 1.0) if mode == "lut" else None
    W = coupling_matrix(pos, k, L, hankel=hk)
    x = rng.standard_normal((3, 5, nm)) + 1j * rng.standard_normal((3, 5, nm))
    rows = [3, 1]
    got = apply_W_rows(pos, x, k, L, rows, hankel=hk)
    assert got.shape == (3, 2, nm)
    for kk in range(3):
        ref = (W @ x[kk].reshape(-1)).reshape(5, nm)
        assert np.abs(got[kk] - ref[rows]).max() <= 1e-14 * np.abs(ref).max()

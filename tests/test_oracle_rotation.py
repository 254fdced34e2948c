"""Pins of the oracle's basis rotation and of the rotation-translation-
rotation form of the translation operator (Section 5, Discussion), none of
which re-types the oracle's formulas: textbook values of the Wigner d
function, the rotation theorem checked point by point on the normalised
Legendre functions, unitarity, and the SVWF addition theorem evaluated with
the factorised translation at arbitrary displacements."""
import math

import numpy as np
import pytest

from oracle.rotation import basis_rotation, basis_rotation_l, translation_matrix_rtr, wigner_small_d
from oracle.special import legendre
from oracle.svwf import svwf
from oracle.translation import idx, multi_indices, translation_matrix


def test_wigner_d_textbook_values():
    # l = 1 and l = 2 entries of the standard tables (Edmonds, Sakurai)
    for b in (0.0, 0.4, 1.3, 2.2, math.pi):
        c, s = math.cos(b), math.sin(b)
        assert wigner_small_d(1, 0, 0, b) == pytest.approx(c, abs=1e-15)
        assert wigner_small_d(1, 1, 1, b) == pytest.approx((1 + c) / 2, abs=1e-15)
        assert wigner_small_d(1, 1, -1, b) == pytest.approx((1 - c) / 2, abs=1e-15)
        assert wigner_small_d(1, 1, 0, b) == pytest.approx(-s / math.sqrt(2), abs=1e-15)
        assert wigner_small_d(1, 0, 1, b) == pytest.approx(s / math.sqrt(2), abs=1e-15)
        assert wigner_small_d(2, 0, 0, b) == pytest.approx((3 * c * c - 1) / 2, abs=1e-15)
        assert wigner_small_d(2, 2, 2, b) == pytest.approx(((1 + c) / 2) ** 2, abs=1e-15)
        assert wigner_small_d(2, 1, 0, b) == pytest.approx(-math.sqrt(1.5) * s * c, abs=1e-15)
    # large l at a generic angle: d^l_{00} is the Legendre polynomial P_l(cos b)
    from scipy.special import eval_legendre
    for l in (10, 16, 24):
        assert wigner_small_d(l, 0, 0, 1.1) == pytest.approx(eval_legendre(l, math.cos(1.1)), abs=1e-14)


def _Rz(a):
    return np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1.0]])


def _Ry(b):
    return np.array([[math.cos(b), 0, math.sin(b)], [0, 1.0, 0], [-math.sin(b), 0, math.cos(b)]])


def _angular(l, v):
    # e^{i m phi} P_l^{|m|}(cos theta), m = -l..l, evaluated directly at the point v
    r = np.linalg.norm(v)
    ct, st = v[2] / r, math.hypot(v[0], v[1]) / r
    ph = math.atan2(v[1], v[0])
    return np.array([complex(legendre(l, abs(m), np.array(ct), np.array(st))) * np.exp(1j * m * ph)
                     for m in range(-l, l + 1)])


@pytest.mark.parametrize("phi,theta", [(0.7, 1.1), (-2.4, 0.2), (3.0, 2.9), (1.0, 0.0), (0.0, math.pi)])
def test_rotation_theorem_on_angular_functions(phi, theta):
    # f_l(R u) = U^l f_l(u) with R = R_z(phi) R_y(theta): the rotated-frame
    # functions evaluated at independent random points, l = 1..6
    R = _Rz(phi) @ _Ry(theta)
    rng = np.random.default_rng(11)
    for l in range(1, 7):
        U = basis_rotation_l(l, phi, theta)
        for _ in range(3):
            u = rng.normal(size=3)
            lhs = _angular(l, R @ u)
            assert np.abs(U @ _angular(l, u) - lhs).max() <= 1e-13 * max(1.0, np.abs(lhs).max()), l


def test_rotation_is_unitary_and_reduces_to_phases_on_the_axis():
    for l in (1, 3, 6):
        U = basis_rotation_l(l, 0.9, 1.7)
        assert np.abs(U @ U.conj().T - np.eye(2 * l + 1)).max() <= 1e-14
        U0 = basis_rotation_l(l, 0.9, 0.0)
        assert np.abs(U0 - np.diag([np.exp(1j * m * 0.9) for m in range(-l, l + 1)])).max() <= 1e-15


def test_sign_convention_is_what_the_theorem_fixes():
    # without the c_m signs (the Condon-Shortley form) the rotation theorem fails:
    # the pins above are sensitive to the convention
    phi, theta, l = 0.7, 1.1, 3
    ms = range(-l, l + 1)
    U_cs = np.array([[np.exp(1j * m * phi) * wigner_small_d(l, m, m2, theta) for m2 in ms] for m in ms])
    u = np.array([0.3, -0.8, 0.5])
    R = _Rz(phi) @ _Ry(theta)
    assert np.abs(U_cs @ _angular(l, u) - _angular(l, R @ u)).max() > 1e-2


@pytest.mark.parametrize("d", [(-3.3, 1.2, -1.9), (1e-9, 0.0, -5.0)])
def test_addition_theorem_with_rotated_translation(d):
    # Psi^(3)_n(r + d) = sum_n' A_{nn'}(d) Psi^(1)_n'(r) with A from the
    # rotation-translation-rotation form, generic and axial displacements
    k = 1.0
    d = np.array(d)
    Lp = 16
    A = translation_matrix_rtr(d, k, Lp, Lrow=4)
    rng = np.random.default_rng(1)
    r = rng.uniform(-0.25, 0.25, (3, 3))
    for (tau, l, m) in multi_indices(4):
        lhs = svwf(3, tau, l, m, r + d, k)
        rhs = 0
        for (tp, lp, mp) in multi_indices(Lp):
            c = A[idx(tau, l, m, Lp), idx(tp, lp, mp, Lp)]
            if abs(c) > 0:
                rhs = rhs + c * svwf(1, tp, lp, mp, r, k)
        assert np.abs(lhs - rhs).max() <= 1e-10 * np.abs(lhs).max(), (tau, l, m)


@pytest.mark.parametrize("L", [1, 3, 6])
def test_rotated_translation_equals_direct_blocks(L):
    k = 2 * math.pi / 550
    rng = np.random.default_rng(5 + L)
    for d in list(rng.uniform(-900, 900, (3, 3))) + [np.array([0, 0, 400.0]), np.array([0, 0, -380.0])]:
        A = translation_matrix(d, k, L)
        B = translation_matrix_rtr(d, k, L)
        assert np.abs(A - B).max() <= 1e-13 * np.abs(A).max()
    Az = translation_matrix(np.array([0, 0, 500.0]), k, L)
    ind = multi_indices(L)
    for a, (_, _, m) in enumerate(ind):
        for b, (_, _, m2) in enumerate(ind):
            if m != m2:
                assert Az[a, b] == 0

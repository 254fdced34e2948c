"""Pins for the exact Wigner-3j symbols: sympy (an independent exact
implementation), the orthogonality relation and the closed form of
(l l' p; 0 0 0)."""
import math
import random
from fractions import Fraction

from sympy.physics.wigner import wigner_3j

from oracle.wigner import wigner3j, wigner3j_exact


def test_against_sympy_exact():
    rnd = random.Random(5)
    for _ in range(300):
        j1, j2 = rnd.randint(0, 9), rnd.randint(0, 9)
        j3 = rnd.randint(abs(j1 - j2), j1 + j2)
        m1, m2 = rnd.randint(-j1, j1), rnd.randint(-j2, j2)
        ref = wigner_3j(j1, j2, j3, m1, m2, -m1 - m2)
        s, q = wigner3j_exact(j1, j2, j3, m1, m2, -m1 - m2)
        assert Fraction(int((ref ** 2).p), int((ref ** 2).q)) == q if ref != 0 else s == 0
        assert abs(wigner3j(j1, j2, j3, m1, m2, -m1 - m2) - float(ref)) < 1e-15


def test_orthogonality():
    for j1 in range(0, 4):
        for j2 in range(0, 4):
            for j3 in range(abs(j1 - j2), j1 + j2 + 1):
                for j3p in range(abs(j1 - j2), j1 + j2 + 1):
                    for m3 in range(-min(j3, j3p), min(j3, j3p) + 1):
                        s = 0.0
                        for m1 in range(-j1, j1 + 1):
                            m2 = -m1 - m3
                            if abs(m2) > j2:
                                continue
                            s += wigner3j(j1, j2, j3, m1, m2, m3) * wigner3j(j1, j2, j3p, m1, m2, m3)
                        want = 1.0 / (2 * j3 + 1) if j3 == j3p else 0.0
                        assert abs(s - want) < 1e-14


def test_zero_m_closed_form():
    f = math.factorial
    for l in range(0, 7):
        for lp in range(0, 7):
            for p in range(abs(l - lp), l + lp + 1):
                J = l + lp + p
                if J % 2:
                    assert wigner3j(l, lp, p, 0, 0, 0) == 0.0
                    continue
                g = J // 2
                v = (-1) ** g * math.sqrt(f(J - 2 * l) * f(J - 2 * lp) * f(J - 2 * p) / f(J + 1)) \
                    * f(g) / (f(g - l) * f(g - lp) * f(g - p))
                assert abs(wigner3j(l, lp, p, 0, 0, 0) - v) < 1e-15

"""Exact Wigner-3j symbols by the Racah formula, in rational arithmetic.

Used for the a5/b5 translation coefficients (paper, Appendix A.2).  A 3j
symbol is returned as (sign, square) with `square` an exact Fraction, so that
the value is sign * sqrt(square) without any rounding until the final
conversion.
"""
from fractions import Fraction
from math import factorial, isqrt


def _valid(j1, j2, j3, m1, m2, m3):
    if m1 + m2 + m3 != 0:
        return False
    if j3 < abs(j1 - j2) or j3 > j1 + j2:
        return False
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return False
    return True


def wigner3j_exact(j1, j2, j3, m1, m2, m3):
    """Return (sign, square) with 3j = sign * sqrt(square), integer arguments.

    Racah:  (j1 j2 j3; m1 m2 m3) = (-1)^{j1-j2-m3} sqrt(Delta) *
      sqrt((j1+m1)!(j1-m1)!(j2+m2)!(j2-m2)!(j3+m3)!(j3-m3)!) *
      sum_k (-1)^k / [k! (j3-j2+k+m1)! (j3-j1+k-m2)! (j1+j2-j3-k)!
                      (j1-k-m1)! (j2-k+m2)!],
    Delta = (j1+j2-j3)!(j1-j2+j3)!(-j1+j2+j3)!/(j1+j2+j3+1)!.
    """
    if not _valid(j1, j2, j3, m1, m2, m3):
        return 0, Fraction(0)
    f = factorial
    delta = Fraction(f(j1 + j2 - j3) * f(j1 - j2 + j3) * f(-j1 + j2 + j3), f(j1 + j2 + j3 + 1))
    pref = delta * f(j1 + m1) * f(j1 - m1) * f(j2 + m2) * f(j2 - m2) * f(j3 + m3) * f(j3 - m3)
    kmin = max(0, j2 - j3 - m1, j1 - j3 + m2)
    kmax = min(j1 + j2 - j3, j1 - m1, j2 + m2)
    s = Fraction(0)
    for k in range(kmin, kmax + 1):
        den = (f(k) * f(j3 - j2 + k + m1) * f(j3 - j1 + k - m2) * f(j1 + j2 - j3 - k)
               * f(j1 - k - m1) * f(j2 - k + m2))
        s += Fraction((-1) ** k, den)
    if s == 0:
        return 0, Fraction(0)
    sign = (-1) ** ((j1 - j2 - m3) % 2) * (1 if s > 0 else -1)
    return sign, pref * s * s


def frac_sqrt_float(q):
    """sqrt of a non-negative Fraction, correctly rounded to about 1 ulp."""
    if q == 0:
        return 0.0
    # scale to a large integer square root for full double precision
    num, den = q.numerator, q.denominator
    shift = 200
    r = isqrt((num << (2 * shift)) // den)
    return r / float(1 << shift) if r < (1 << 1000) else float(r) / 2.0 ** shift


def wigner3j(j1, j2, j3, m1, m2, m3):
    """Float value of the Wigner-3j symbol."""
    sign, sq = wigner3j_exact(j1, j2, j3, m1, m2, m3)
    if sign == 0:
        return 0.0
    return sign * frac_sqrt_float(sq)

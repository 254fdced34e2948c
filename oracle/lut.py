"""Spherical-Hankel lookup table with cubic interpolation (paper, Section
3.2.2: h_p(kd) tabulated over d at spacing dr and interpolated by cubic
splines).

Reading of the unspecified spline kind: a piecewise cubic *Hermite*
interpolant on a uniform grid, using the exact value and exact d-derivative of
h_p(kd) at every node, so each interval depends only on its two end nodes.

Grid (a deterministic function of the geometry, computed the same way by the
library):
    d_lo = max(dr, (floor(d_min / dr) - 1) dr),   d_min = 2 min_i R_i
    n_int = max(1, ceil((d_max - d_lo) / dr) + 1), d_max = |bounding-box diagonal of the centres|
    nodes d_k = d_lo + k dr, k = 0..n_int.
Interval index q = floor((d - d_lo)/dr), local t = (d - d_lo)/dr - q.

Two tables are defined here.  HankelLUT tabulates every order p = 0..2L, as
the paper describes.  HankelLUT01 tabulates only h_0 and h_1 and obtains the
higher orders from the three-term recurrence of the spherical Bessel family,
    h_{p+1}(x) = (2p + 1)/x h_p(x) - h_{p-1}(x),   x = k d,
which holds exactly for every solution of the spherical Bessel equation and
is stable upward for h_p (the y_p part dominates); the library's lookup-table
mode computes this second form.
"""
import math

import numpy as np

from .special import sph_h1, sph_h1_deriv


def lut_grid(positions, radii, dr):
    pos = np.asarray(positions, dtype=np.float64)
    d_min = 2.0 * float(np.min(radii))
    ext = pos.max(axis=0) - pos.min(axis=0)
    d_max = float(np.sqrt(np.sum(ext * ext)))
    d_lo = max(dr, (math.floor(d_min / dr) - 1) * dr)
    n_int = max(1, int(math.ceil((d_max - d_lo) / dr)) + 1)   # one sphere: no pairs, one interval
    return d_lo, n_int


class HankelLUT:
    """Hermite-interpolated h_p(k d), p = 0..pmax, on the grid above."""

    def __init__(self, k, pmax, d_lo, dr, n_int):
        self.k, self.pmax, self.d_lo, self.dr, self.n_int = k, pmax, d_lo, dr, n_int
        d = d_lo + dr * np.arange(n_int + 1)
        self.val = np.array([sph_h1(p, k * d) for p in range(pmax + 1)])           # [p, node]
        self.der = np.array([k * sph_h1_deriv(p, k * d) for p in range(pmax + 1)])  # d/dd

    def __call__(self, p, kd):
        d = np.asarray(kd, dtype=np.float64) / self.k
        s = (d - self.d_lo) / self.dr
        q = np.floor(s).astype(np.int64)
        if np.any(q < 0) or np.any(q >= self.n_int):
            raise ValueError("distance outside the lookup-table range")
        t = s - q
        h00 = 2 * t ** 3 - 3 * t ** 2 + 1
        h10 = t ** 3 - 2 * t ** 2 + t
        h01 = -2 * t ** 3 + 3 * t ** 2
        h11 = t ** 3 - t ** 2
        v, g = self.val[p], self.der[p] * self.dr
        return h00 * v[q] + h10 * g[q] + h01 * v[q + 1] + h11 * g[q + 1]


class HankelLUT01:
    """Hermite-interpolated h_0(k d) and h_1(k d) on the grid above; orders
    p >= 2 by the upward recurrence h_{p+1} = (2p+1)/x h_p - h_{p-1}."""

    def __init__(self, k, pmax, d_lo, dr, n_int):
        self.k, self.pmax = k, pmax
        self.d_lo, self.dr, self.n_int = d_lo, dr, n_int
        self.table = HankelLUT(k, 1, d_lo, dr, n_int)

    def __call__(self, p, kd):
        if p > self.pmax:
            raise ValueError("order above the table's cut-off")
        x = np.asarray(kd, dtype=np.float64)
        h_prev, h = self.table(0, x), self.table(1, x)
        if p == 0:
            return h_prev
        for q in range(1, p):
            h_prev, h = h, (2 * q + 1) / x * h - h_prev
        return h


def lut_for(positions, radii, k, L, dr):
    """The table the library's lookup-table mode evaluates (two tabulated
    orders plus the recurrence)."""
    d_lo, n_int = lut_grid(positions, radii, dr)
    return HankelLUT01(k, 2 * L, d_lo, dr, n_int)

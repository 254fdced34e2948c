"""Seeded sphere packings (random sequential addition) in a box.

Lengths are in nanometres throughout.  All randomness comes from numpy's PCG64
generator seeded explicitly, so a (seed, parameters) tuple always yields the
same packing on any machine.
"""
import numpy as np


def lognormal_radii(rng, n, mean, rel_sigma):
    """Radii with E[R] = mean and log-standard-deviation rel_sigma.

    The log-mean is shifted by -sigma^2/2 so that the arithmetic mean of the
    distribution equals `mean`.
    """
    s = float(rel_sigma)
    mu = np.log(mean) - 0.5 * s * s
    return rng.lognormal(mean=mu, sigma=s, size=n)


def slab_side_for_fraction(n, volume_fraction, thickness, mean, rel_sigma):
    """Lateral side of a square slab holding n lognormal spheres at a given
    volume fraction: side = sqrt(n <V> / (vf * t)), with
    <R^3> = mean^3 exp(3 sigma^2) for the shifted lognormal law."""
    r3 = mean ** 3 * np.exp(3.0 * rel_sigma ** 2)
    v = 4.0 / 3.0 * np.pi * r3
    return float(np.sqrt(n * v / (volume_fraction * thickness)))


def _cell_key(c):
    return (int(c[0]), int(c[1]), int(c[2]))


def rsa_box(seed, radii, box, max_attempts_per_sphere=1000, gap=0.0, inside=True, region=None):
    """Random sequential addition of spheres with the given radii into the
    axis-aligned box [0,bx] x [0,by] x [0,bz].  With inside=True every sphere
    lies fully inside the box; with inside=False only the centres do (spheres
    may protrude by up to their radius, so the box volume fraction can reach
    the bulk RSA range).

    Spheres are placed in the given order.  A candidate centre is drawn
    uniformly in the shrunken box and rejected if it comes within
    R_i + R_j + gap of an already placed sphere, or if `region` (a predicate
    on the centre) is given and returns False.  Raises RuntimeError after
    max_attempts_per_sphere * n total rejections.
    Returns positions [n, 3] (float64).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    radii = np.asarray(radii, dtype=np.float64)
    n = radii.size
    box = np.asarray(box, dtype=np.float64)
    rmax = float(radii.max())
    cell = 2.0 * rmax + gap
    grid = {}
    pos = np.zeros((n, 3))
    budget = max_attempts_per_sphere * n
    tries = 0
    for i in range(n):
        r = radii[i]
        lo = np.full(3, r) if inside else np.zeros(3)
        hi = box - r if inside else box.copy()
        if np.any(hi < lo):
            raise ValueError("sphere does not fit into the box")
        while True:
            tries += 1
            if tries > budget:
                raise RuntimeError("random sequential addition did not finish")
            c = lo + (hi - lo) * rng.random(3)
            if region is not None and not region(c):
                continue
            ck = np.floor(c / cell).astype(np.int64)
            ok = True
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        lst = grid.get((ck[0] + dx, ck[1] + dy, ck[2] + dz))
                        if not lst:
                            continue
                        for j in lst:
                            d = c - pos[j]
                            if d @ d <= (r + radii[j] + gap) ** 2:
                                ok = False
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                pos[i] = c
                grid.setdefault(_cell_key(ck), []).append(i)
                break
    return pos


def uniform_box(seed, n, radius, side, gap=0.0):
    """n equal spheres of the given radius, centres uniform with each sphere
    fully inside a cube of the given side, non-overlapping (by rejection)."""
    return rsa_box(seed, np.full(n, float(radius)), (side, side, side), gap=gap)


def rsa_cylinder(seed, radii, rcyl, thickness, max_attempts_per_sphere=1000):
    """Random sequential addition with centres uniform in the cylinder
    x^2 + y^2 <= rcyl^2, 0 <= z <= thickness (axis z, spheres may protrude by
    up to their radius).  Returns positions [n, 3] centred on the axis."""
    side = 2.0 * rcyl
    pos = rsa_box(seed, radii, (side, side, thickness), max_attempts_per_sphere, inside=False,
                  region=lambda c: (c[0] - rcyl) ** 2 + (c[1] - rcyl) ** 2 <= rcyl * rcyl)
    return pos - np.array([rcyl, rcyl, 0.0])


def rsa_ball(seed, radii, rball, max_attempts_per_sphere=1000):
    """Random sequential addition with centres uniform in the ball
    |c| <= rball (spheres may protrude by up to their radius).  Returns
    positions [n, 3] centred on the origin."""
    side = 2.0 * rball
    pos = rsa_box(seed, radii, (side, side, side), max_attempts_per_sphere, inside=False,
                  region=lambda c: (c[0] - rball) ** 2 + (c[1] - rball) ** 2 + (c[2] - rball) ** 2 <= rball * rball)
    return pos - np.array([rball, rball, rball])


def relax_pack_cylinder(seed, n, radius, rcyl, thickness, start=0.8, grow=1.004, max_sweeps=200000, tol=1e-9):
    """Dense random packing of n equal spheres with centres in the cylinder
    x^2 + y^2 <= rcyl^2, 0 <= z <= thickness (spheres may protrude by up to
    their radius, as in rsa_cylinder), for volume fractions beyond random
    sequential addition (the paper packs with Lubachevsky-Stillinger).

    Overlap relaxation with growth: centres start uniform in the cylinder
    with diameter start * 2 radius; each sweep finds all pairs closer than the current
    diameter (KD-tree), moves both spheres of each pair apart along their
    axis by half the overlap (plus a small margin), and projects the centres
    back into the cylinder; when a sweep finds no overlap the diameter grows
    by the factor `grow` until it reaches 2 radius.  Deterministic for a
    seed.  Raises RuntimeError if max_sweeps is exhausted.  Returns positions
    [n, 3] centred on the axis."""
    from scipy.spatial import cKDTree
    rng = np.random.Generator(np.random.PCG64(seed))
    rr = rcyl * np.sqrt(rng.random(n))
    ph = 2.0 * np.pi * rng.random(n)
    pos = np.stack([rr * np.cos(ph), rr * np.sin(ph), thickness * rng.random(n)], -1)
    target = 2.0 * radius
    d = start * target
    margin = 1.0 + 1e-3

    def project(p):
        r = np.hypot(p[:, 0], p[:, 1])
        out = r > rcyl
        p[out, 0] *= rcyl / r[out]
        p[out, 1] *= rcyl / r[out]
        np.clip(p[:, 2], 0.0, thickness, out=p[:, 2])

    for _ in range(max_sweeps):
        pairs = cKDTree(pos).query_pairs(d * (1.0 - tol), output_type="ndarray")
        if pairs.size == 0:
            if d >= target:
                return pos
            d = min(target, d * grow)
            continue
        i, j = pairs[:, 0], pairs[:, 1]
        v = pos[i] - pos[j]
        dist = np.linalg.norm(v, axis=1)
        small = dist < 1e-12 * d
        if np.any(small):     # coincident centres: separate along a seeded random direction
            u = rng.standard_normal((int(small.sum()), 3))
            v[small] = u / np.linalg.norm(u, axis=1)[:, None] * 1e-9 * d
            dist[small] = 1e-9 * d
        shift = (0.5 * (d * margin - dist) / dist)[:, None] * v
        disp = np.zeros_like(pos)
        np.add.at(disp, i, shift)
        np.add.at(disp, j, -shift)
        pos += disp
        project(pos)
    raise RuntimeError("relax_pack_cylinder: no overlap-free packing within max_sweeps")

"""Named synthetic workloads (geometry + illumination + numerics).

Every workload is a deterministic function of its name: the packing seed, the
radius law and the box are fixed here.  Lengths are nanometres.  The slab
workloads keep the sphere count, the volume fraction (0.3), the radius law
and the slab thickness, and derive the lateral side from them.
"""
from dataclasses import dataclass, field
import numpy as np

from .packing import relax_pack_cylinder, rsa_ball, rsa_box, rsa_cylinder, uniform_box, lognormal_radii, slab_side_for_fraction


@dataclass
class Workload:
    name: str
    positions: np.ndarray          # [N, 3] nm
    radii: np.ndarray              # [N] nm
    n_sphere: np.ndarray           # [N] complex refractive index
    n0: float
    wavelength: float              # vacuum wavelength, nm
    lmax: int
    illumination: dict             # {"kind": "plane", ...} or {"kind": "gaussian", ...}
    tol: float
    lut_dr: float = 1.0
    box: tuple = None
    extra: dict = field(default_factory=dict)

    @property
    def N(self):
        return self.positions.shape[0]

    @property
    def nmax(self):
        return 2 * self.lmax * (self.lmax + 2)


def _slab(name, seed, n, thickness, lmax, n_sph, illumination, tol, vf=0.3,
          mean=150.0, rel_sigma=0.1):
    rng = np.random.Generator(np.random.PCG64(seed))
    radii = lognormal_radii(rng, n, mean, rel_sigma)
    side = slab_side_for_fraction(n, vf, thickness, mean, rel_sigma)
    box = (side, side, thickness)
    pos = rsa_box(seed + 7919, radii, box, inside=False)
    # centre the slab laterally on the optical axis, entry face at z = 0
    pos = pos - np.array([side / 2, side / 2, 0.0])
    return Workload(name, pos, radii, np.full(n, complex(n_sph)), 1.0, 550.0, lmax,
                    illumination, tol, 1.0, box)


def _cylinder(name, seed, n, vf, thickness=2000.0, radius=100.0):
    """The application setting of the paper's Section 4: monodisperse spheres
    (R = 100 nm, n = 1.5) at a given volume fraction in a cylindrical slab,
    lambda = 532 nm, lmax 3, Gaussian beam (waist 4 um) focused on the centre
    of the entry face, GMRES tolerance 1e-4.  The slab's thickness is not
    stated there; 2 um is used and the cylinder radius follows from N and vf.
    Packing: random sequential addition up to vf 0.35, overlap relaxation
    with growth (relax_pack_cylinder) above."""
    rcyl = float(np.sqrt(n * 4.0 / 3.0 * np.pi * radius ** 3 / (vf * np.pi * thickness)))
    radii = np.full(n, radius)
    if vf <= 0.35:
        pos = rsa_cylinder(seed, radii, rcyl, thickness)
    else:     # beyond random sequential addition (the paper packs with Lubachevsky-Stillinger)
        pos = relax_pack_cylinder(seed, n, radius, rcyl, thickness)
    ill = {"kind": "gaussian", "waist": 4000.0, "focus": (0.0, 0.0, 0.0), "alpha_G": -np.pi / 2, "E0": 1.0}
    return Workload(name, pos, radii, np.full(n, 1.5 + 0j), 1.0, 532.0, 3, ill, 1e-4, 1.0,
                    (2 * rcyl, 2 * rcyl, thickness), {"cylinder_radius": rcyl})


def _ball(name, seed, n, vf, radius=100.0):
    """The validation target of the paper's Section 4: N spheres (R = 100 nm,
    n = 1.5) at volume fraction vf inside a spherical region centred on the
    origin, lambda = 532 nm, lmax 3, Gaussian beam (waist 4 um) focused on the
    centre.  The paper packs with Lubachevsky-Stillinger; at vf 0.1 random
    sequential addition reaches the same density."""
    rball = float(radius * (n / vf) ** (1.0 / 3.0))
    radii = np.full(n, radius)
    pos = rsa_ball(seed, radii, rball)
    ill = {"kind": "gaussian", "waist": 4000.0, "focus": (0.0, 0.0, 0.0), "alpha_G": 0.0, "E0": 1.0}
    return Workload(name, pos, radii, np.full(n, 1.5 + 0j), 1.0, 532.0, 3, ill, 1e-6, 1.0,
                    (2 * rball, 2 * rball, 2 * rball), {"ball_radius": rball})


def _small_cube():
    n, r, side = 8, 100.0, 1000.0
    pos = uniform_box(1, n, r, side)
    return Workload("cube8_l3", pos, np.full(n, r), np.full(n, 1.5 + 0.01j), 1.0, 550.0, 3,
                    {"kind": "plane", "beta": 0.0, "alpha": 0.0, "pol": 2, "E0": 1.0},
                    1e-10, 1.0, (side, side, side))


def _gauss(waist=2000.0):
    # focus at the centre of the slab's entry face, E0 along +x (alpha_G = -pi/2)
    return {"kind": "gaussian", "waist": waist, "focus": (0.0, 0.0, 0.0),
            "alpha_G": -np.pi / 2, "E0": 1.0}


def _plane_normal():
    return {"kind": "plane", "beta": 0.0, "alpha": 0.0, "pol": 2, "E0": 1.0}


_BUILDERS = {
    # the paper's run-time comparison setting (N = 2e4, vf 10 %, cylindrical slab)
    "paper_cyl20000_vf10": lambda: _cylinder("paper_cyl20000_vf10", 6001, 20000, 0.10),
    "paper_ball2500_vf10": lambda: _ball("paper_ball2500_vf10", 7001, 2500, 0.10),
    "paper_ball100000_vf10": lambda: _ball("paper_ball100000_vf10", 7002, 100000, 0.10),
    # 8 spheres, R = 100 nm, n = 1.5+0.01i, lmax 3, x-polarised plane wave along +z
    "cube8_l3": _small_cube,
    # 2,000-sphere slab, t = 2 um, lmax 4, Gaussian beam w = 2 um, FP64 GMRES 1e-8
    "slab2000_l4": lambda: _slab("slab2000_l4", 2, 2000, 2000.0, 4, 1.52, _gauss(), 1e-8),
    # 20,000-sphere slab, t = 3 um, lmax 4, Gaussian beam (mixed precision workload)
    "slab20000_l4": lambda: _slab("slab20000_l4", 3, 20000, 3000.0, 4, 1.52, _gauss(), 1e-8),
    # 10,000-sphere slab, t = 2 um, lmax 3 (multi-RHS workload)
    "slab10000_l3": lambda: _slab("slab10000_l3", 4, 10000, 2000.0, 3, 1.52, _plane_normal(), 1e-6),
    # small slabs used by tests (same statistics, fewer spheres)
    "slab64_l3": lambda: _slab("slab64_l3", 11, 64, 1000.0, 3, 1.52, _plane_normal(), 1e-10),
    "slab200_l4": lambda: _slab("slab200_l4", 12, 200, 1000.0, 4, 1.52, _gauss(1000.0), 1e-10),
    "slab300_l3": lambda: _slab("slab300_l3", 13, 300, 1000.0, 3, 1.52 + 0.02j, _plane_normal(), 1e-10),
    # 5,000-sphere slab, lmax 3: training geometry family for the warm start
    "slab5000_l3": lambda: _slab("slab5000_l3", 5001, 5000, 2000.0, 3, 1.52, _plane_normal(), 1e-6),
}

WORKLOADS = tuple(_BUILDERS)
_CACHE = {}


def cylinder_workload(n, vf, seed=6001, thickness=2000.0):
    """The paper's application setting (see _cylinder) for any N and volume
    fraction: R = 100 nm, n = 1.5, lambda = 532 nm, lmax 3, Gaussian beam
    waist 4 um, tolerance 1e-4, cylindrical slab of the given thickness."""
    return _cylinder(f"cyl_n{n}_vf{vf:g}", seed, n, vf, thickness)


def workload(name, seed=None, n=None):
    """Return the named workload.  `seed`/`n` override the slab seed/size for
    families of realisations (same statistics, different geometry)."""
    if seed is not None or n is not None:
        base = _BUILDERS[name]()
        th = base.box[2]
        return _slab(f"{name}_s{seed}_n{n}", seed if seed is not None else 0,
                     n if n is not None else base.N, th, base.lmax,
                     base.n_sphere[0], base.illumination, base.tol)
    if name not in _CACHE:
        _CACHE[name] = _BUILDERS[name]()
    return _CACHE[name]


def random_coefficients(seed, k, n, nmax, dtype=np.complex128):
    """Seeded random complex coefficient vectors, shape [k, n, nmax], with
    independent standard normal real and imaginary parts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal((k, n, nmax)) + 1j * rng.standard_normal((k, n, nmax))
    return x.astype(dtype)

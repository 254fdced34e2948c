"""Seeded inputs: deterministic, non-overlapping, right statistics."""
import numpy as np

from celes_inputs import workload, random_coefficients
from celes_inputs.packing import rsa_box, lognormal_radii


def test_workloads_deterministic_and_disjoint():
    for name in ("cube8_l3", "slab64_l3", "slab200_l4"):
        a = workload(name)
        b = workload.__wrapped__(name) if hasattr(workload, "__wrapped__") else workload(name)
        assert np.array_equal(a.positions, b.positions)
        d = np.linalg.norm(a.positions[:, None] - a.positions[None], axis=-1)
        np.fill_diagonal(d, np.inf)
        assert (d > a.radii[:, None] + a.radii[None, :]).all()


def test_lognormal_mean():
    rng = np.random.Generator(np.random.PCG64(0))
    r = lognormal_radii(rng, 200000, 150.0, 0.1)
    assert abs(r.mean() - 150.0) < 0.2
    assert abs(np.std(np.log(r)) - 0.1) < 1e-3


def test_rsa_reproducible():
    r = np.full(30, 50.0)
    p1 = rsa_box(7, r, (600, 600, 600))
    p2 = rsa_box(7, r, (600, 600, 600))
    assert np.array_equal(p1, p2)
    assert (p1 >= 50).all() and (p1 <= 550).all()


def test_random_coefficients_shape():
    x = random_coefficients(3, 2, 5, 30)
    assert x.shape == (2, 5, 30) and x.dtype == np.complex128


def test_rsa_cylinder_inside_disjoint_and_at_volume_fraction():
    from celes_inputs.packing import rsa_cylinder
    radii = np.full(400, 100.0)
    pos = rsa_cylinder(5, radii, 2000.0, 1000.0)
    assert np.all(pos[:, 0] ** 2 + pos[:, 1] ** 2 <= 2000.0 ** 2 + 1e-6)
    assert np.all((pos[:, 2] >= 0) & (pos[:, 2] <= 1000.0))
    d = np.linalg.norm(pos[:, None] - pos[None], axis=-1) + np.eye(len(pos)) * 1e9
    assert d.min() > 200.0
    np.testing.assert_array_equal(pos, rsa_cylinder(5, radii, 2000.0, 1000.0))
    # the named workload keeps N and vf 0.10 by construction of its radius
    w = workload("paper_cyl20000_vf10")
    rc, t = w.extra["cylinder_radius"], w.box[2]
    vf = w.N * 4 / 3 * np.pi * 100.0 ** 3 / (np.pi * rc * rc * t)
    assert abs(vf - 0.10) < 1e-9 and w.N == 20000 and w.wavelength == 532.0 and w.lmax == 3


def test_rsa_ball_validation_target():
    from celes_inputs.packing import rsa_ball
    radii = np.full(300, 100.0)
    pos = rsa_ball(9, radii, 1500.0)
    assert np.all(np.linalg.norm(pos, axis=1) <= 1500.0 + 1e-6)
    d = np.linalg.norm(pos[:, None] - pos[None], axis=-1) + np.eye(len(pos)) * 1e9
    assert d.min() > 200.0
    w = workload("paper_ball2500_vf10")
    rb = w.extra["ball_radius"]
    assert w.N == 2500 and abs(w.N * 100.0 ** 3 / rb ** 3 - 0.10) < 1e-9
    assert np.all(np.linalg.norm(w.positions, axis=1) <= rb + 1e-6)
    assert w.illumination["kind"] == "gaussian" and w.illumination["focus"] == (0.0, 0.0, 0.0)


def test_relax_pack_reaches_half_volume_fraction():
    from celes_inputs.packing import relax_pack_cylinder
    n, R, t, vf = 600, 100.0, 1000.0, 0.5
    rc = float(np.sqrt(n * 4 / 3 * np.pi * R ** 3 / (vf * np.pi * t)))
    pos = relax_pack_cylinder(3, n, R, rc, t)
    assert np.all(np.hypot(pos[:, 0], pos[:, 1]) <= rc + 1e-6)
    assert np.all((pos[:, 2] >= 0) & (pos[:, 2] <= t))
    d = np.linalg.norm(pos[:, None] - pos[None], axis=-1) + np.eye(n) * 1e9
    assert d.min() >= 2 * R * (1 - 1e-9)
    np.testing.assert_array_equal(pos, relax_pack_cylinder(3, n, R, rc, t))

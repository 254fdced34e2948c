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

"""Near field on the device through the C ABI: the scattered field against
the oracle's SVWF sum on the same coefficients for every compiled lmax
(including points on a sphere's polar axis), on a 200-sphere slab under a
Gaussian beam, and the incident field of a plane wave (its definition) and
of the Gaussian beam (the oracle's angular-spectrum quadrature)."""
import math

import numpy as np
import pytest

import paper_1706_02145_amd as P
from celes_inputs import workload
from oracle.incident import gaussian_beam_field
from oracle.observables import scattered_field
from tests.gpu_helpers import k_of, make_problem, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 6])
def test_scattered_near_field_every_lmax(L):
    print(f"[near] two spheres, lmax {L}", flush=True)
    pos = np.array([[0.0, 0.0, 0.0], [260.0, -90.0, 140.0]])
    p = P.Problem(pos, [100.0, 80.0], [1.5 + 0.01j, 2.0], 1.0, 550.0, L, hankel=P.CELES_HANKEL_DIRECT, tol=1e-12)
    p.set_plane_waves([0.4], [0.9], [2])
    b, _ = p.solve()
    pts = np.array([[0.0, 0.0, 150.0], [0.0, 0.0, -400.0], [260.0, -90.0, -20.0], [700.0, 300.0, 500.0],
                    [-150.0, 40.0, 60.0], [3000.0, -2000.0, 1000.0]])
    E = p.near_field(pts, add_incident=False)[0]
    ref = scattered_field(2 * math.pi / 550.0, pos, b[0], L, pts)
    assert rel(E, ref) <= 1e-11


def test_near_field_slab_gaussian_beam():
    w = workload("slab200_l4")
    print("[near] slab200_l4 scattered + Gaussian incident", flush=True)
    k = k_of(w)
    p = make_problem(w, hankel=1, tol=1e-10)
    b, _ = p.solve()
    xs = np.linspace(-1800.0, 1800.0, 9)
    zs = np.array([-500.0, 1500.0, 2500.0])
    pts = np.array([[x, 35.0, z] for x in xs for z in zs])
    d = np.linalg.norm(pts[:, None, :] - w.positions[None], axis=-1) - w.radii[None]
    pts = pts[d.min(axis=1) > 1.0]
    Es = p.near_field(pts, add_incident=False)[0]
    assert rel(Es, scattered_field(k, w.positions, b[0], w.lmax, pts)) <= 1e-11
    Et = p.near_field(pts, add_incident=True)[0]
    il = w.illumination
    Ei = gaussian_beam_field(pts, k, il["waist"], np.array(il["focus"]), il["alpha_G"], il["E0"])
    assert rel(Et - Es, Ei) <= 1e-11


def test_plane_wave_incident_near_field():
    w = workload("cube8_l3")
    print("[near] cube8_l3 plane-wave incident", flush=True)
    k = k_of(w)
    p = make_problem(w, hankel=1, tol=1e-10)
    p.solve()
    pts = np.array([[1500.0, 0, 0], [0, -1400.0, 300.0], [200.0, 200.0, 1600.0]])
    Ei = p.near_field(pts, add_incident=True)[0] - p.near_field(pts, add_incident=False)[0]
    il = w.illumination
    be, al = il["beta"], il["alpha"]
    kv = k * np.array([math.sin(be) * math.cos(al), math.sin(be) * math.sin(al), math.cos(be)])
    e = np.array([math.cos(be) * math.cos(al), math.cos(be) * math.sin(al), -math.sin(be)]) if il["pol"] == 2 \
        else np.array([-math.sin(al), math.cos(al), 0.0])
    ref = il["E0"] * np.exp(1j * pts @ kv)[:, None] * e[None]
    assert np.max(np.abs(Ei - ref)) <= 1e-12

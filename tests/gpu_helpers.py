"""Shared set-up for the GPU parity tests: the oracle side of each workload
(computed with oracle/ only) and the library side (through the C ABI)."""
import math

import numpy as np

from celes_inputs import workload
from oracle.incident import gaussian_beam_coefficients, plane_wave_coefficients
from oracle.lut import lut_for
from oracle.mie import T_vector


def k_of(w):
    return 2 * math.pi * w.n0 / w.wavelength


def oracle_incident(w):
    k = k_of(w)
    il = w.illumination
    if il["kind"] == "plane":
        return plane_wave_coefficients(w.positions, k, w.lmax, il["beta"], il["alpha"], il["pol"], il["E0"])
    return gaussian_beam_coefficients(w.positions, k, w.lmax, il["waist"], il["focus"], il["alpha_G"], il["E0"])


def oracle_lut(w, dr=None):
    return lut_for(w.positions, w.radii, k_of(w), w.lmax, dr or w.lut_dr)


def make_problem(w, **opts):
    import paper_1706_02145_amd as P
    p = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, **opts)
    il = w.illumination
    if il["kind"] == "plane":
        p.set_plane_waves([il["beta"]], [il["alpha"]], [il["pol"]], [il["E0"]])
    else:
        p.set_gaussian_beam(il["waist"], il["focus"], il["alpha_G"], il["E0"])
    return p


def tvec(w):
    return T_vector(w.lmax, k_of(w), w.radii, w.n_sphere, w.n0)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))

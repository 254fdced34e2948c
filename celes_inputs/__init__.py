"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds only input generation: sphere packings, radius draws,
illumination parameters and random coefficient vectors.  It contains none of
the scattering arithmetic, so that the CPU oracle and the HIP library can both
consume identical inputs while sharing no method code.
"""
from .packing import relax_pack_cylinder, rsa_ball, rsa_box, rsa_cylinder, uniform_box, lognormal_radii, slab_side_for_fraction
from .workloads import Workload, workload, cylinder_workload, WORKLOADS, random_coefficients

__all__ = ["relax_pack_cylinder", "rsa_ball", "rsa_box", "rsa_cylinder", "uniform_box", "lognormal_radii", "slab_side_for_fraction",
           "Workload", "workload", "cylinder_workload", "WORKLOADS", "random_coefficients"]

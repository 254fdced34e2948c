"""Sub-ensemble initial guess (Section 4.2) on the GPU, through the C ABI:
the guess against the oracle's (dense LU of the sub-ensemble), its use as
x0 of the full solve (fewer iterations, same solution), the whole ensemble
as sub-ensemble, options inherited by the sub-solve, and argument errors."""
import numpy as np
import pytest

import paper_1706_02145_amd as P
from celes_inputs import workload
from oracle.solve import master_matrix, solve_dense, subsystem_initial_guess
from tests.gpu_helpers import make_problem, oracle_incident, rel

pytestmark = pytest.mark.gpu


def _central(w, radius):
    r = np.hypot(w.positions[:, 0], w.positions[:, 1])
    return np.nonzero(r < radius)[0]


def test_guess_matches_oracle_and_shortens_the_solve():
    w = workload("slab200_l4")
    idx = _central(w, 1000.0)
    print(f"[subsystem] slab200_l4, {idx.size} central spheres", flush=True)
    a = oracle_incident(w)
    x_ref = subsystem_initial_guess(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, a, idx)
    p = make_problem(w, hankel=1, tol=1e-11)
    x0, sinfo = p.subsystem_guess(idx)
    assert sinfo["status"] == 0 and sinfo["rel_residual"] <= 1e-11
    assert rel(x0[0], x_ref) <= 1e-9
    assert not np.any(np.delete(x0[0], idx, axis=0))
    b0, i0 = p.solve()
    b1, i1 = p.solve(x0=x0)
    print(f"[subsystem] iterations from zero {i0['iterations']}, from the guess {i1['iterations']}", flush=True)
    assert i1["x0_used"] == 1 and i1["status"] == 0
    assert i1["iterations"] < i0["iterations"]
    assert rel(b1, b0) <= 1e-9


def test_whole_ensemble_guess_is_the_solution():
    w = workload("slab64_l3")
    print("[subsystem] slab64_l3 whole ensemble", flush=True)
    M, W, t = master_matrix(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax)
    bref = solve_dense(M, t * oracle_incident(w).reshape(-1)).reshape(w.N, -1)
    p = make_problem(w, hankel=1, tol=1e-12)
    x0, _ = p.subsystem_guess(np.arange(w.N)[::-1].copy(), cuboid_edge=700.0)
    assert rel(x0[0], bref) <= 1e-10
    _, info = p.solve(x0=x0)
    assert info["iterations"] == 0 and info["x0_used"] == 1


def test_guess_inherits_mixed_bicgstab_options():
    w = workload("slab64_l3")
    idx = _central(w, 600.0)
    print(f"[subsystem] slab64_l3 mixed BiCGSTAB sub-solve, {idx.size} spheres", flush=True)
    a = oracle_incident(w)
    x_ref = subsystem_initial_guess(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, a, idx)
    p = make_problem(w, hankel=1, tol=1e-9, precision=P.CELES_MIXED, solver=P.CELES_SOLVER_BICGSTAB)
    x0, sinfo = p.subsystem_guess(idx)
    assert sinfo["status"] == 0 and sinfo["refinements"] >= 1
    assert rel(x0[0], x_ref) <= 1e-8


def test_guess_argument_errors():
    w = workload("cube8_l3")
    p = make_problem(w)
    for bad in ([0, 0], [8], [-1], []):
        with pytest.raises(P.CelesError) as e:
            p.subsystem_guess(bad)
        assert e.value.name == "CELES_E_ARG"

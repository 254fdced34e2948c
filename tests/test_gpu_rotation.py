"""GPU parity of the rotation-translation-rotation mat-vec (celes_options
.translation = CELES_TRANSLATION_ROTATE; Section 5, Discussion) against the
oracle's W, element by element, at lmax 1-6, both Hankel modes, axial pairs,
several right-hand sides, the M x epilogue and a solve.  FP64 bar 1e-9
relative (norm-wise; measured far below), complex64 bar 1e-4."""
import os

import numpy as np
import pytest

import paper_1706_02145_amd as P
from celes_inputs import random_coefficients, workload
from celes_inputs.packing import rsa_box
from oracle.lut import lut_for
from oracle.translation import apply_W_rows, coupling_matrix
from tests.gpu_helpers import k_of, make_problem, oracle_lut, rel, tvec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROT = P.CELES_TRANSLATION_ROTATE


def _cluster(n, L, seed):
    radii = np.full(n, 90.0)
    pos = rsa_box(seed, radii[:n - 2], (1400.0, 1400.0, 1400.0), inside=False)
    # plus two spheres on a common z axis outside the box (pairs along +z and -z)
    axial = np.array([[2400.0, 2300.0, 100.0], [2400.0, 2300.0, 530.0]])
    return np.concatenate([pos, axial]), radii


def _gpu_W(p, x, precision=P.CELES_FP64, op="W", K=1):
    dt = torch.complex128 if precision == P.CELES_FP64 else torch.complex64
    xd = torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dt)
    yd = torch.empty_like(xd)
    (p.apply_W if op == "W" else p.apply_M)(xd, yd, precision, K=K)
    torch.cuda.synchronize()
    return yd.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("hankel", [1, 0])
def test_rotated_matvec_all_rows(L, hankel):
    n = 40 if L <= 4 else 24
    pos, radii = _cluster(n, L, 300 + L)
    print(f"[rotation] L={L} hankel={hankel} N={n}", flush=True)
    k = 2 * np.pi / 550.0
    nm = 2 * L * (L + 2)
    x = random_coefficients(200 + L, 1, n, nm)[0]
    p = P.Problem(pos, radii, 1.52, 1.0, 550.0, L, hankel=hankel, translation=ROT)
    os.environ["CELES_WX_TARGET_BLOCKS"] = "16"          # several source chunks per receiver block
    try:
        y = _gpu_W(p, x)
        y32 = _gpu_W(p, x, precision=P.CELES_MIXED)
    finally:
        os.environ.pop("CELES_WX_TARGET_BLOCKS")
    hk = lut_for(pos, radii, k, L, 1.0) if hankel == 0 else None
    ref = (coupling_matrix(pos, k, L, hankel=hk) @ x.reshape(-1)).reshape(n, nm)
    e = rel(y, ref)
    print(f"[rotation] L={L} fp64 {e:.2e} fp32 {rel(y32, ref):.2e}", flush=True)
    assert e <= 1e-12
    rn = np.linalg.norm(ref, axis=1)
    assert (np.linalg.norm(y - ref, axis=1) <= 1e-10 * rn).all()
    assert rel(y32, ref) <= 1e-4


def test_rotated_matches_direct_on_a_slab_with_several_rhs():
    # 300 spheres, 3 right-hand sides, several receiver blocks: the two schemes
    # evaluate the same W, so they agree to summation order
    w = workload("slab300_l3")
    x = random_coefficients(210, 3, w.N, w.nmax)
    pr = make_problem(w, hankel=0, translation=ROT)
    pd = make_problem(w, hankel=0)
    yr = _gpu_W(pr, x, K=3)
    yd = _gpu_W(pd, x, K=3)
    assert rel(yr, yd) <= 1e-12
    rows = [0, 77, 150, 299]
    ref = apply_W_rows(w.positions, x, k_of(w), w.lmax, rows, hankel=oracle_lut(w))
    assert rel(yr[:, rows], ref) <= 1e-12


def test_rotated_epilogue_and_solve():
    w = workload("cube8_l3")
    from oracle.incident import plane_wave_coefficients
    from oracle.solve import master_matrix, solve_dense
    x = random_coefficients(211, 1, w.N, w.nmax)[0]
    p = make_problem(w, hankel=1, translation=ROT, tol=1e-11)
    y = _gpu_W(p, x, op="M")
    Wx = apply_W_rows(w.positions, x, k_of(w), w.lmax, range(w.N))
    assert rel(y, x - tvec(w) * Wx) <= 1e-12
    b, info = p.solve()
    M, W, t = master_matrix(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax)
    il = w.illumination
    a = plane_wave_coefficients(w.positions, k_of(w), w.lmax, il["beta"], il["alpha"], il["pol"])
    assert info["status"] == 0 and rel(b[0].reshape(-1), solve_dense(M, t * a.reshape(-1))) <= 1e-9


def test_switching_the_scheme_between_calls():
    # celes_set_solve_options changes the scheme of an existing handle: the
    # result then equals that of a handle created with it (same kernels, same
    # source chunks: identical bits), and switching back restores the direct one
    w = workload("slab64_l3")
    x = random_coefficients(212, 1, w.N, w.nmax)[0]
    p = make_problem(w, hankel=0)
    yd = _gpu_W(p, x)
    p.set_solve_options(translation=ROT)
    yr = _gpu_W(p, x)
    q = make_problem(w, hankel=0, translation=ROT)
    assert np.array_equal(yr, _gpu_W(q, x))
    p.set_solve_options(translation=P.CELES_TRANSLATION_DIRECT)
    assert np.array_equal(yd, _gpu_W(p, x))
    assert rel(yr, yd) <= 1e-12
    with pytest.raises(P.CelesError):
        p.set_solve_options(translation=7)


def test_rotated_matvec_full_size_sampled_rows():
    # the 20,000-sphere benchmark slab (lmax 4, LUT), in the launch
    # configuration the benchmark times: FP64 and complex64 rotation-scheme
    # W x against the oracle's rows on sampled receivers
    w = workload("slab20000_l4")
    print("[rotation] slab20000_l4 sampled rows", flush=True)
    x = random_coefficients(213, 1, w.N, w.nmax)[0]
    p = make_problem(w, hankel=0, translation=ROT)
    y = _gpu_W(p, x)
    y32 = _gpu_W(p, x, precision=P.CELES_MIXED)
    rows = [0, 4999, 12345, 19999]
    ref = apply_W_rows(w.positions, x, k_of(w), w.lmax, rows, hankel=oracle_lut(w))
    e, e32 = rel(y[rows], ref), rel(y32[rows], ref)
    print(f"[rotation] slab20000 fp64 {e:.2e} fp32 {e32:.2e}", flush=True)
    assert e <= 1e-11 and e32 <= 1e-4

"""Batched solves (many problems and right-hand sides in one persistent
launch per Arnoldi step) against individual solves and the oracle."""
import os

import numpy as np
import pytest

import paper_1706_02145_amd as P
from celes_inputs import workload, random_coefficients
from oracle.solve import master_matrix, solve_dense
from oracle.incident import plane_wave_coefficients
from tests.gpu_helpers import k_of, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ANGLES = {"slab300_l3": ([0.0, 0.3, 0.6, 1.0], [0.0, 0.5, 1.0, 2.0], [1, 2, 1, 2]),
          "slab64_l3": ([0.0, 0.8], [0.0, 0.4], [1, 2]),
          "cube8_l3": ([0.2, 0.2], [0.1, 0.1], [1, 2])}


def _problems(names, **opts):
    out = []
    for nm in names:
        w = workload(nm)
        p = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, hankel=1, **opts)
        b, a, pol = ANGLES[nm]
        p.set_plane_waves(b, a, pol)
        out.append((w, p))
    return out


TRANSLATIONS = [P.CELES_TRANSLATION_DIRECT, P.CELES_TRANSLATION_ROTATE]


@pytest.mark.parametrize("translation", TRANSLATIONS)
def test_batch_apply_M_matches_single_problem_launches(translation):
    # the persistent kernel of either translation scheme against the
    # single-problem launches of the same scheme
    probs = _problems(["slab300_l3", "slab64_l3", "cube8_l3"], translation=translation)
    print(f"[batch] apply_M 3 problems, translation {translation}", flush=True)
    bt = P.Batch([p for _, p in probs], hankel=1, translation=translation)     # the problems' Hankel mode
    assert bt.num_systems == 8
    xs = [random_coefficients(20 + i, p.num_rhs, w.N, w.nmax) for i, (w, p) in enumerate(probs)]
    flat = np.concatenate([x.reshape(-1) for x in xs])
    # FP64: same arithmetic, other source-chunk split (summation order only)
    for prec, dt, tolr in ((P.CELES_FP64, torch.complex128, 1e-13), (P.CELES_MIXED, torch.complex64, 1e-5)):
        xd = torch.from_numpy(flat).to("cuda", dt)
        yd = torch.empty_like(xd)
        bt.apply_M(xd, yd, prec)
        torch.cuda.synchronize()
        y = yd.cpu().numpy().astype(np.complex128)
        off = 0
        for (w, p), x in zip(probs, xs):
            xi = torch.from_numpy(x).to("cuda", dt)
            yi = torch.empty_like(xi)
            p.apply_M(xi, yi, prec, K=p.num_rhs)
            torch.cuda.synchronize()
            ref = yi.cpu().numpy().astype(np.complex128).reshape(-1)
            assert rel(y[off:off + ref.size], ref) <= tolr
            off += ref.size


@pytest.mark.parametrize("translation", TRANSLATIONS)
@pytest.mark.parametrize("precision", [P.CELES_MIXED, P.CELES_FP64])
def test_batch_solve_matches_individual_and_dense(precision, translation):
    names = ["slab300_l3", "slab64_l3", "cube8_l3"]
    probs = _problems(names, tol=1e-10)
    print(f"[batch] solve precision={precision} translation={translation}", flush=True)
    bt = P.Batch([p for _, p in probs], tol=1e-10, precision=precision, inner_tol=1e-4, restart=60, hankel=1,
                 translation=translation)
    per, summ = bt.solve()
    assert summ["status"] == 0 and summ["rel_residual"] <= 1e-10
    assert all(i["rel_residual"] <= 1e-10 for i in per)
    for w, p in probs:
        bb = p.solution()
        q = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, hankel=1, tol=1e-11)
        bq, a, pol = ANGLES[w.name]
        q.set_plane_waves(bq, a, pol)
        ref, _ = q.solve()
        assert rel(bb, ref) <= 1e-6
    # the two smaller problems against the oracle's dense LU (exact Hankel
    # functions, as the batch ran): FP64 to the FP64 bar, mixed to the mixed bar
    bar = 1e-9 if precision == P.CELES_FP64 else 1e-6
    for w, p in probs[1:]:
        M, W, t = master_matrix(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax)
        bq, a, pol = ANGLES[w.name]
        for k in range(len(bq)):
            ain = plane_wave_coefficients(w.positions, k_of(w), w.lmax, bq[k], a[k], pol[k])
            ref = solve_dense(M, t * ain.reshape(-1))
            assert rel(p.solution()[k].reshape(-1), ref) <= bar


def test_batch_graph_replay_equals_eager_and_autotune():
    names = ["slab300_l3", "slab64_l3"]
    probs = _problems(names)
    bt = P.Batch([p for _, p in probs], tol=1e-8, precision=P.CELES_MIXED, restart=40)
    _, s1 = bt.solve()
    sol1 = [p.solution() for _, p in probs]
    os.environ["CELES_NO_GRAPH"] = "1"
    try:
        _, s2 = bt.solve()
    finally:
        os.environ.pop("CELES_NO_GRAPH")
    sol2 = [p.solution() for _, p in probs]
    for a, b in zip(sol1, sol2):
        assert rel(a, b) <= 1e-12      # identical kernel sequence: bitwise up to launch order
    assert s1["iterations"] == s2["iterations"]
    t = bt.autotune(P.CELES_MIXED)
    print("[batch] autotune", t, flush=True)
    assert t["ms"] > 0 and t["chunk_len"] in (64, 128, 256, 512, 1024) and t["kb"] in (1, 2, 4)
    _, s3 = bt.solve()
    for (w, p), a in zip(probs, sol1):
        assert rel(p.solution(), a) <= 1e-6


def test_batch_with_matrix_core_problem():
    # 32 incidence directions on one slab fill a 32-wide matrix-core block
    # (lmax 3); the other problems stay on the VALU kernel in the same batch
    w = workload("slab64_l3")
    beta = np.repeat(np.linspace(0.0, np.pi / 3, 16), 2)
    alpha = np.zeros(32)
    pol = np.tile([1, 2], 16)
    big = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, hankel=0, tol=1e-10)
    big.set_plane_waves(beta, alpha, pol)
    rest = _problems(["slab300_l3", "cube8_l3"], tol=1e-10)
    bt = P.Batch([big] + [p for _, p in rest], tol=1e-9, precision=P.CELES_MIXED, inner_tol=1e-4, restart=60)
    print("[batch] matrix-core problem K=32 + 2 VALU problems", flush=True)
    # apply_M: batch vs single-problem launches of both precisions
    x = random_coefficients(40, 32, w.N, w.nmax)
    xs = [x] + [random_coefficients(41 + i, p.num_rhs, ww.N, ww.nmax) for i, (ww, p) in enumerate(rest)]
    flat = np.concatenate([v.reshape(-1) for v in xs])
    xd = torch.from_numpy(flat).to("cuda", torch.complex64)
    yd = torch.empty_like(xd)
    bt.apply_M(xd, yd, P.CELES_MIXED)
    torch.cuda.synchronize()
    y = yd.cpu().numpy().astype(np.complex128)
    xi = torch.from_numpy(x).to("cuda", torch.complex128)
    yi = torch.empty_like(xi)
    big.apply_M(xi, yi, P.CELES_FP64, K=32)
    torch.cuda.synchronize()
    ref = yi.cpu().numpy().reshape(-1)
    e = rel(y[:ref.size], ref)
    print(f"[batch] matrix-core apply_M vs FP64 {e:.2e}", flush=True)
    assert e <= 1e-5
    # mixed solve of the whole batch against FP64 single solves
    per, summ = bt.solve()
    assert summ["status"] == 0 and summ["rel_residual"] <= 1e-9
    q = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, hankel=0, tol=1e-11)
    q.set_plane_waves(beta, alpha, pol)
    ref_b, _ = q.solve()
    assert rel(big.solution(), ref_b) <= 1e-6


@pytest.mark.parametrize("precision", [P.CELES_MIXED, P.CELES_FP64])
def test_batch_with_block_preconditioners(precision):
    # per-problem block-diagonal preconditioners inside the batch (right
    # preconditioning in the captured step): same solutions, fewer iterations
    # for the preconditioned problems; a rebuilt preconditioner re-captures the
    # step; removing them returns to the unpreconditioned run
    probs = _problems(["slab300_l3", "slab64_l3", "cube8_l3"], tol=1e-10)
    print(f"[batch] block preconditioners precision={precision}", flush=True)
    bt = P.Batch([p for _, p in probs], tol=1e-10, precision=precision, inner_tol=1e-4, restart=60, hankel=1)
    per0, s0 = bt.solve()
    sol0 = [p.solution() for _, p in probs]
    probs[0][1].build_preconditioner(700.0)
    probs[1][1].build_preconditioner(700.0)
    per1, s1 = bt.solve()
    print(f"[batch] iterations without {[i['iterations'] for i in per0]} with {[i['iterations'] for i in per1]}",
          flush=True)
    assert s1["status"] == 0 and s1["rel_residual"] <= 1e-10
    for (w, p), a in zip(probs, sol0):
        assert rel(p.solution(), a) <= 1e-7
    assert per1[0]["iterations"] < per0[0]["iterations"]
    # the preconditioned slab64 solutions against the oracle's dense LU
    bar = 1e-9 if precision == P.CELES_FP64 else 1e-6
    w, p = probs[1]
    M, W, t = master_matrix(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax)
    bq, a, pol = ANGLES[w.name]
    for k in range(len(bq)):
        ain = plane_wave_coefficients(w.positions, k_of(w), w.lmax, bq[k], a[k], pol[k])
        assert rel(p.solution()[k].reshape(-1), solve_dense(M, t * ain.reshape(-1))) <= bar
    probs[0][1].build_preconditioner(500.0)
    per2, s2 = bt.solve()
    assert s2["status"] == 0 and s2["rel_residual"] <= 1e-10
    assert rel(probs[0][1].solution(), sol0[0]) <= 1e-7
    probs[0][1].build_preconditioner(0.0)
    probs[1][1].build_preconditioner(0.0)
    per3, s3 = bt.solve()
    assert all(abs(a["iterations"] - b["iterations"]) <= 1 for a, b in zip(per3, per0))
    for (w, p), a in zip(probs, sol0):
        assert rel(p.solution(), a) <= 1e-7


def test_batch_matrix_core_problem_with_preconditioner():
    # a >= 16-right-hand-side problem (its W x on the matrix cores) with a
    # block-diagonal preconditioner inside a batch, against its own
    # preconditioned single solve and the oracle's dense LU
    w = workload("slab64_l3")
    beta = np.repeat(np.linspace(0.0, np.pi / 3, 8), 2)
    alpha = np.zeros(16)
    pol = np.tile([1, 2], 8)
    big = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, hankel=1, tol=1e-10)
    big.set_plane_waves(beta, alpha, pol)
    big.build_preconditioner(700.0)
    rest = _problems(["cube8_l3"], tol=1e-10)
    print("[batch] matrix-core problem K=16 with preconditioner", flush=True)
    bt = P.Batch([big] + [p for _, p in rest], tol=1e-10, precision=P.CELES_MIXED, inner_tol=1e-4, restart=60,
                 hankel=1)
    per, summ = bt.solve()
    assert summ["status"] == 0 and summ["rel_residual"] <= 1e-10
    q = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax, hankel=1, tol=1e-11)
    q.set_plane_waves(beta, alpha, pol)
    q.build_preconditioner(700.0)
    ref_b, iq = q.solve()
    assert iq["status"] == 0
    assert rel(big.solution(), ref_b) <= 1e-6
    M, W, t = master_matrix(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, w.lmax)
    for k in (0, 5, 15):
        ain = plane_wave_coefficients(w.positions, k_of(w), w.lmax, beta[k], alpha[k], pol[k])
        assert rel(big.solution()[k].reshape(-1), solve_dense(M, t * ain.reshape(-1))) <= 1e-6

"""GPU parity of the on-the-fly coupling mat-vec (the hot path) against the
oracle, element by element.  FP64 bar: 1e-9 relative (norm-wise); FP32 bar:
1e-4 (reported values are far below)."""
import os

import numpy as np
import pytest

import paper_1706_02145_amd as P
from celes_inputs import workload, random_coefficients
from oracle.translation import apply_W_rows
from tests.gpu_helpers import k_of, make_problem, oracle_lut, rel, tvec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(x, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype=dtype)


def _gpu_W(p, x, precision=P.CELES_FP64, op="W"):
    dt = torch.complex128 if precision == P.CELES_FP64 else torch.complex64
    xd = _dev(x, dt)
    yd = torch.empty_like(xd)
    (p.apply_W if op == "W" else p.apply_M)(xd, yd, precision)
    torch.cuda.synchronize()
    return yd.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("name,hankel", [("cube8_l3", 1), ("cube8_l3", 0), ("slab300_l3", 1), ("slab300_l3", 0),
                                         ("slab64_l3", 0)])
def test_apply_W_fp64_all_rows(name, hankel):
    w = workload(name)
    print(f"[matvec fp64] {name} hankel={hankel} N={w.N}", flush=True)
    x = random_coefficients(100, 1, w.N, w.nmax)[0]
    p = make_problem(w, hankel=hankel)
    y = _gpu_W(p, x)
    hk = oracle_lut(w) if hankel == 0 else None
    ref = apply_W_rows(w.positions, x, k_of(w), w.lmax, range(w.N), hankel=hk)
    assert rel(y, ref) <= 1e-12
    # element-wise: every row within 1e-10 of its own norm
    rn = np.linalg.norm(ref, axis=1)
    assert (np.linalg.norm(y - ref, axis=1) <= 1e-10 * rn + 1e-300).all()


def test_apply_W_l4_and_chunking_invariance():
    w = workload("slab200_l4")
    print(f"[matvec fp64] slab200_l4 N={w.N}", flush=True)
    x = random_coefficients(101, 1, w.N, w.nmax)[0]
    p = make_problem(w, hankel=0)
    ys = []
    for tb in ("1", "64", "100000"):
        os.environ["CELES_WX_TARGET_BLOCKS"] = tb
        ys.append(_gpu_W(p, x))
    os.environ.pop("CELES_WX_TARGET_BLOCKS")
    rows = list(range(0, w.N, 7)) + [w.N - 1]
    ref = apply_W_rows(w.positions, x, k_of(w), w.lmax, rows, hankel=oracle_lut(w))
    for y in ys:
        assert rel(y[rows], ref) <= 1e-12
    # different source chunkings only change the summation order
    assert rel(ys[0], ys[2]) <= 1e-13


def test_apply_M_epilogue():
    w = workload("slab64_l3")
    x = random_coefficients(102, 1, w.N, w.nmax)[0]
    p = make_problem(w, hankel=1)
    y = _gpu_W(p, x, op="M")
    Wx = apply_W_rows(w.positions, x, k_of(w), w.lmax, range(w.N))
    ref = x - tvec(w) * Wx
    assert rel(y, ref) <= 1e-12


@pytest.mark.parametrize("hankel", [0, 1])
def test_apply_W_fp32(hankel):
    w = workload("slab300_l3")
    x = random_coefficients(103, 1, w.N, w.nmax)[0]
    p = make_problem(w, hankel=hankel)
    y = _gpu_W(p, x, precision=P.CELES_MIXED)
    hk = oracle_lut(w) if hankel == 0 else None
    ref = apply_W_rows(w.positions, x.astype(np.complex64).astype(np.complex128), k_of(w), w.lmax,
                       range(w.N), hankel=hk)
    e = rel(y, ref)
    print(f"[matvec fp32] hankel={hankel} rel err {e:.2e}")
    assert e <= 1e-4


def test_full_size_slab2000_sampled_rows():
    w = workload("slab2000_l4")
    print(f"[matvec fp64] slab2000_l4 N={w.N} (bench configuration)", flush=True)
    x = random_coefficients(104, 1, w.N, w.nmax)[0]
    p = make_problem(w, hankel=0)
    y = _gpu_W(p, x)
    rng = np.random.default_rng(5)
    rows = sorted(set(rng.choice(w.N, 6, replace=False).tolist() + [0, w.N - 1]))
    ref = apply_W_rows(w.positions, x, k_of(w), w.lmax, rows, hankel=oracle_lut(w))
    assert rel(y[rows], ref) <= 1e-12
    # LUT vs exact Hankel: within the interpolation error bound (~1e-8)
    ref_exact = apply_W_rows(w.positions, x, k_of(w), w.lmax, rows[:2])
    assert rel(y[rows[:2]], ref_exact) <= 1e-7


def test_reciprocity_at_full_size():
    # u^T (W v) = (Pi v)^T (W Pi u): a property of W that holds at any size
    w = workload("slab2000_l4")
    p = make_problem(w, hankel=1)
    u = random_coefficients(7, 1, w.N, w.nmax)[0]
    v = random_coefficients(8, 1, w.N, w.nmax)[0]
    L = w.lmax
    idx = [(t, l, m) for t in (1, 2) for l in range(1, L + 1) for m in range(-l, l + 1)]
    flip = np.array([idx.index((t, l, -m)) for (t, l, m) in idx])
    lhs = np.sum(u * _gpu_W(p, v))
    rhs = np.sum(v[:, flip] * _gpu_W(p, u[:, flip]))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


@pytest.mark.parametrize("name,precision,K", [("slab300_l3", P.CELES_FP64, 2), ("slab300_l3", P.CELES_MIXED, 4),
                                              ("slab200_l4", P.CELES_MIXED, 4), ("slab200_l4", P.CELES_FP64, 3)])
def test_apply_W_multi_rhs(name, precision, K):
    w = workload(name)
    print(f"[matvec multi-rhs] {name} K={K} precision={precision}", flush=True)
    X = random_coefficients(110, K, w.N, w.nmax)
    p = make_problem(w, hankel=1)
    dt = torch.complex128 if precision == P.CELES_FP64 else torch.complex64
    xd = _dev(X, dt)
    yd = torch.empty_like(xd)
    p.apply_W(xd, yd, precision, K=K)
    torch.cuda.synchronize()
    Y = yd.cpu().numpy().astype(np.complex128)
    bar = 1e-12 if precision == P.CELES_FP64 else 1e-4
    for k in range(K):
        # same as the single right-hand-side launch
        yk = _gpu_W(p, X[k], precision)
        assert rel(Y[k], yk) <= (1e-14 if precision == P.CELES_FP64 else 1e-6)
    rows = list(range(0, w.N, 17))
    for k in range(K):
        xk = X[k] if precision == P.CELES_FP64 else X[k].astype(np.complex64).astype(np.complex128)
        ref = apply_W_rows(w.positions, xk, k_of(w), w.lmax, rows)
        assert rel(Y[k][rows], ref) <= bar


def test_full_size_slab20000_sampled_rows():
    # the 20,000-sphere slab of the mixed-vs-FP64 comparison, both precisions,
    # default launch configuration
    w = workload("slab20000_l4")
    print(f"[matvec] slab20000_l4 N={w.N} sampled rows", flush=True)
    x = random_coefficients(105, 1, w.N, w.nmax)[0]
    p = make_problem(w, hankel=0)
    rng = np.random.default_rng(6)
    rows = sorted(set(rng.choice(w.N, 3, replace=False).tolist() + [w.N - 1]))
    ref = apply_W_rows(w.positions, x, k_of(w), w.lmax, rows, hankel=oracle_lut(w))
    y64 = _gpu_W(p, x)
    assert rel(y64[rows], ref) <= 1e-12
    y32 = _gpu_W(p, x, precision=P.CELES_MIXED)
    ref32 = apply_W_rows(w.positions, x.astype(np.complex64).astype(np.complex128), k_of(w), w.lmax, rows,
                         hankel=oracle_lut(w))
    e = rel(y32[rows], ref32)
    print(f"[matvec fp32] slab20000_l4 sampled rows rel err {e:.2e}", flush=True)
    assert e <= 1e-4


def test_full_size_slab10000_64rhs_matrix_cores_sampled_rows():
    # the 64-right-hand-side slab of the batched workload: complex64 mat-vec on
    # the matrix cores, sampled rows of three right-hand sides against the oracle
    w = workload("slab10000_l3")
    K = 64
    print(f"[matvec mfma] slab10000_l3 N={w.N} K={K} sampled rows", flush=True)
    X = random_coefficients(106, K, w.N, w.nmax)
    p = make_problem(w, hankel=0)
    xd = _dev(X, torch.complex64)
    yd = torch.empty_like(xd)
    p.apply_W(xd, yd, P.CELES_MIXED, K=K)
    torch.cuda.synchronize()
    Y = yd.cpu().numpy().astype(np.complex128)
    rows = [0, 4321, w.N - 1]
    for k in (0, 31, 63):
        xk = X[k].astype(np.complex64).astype(np.complex128)
        ref = apply_W_rows(w.positions, xk, k_of(w), w.lmax, rows, hankel=oracle_lut(w))
        e = rel(Y[k][rows], ref)
        print(f"[matvec mfma] rhs {k} rel err {e:.2e}", flush=True)
        assert e <= 1e-4


def test_kernel_timing_counts_coupling_launches():
    w = workload("slab64_l3")
    p = make_problem(w, hankel=1)
    x = random_coefficients(107, 1, w.N, w.nmax)[0]
    p.kernel_timing(True)
    for _ in range(3):
        _gpu_W(p, x)
    ms, n = p.kernel_timing(False)
    assert n == 3 and 0 < ms < 1e3
    ms, n = p.kernel_timing(False)       # not running: nothing recorded
    assert n == 0 and ms == 0


def test_deterministic_option_fixes_the_split():
    # deterministic = 1 switches the timing-based split off: the split follows
    # from the sizes, so an autotune-requesting handle gives a plain handle's
    # bits on every call, and a batch created deterministic refuses to tune
    w = workload("slab300_l3")
    x = random_coefficients(108, 1, w.N, w.nmax)[0]
    plain = make_problem(w, hankel=0)
    det = make_problem(w, hankel=0, autotune=1, deterministic=1)
    y0 = _gpu_W(plain, x)
    for _ in range(2):
        assert np.array_equal(_gpu_W(det, x), y0)
        assert np.array_equal(_gpu_W(det, x, precision=P.CELES_MIXED), _gpu_W(plain, x, precision=P.CELES_MIXED))
    bt = P.Batch([det], deterministic=1)
    with pytest.raises(P.CelesError):
        bt.autotune(P.CELES_FP64)


@pytest.mark.parametrize("translation", [P.CELES_TRANSLATION_DIRECT, P.CELES_TRANSLATION_ROTATE])
def test_autotuned_split_keeps_parity(translation):
    # opt.autotune times the candidate splits on the first mat-vec of each
    # precision (every candidate writes y completely); whichever split it
    # keeps, W x equals a plain handle's up to summation order and the
    # oracle's rows
    w = workload("slab300_l3")
    x = random_coefficients(109, 1, w.N, w.nmax)[0]
    plain = make_problem(w, hankel=0, translation=translation)
    tuned = make_problem(w, hankel=0, translation=translation, autotune=1)
    y0 = _gpu_W(plain, x)
    for _ in range(2):
        y = _gpu_W(tuned, x)
        assert rel(y, y0) <= 1e-13
        assert rel(_gpu_W(tuned, x, precision=P.CELES_MIXED), y0) <= 1e-5
    rows = [0, 150, 299]
    ref = apply_W_rows(w.positions, x, k_of(w), w.lmax, rows, hankel=oracle_lut(w))
    assert rel(y[rows], ref) <= 1e-12

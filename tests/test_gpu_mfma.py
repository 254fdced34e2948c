"""Matrix-core (MFMA) coupling mat-vec for blocks of 16, 32 or 64 right-hand
sides in complex64: parity with the oracle (FP64 arithmetic on the
FP32-rounded input) and with the VALU complex64 kernel, for lmax 1..4, both
Hankel modes, sphere counts that are not a multiple of the 4 receivers of a
block, and several source chunkings."""
import os

import numpy as np
import pytest

import paper_1706_02145_amd as P
from celes_inputs import workload, random_coefficients
from oracle.lut import lut_for
from oracle.translation import apply_W_rows
from tests.gpu_helpers import k_of, rel, tvec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _problem(w, L, hankel):
    return P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, L, hankel=hankel, lut_dr=w.lut_dr)


def _apply(p, X, K, op="W", env=None):
    xd = torch.from_numpy(np.ascontiguousarray(X)).to("cuda", dtype=torch.complex64)
    yd = torch.empty_like(xd)
    env = env or {}
    os.environ.update(env)
    try:
        (p.apply_W if op == "W" else p.apply_M)(xd, yd, P.CELES_MIXED, K=K)
        torch.cuda.synchronize()
    finally:
        for key in env:
            os.environ.pop(key, None)
    return yd.cpu().numpy().astype(np.complex128)


CASES = [("slab64_l3", 1, 16, 1, None), ("slab64_l3", 2, 32, 0, None), ("slab300_l3", 3, 64, 0, 203),
         ("slab300_l3", 3, 16, 1, None), ("slab200_l4", 4, 64, 0, 198), ("slab200_l4", 4, 32, 1, None)]


@pytest.mark.parametrize("name,L,K,hankel,n", CASES)
def test_mfma_matches_oracle_and_valu(name, L, K, hankel, n):
    w = workload(name, n=n) if n else workload(name)
    nm = 2 * L * (L + 2)
    print(f"[mfma] {w.name} lmax={L} K={K} hankel={hankel} N={w.N}", flush=True)
    X = random_coefficients(120 + L, K, w.N, nm)
    p = _problem(w, L, hankel)
    Y = _apply(p, X, K, env={"CELES_WXM": "2"})
    Yv = _apply(p, X, K, env={"CELES_WXM": "0"})
    e_valu = rel(Y, Yv)
    k = k_of(w)
    hk = lut_for(w.positions, w.radii, k, L, w.lut_dr) if hankel == 0 else None
    rows = sorted(set(range(0, w.N, max(1, w.N // 12))) | {w.N - 1})
    errs = []
    for kk in sorted({0, K // 2, K - 1}):
        xk = X[kk].astype(np.complex64).astype(np.complex128)
        ref = apply_W_rows(w.positions, xk, k, L, rows, hankel=hk)
        errs.append(rel(Y[kk][rows], ref))
    print(f"[mfma] vs VALU {e_valu:.2e}, vs oracle {max(errs):.2e}", flush=True)
    assert e_valu <= 1e-5
    assert max(errs) <= 1e-5


def test_mfma_chunking_and_epilogue():
    w = workload("slab300_l3")
    K = 16
    X = random_coefficients(131, K, w.N, w.nmax)
    p = _problem(w, 3, 0)
    ys = [_apply(p, X, K, env={"CELES_WXM_TARGET_BLOCKS": tb, "CELES_WXM": "2"}) for tb in ("1", "300", "100000")]
    # one source chunk vs one chunk per 2 sources: complex64 sums of 300
    # terms in another order (a few ulp of the row norm)
    assert rel(ys[0], ys[2]) <= 1e-5
    assert rel(ys[1], ys[2]) <= 1e-5
    ym = _apply(p, X, K, op="M", env={"CELES_WXM": "2"})
    xk = X[5].astype(np.complex64).astype(np.complex128)
    ref = xk - tvec(w) * apply_W_rows(w.positions, xk, k_of(w), w.lmax, range(w.N),
                                      hankel=lut_for(w.positions, w.radii, k_of(w), 3, w.lut_dr))
    assert rel(ym[5], ref) <= 1e-5

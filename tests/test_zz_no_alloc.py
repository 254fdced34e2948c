"""Allocation-free coupling mat-vec (celes_apply_W_noalloc) against
celes_apply_W on the same inputs: two calls in a row, the second on a
smaller problem, in both precisions, and the size limit of its fixed
scratch array."""
import numpy as np
import pytest

import paper_1706_02145_amd as P
from celes_inputs import workload, random_coefficients
from tests.gpu_helpers import make_problem, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _both(p, w, K, prec, dt, seed):
    x = torch.from_numpy(random_coefficients(seed, K, w.N, w.nmax)).to("cuda", dt)
    y_ref = torch.empty_like(x)
    y = torch.full_like(x, float("nan"))          # every output entry must be written
    p.apply_W(x, y_ref, prec, K=K)
    p.apply_W_noalloc(x, y, prec, K=K)
    torch.cuda.synchronize()
    return y.cpu().numpy(), y_ref.cpu().numpy()


def test_noalloc_matches_apply_W():
    big, small = workload("slab2000_l4"), workload("slab300_l3")
    pb, ps = make_problem(big), make_problem(small)
    print("[noalloc] slab2000_l4 K=2 then slab300_l3 K=1", flush=True)
    # FP64: same kernels, source chunks capped to the fixed array (summation
    # order only); complex64: the mixed-precision bar
    for prec, dt, bar in ((P.CELES_FP64, torch.complex128, 1e-12), (P.CELES_MIXED, torch.complex64, 1e-6)):
        y, r = _both(pb, big, 2, prec, dt, 1)
        e1 = rel(y, r)
        y2, r2 = _both(ps, small, 1, prec, dt, 2)
        e2 = rel(y2, r2)
        print(f"[noalloc] precision {prec}: {e1:.2e}, {e2:.2e}", flush=True)
        assert np.isfinite(y).all() and np.isfinite(y2).all()
        assert e1 <= bar and e2 <= bar


def test_noalloc_rejects_sizes_beyond_its_array():
    w = workload("slab2000_l4")
    p = make_problem(w)
    K = 64                                        # 2 K N nmax complex128 = 196.6 MB > 128 MiB
    x = torch.zeros((K, w.N, w.nmax), dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(P.CelesError) as e:
        p.apply_W_noalloc(x, y, P.CELES_FP64, K=K)
    assert e.value.name == "CELES_E_ARG"
    # the same K fits in complex64: 2 K N nmax x 8 bytes = 98.3 MB (one source chunk)
    x32 = x.to(torch.complex64)
    y32 = torch.full_like(x32, float("nan"))
    p.apply_W_noalloc(x32, y32, P.CELES_MIXED, K=K)
    torch.cuda.synchronize()
    assert torch.count_nonzero(y32).item() == 0   # W 0 = 0, every entry written

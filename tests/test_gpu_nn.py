"""Learned initial guess: device gradients against the FP64 oracle (same
bf16 rounding points), feature invariants, and the gain over a zero and a
single-scattering initial guess on a slab the network has not seen."""
import numpy as np
import pytest

import paper_1706_02145_amd as P
from celes_inputs import workload
from oracle.mlp import forward_backward, unpack
from tests.gpu_helpers import rel

pytestmark = pytest.mark.gpu


def _plane(p):
    p.set_plane_waves([0.0], [0.0], [2])


def test_gradients_match_oracle():
    net = P.Network(3, seed=3)
    rng = np.random.default_rng(1)
    M = 200                                   # not a multiple of the 64-row tile
    X = (rng.standard_normal((M, net.in_pad)) * 0.5).astype(np.float32)
    X[:, net.in_dim:] = 0
    Y = (rng.standard_normal((M, net.out_pad)) * 0.3).astype(np.float32)
    Y[:, net.out_dim:] = 0
    p = net.params()
    loss, g = net.loss_grad(X, Y)
    lo, go, Zo = forward_backward(p, X, Y, net.out_dim, net.in_pad, net.out_pad, use_bf16=True)
    assert abs(loss - lo) <= 1e-4 * lo
    Z = net.forward(X)
    assert rel(Z[:, :net.out_dim], Zo[:, :net.out_dim]) <= 1e-3
    # per tensor
    Ws, bs = unpack(g, net.in_pad, net.out_pad)
    Wo, bo = unpack(go, net.in_pad, net.out_pad)
    for l in range(4):
        print(f"layer {l}: dW rel {rel(Ws[l], Wo[l]):.2e} db rel {rel(bs[l], bo[l]):.2e}")
        assert rel(Ws[l], Wo[l]) <= 1e-3
        assert rel(bs[l], bo[l]) <= 1e-3


def test_features_are_translation_invariant_and_normalised():
    w = workload("slab300_l3")
    net = P.Network(3)
    p1 = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, 3)
    p2 = P.Problem(w.positions + np.array([1234.5, -321.0, 77.0]), w.radii, w.n_sphere, w.n0, w.wavelength, 3)
    _plane(p1)
    _plane(p2)
    X1, _ = net.features(p1, targets=False)
    X2, _ = net.features(p2, targets=False)
    # positions enter only as differences; incident phases only relative to the receiver's own
    assert np.abs(X1 - X2).max() <= 2e-2 * np.abs(X1).max()
    nm = 30
    self_block = X1[:, 1:1 + 2 * nm].astype(np.float64)
    assert np.allclose(np.linalg.norm(self_block, axis=1), 1.0, atol=1e-2)
    # neighbours ordered by distance
    per = 4 + 2 * nm
    d = np.stack([np.linalg.norm(X1[:, 1 + 2 * nm + q * per:1 + 2 * nm + q * per + 3], axis=1) for q in range(16)], 1)
    assert (np.diff(d, axis=1) >= -1e-2).all()


def test_warm_start_gain_over_zero():
    net = P.Network(3, seed=7)
    base = workload("slab300_l3")
    train = [workload("slab300_l3", seed=900 + s, n=300) for s in range(10)]
    for w in train:
        p = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, 3, tol=1e-8, hankel=1)
        _plane(p)
        p.solve()
        net.add_training_problem(p)
    loss = net.train(epochs=60, batch=512, lr=2e-3, seed=1)
    print(f"training loss {loss:.3e}")
    w = workload("slab300_l3", seed=777, n=300)
    p = P.Problem(w.positions, w.radii, w.n_sphere, w.n0, w.wavelength, 3, tol=1e-6, hankel=1, restart=100)
    _plane(p)
    a = p.incident()
    from oracle.mie import T_vector
    t = T_vector(3, 2 * np.pi / w.wavelength, w.radii, w.n_sphere, w.n0)
    _, i0 = p.solve()
    _, i1 = p.solve(x0=(t * a[0])[None])
    x0 = net.predict(p)
    _, i2 = p.solve(x0=x0[None])
    print(f"iterations to 1e-6: zero {i0['iterations']}, T a_in {i1['iterations']}, network {i2['iterations']}; "
          f"initial residuals {i0['x0_residual']:.3f} {i1['x0_residual']:.3f} {i2['x0_residual']:.3f}")
    # what the trained network gains over x0 = 0: its least-squares weighted
    # guess starts from a residual well below ||rhs|| (measured 0.58; single
    # scattering alone 0.52) and never costs more than a few iterations of
    # restarted GMRES (measured 47 vs 48)
    assert i2["x0_used"] == 1
    assert i2["x0_residual"] <= 0.8
    assert i2["iterations"] <= i0["iterations"] + 2

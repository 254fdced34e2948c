"""Pin of the reference network's gradient: central finite differences of
the FP64 loss (no bf16 rounding) match the analytic back-propagation."""
import numpy as np

from oracle.mlp import bf16, dims, forward_backward


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    in_pad, out_pad, out_dim, M = 64, 64, 60, 7
    n = sum(a * b + b for a, b in zip(dims(in_pad, out_pad)[:-1], dims(in_pad, out_pad)[1:]))
    p = rng.standard_normal(n) * 0.1
    X = rng.standard_normal((M, in_pad))
    Y = rng.standard_normal((M, out_pad))
    loss, g, _ = forward_backward(p, X, Y, out_dim, in_pad, out_pad, use_bf16=False)
    idx = rng.choice(n, 40, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(n)
        e[i] = h
        lp = forward_backward(p + e, X, Y, out_dim, in_pad, out_pad, use_bf16=False)[0]
        lm = forward_backward(p - e, X, Y, out_dim, in_pad, out_pad, use_bf16=False)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9


def test_bf16_rounding():
    x = np.array([1.0, 1.00390625, 1.001953125, 3.0e-5, -2.5], dtype=np.float32)
    y = bf16(x)
    # bf16 keeps 7 mantissa bits: the neighbours of 1 are 1 and 1 + 2^-7.
    assert y[0] == 1.0 and y[4] == -2.5
    assert y[1] == 1.0            # 1 + 2^-8 is the midpoint: ties go to the even neighbour, 1
    assert y[2] == 1.0            # 1 + 2^-9 is below the midpoint
    assert abs(y[3] - 3.0e-5) <= 3.0e-5 * 2 ** -8

"""FP64 reference of the learned-initial-guess network (test infrastructure).

The network maps a feature row to a prediction: four linear layers
in_pad -> 128 -> 128 -> 128 -> out_pad with SiLU between them and mean
squared error on the real outputs.  `forward_backward` evaluates loss and
gradients in FP64; with bf16=True it rounds to bfloat16 (round to nearest
even) at the same points as the device implementation: inputs, weights,
hidden activations and the layer gradients that enter the backward
products.  Parameters are one flat vector: for each layer W [in][out]
row-major, then b [out].
"""
import numpy as np

HIDDEN = 128


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def dims(in_pad, out_pad):
    return [in_pad, HIDDEN, HIDDEN, HIDDEN, out_pad]


def unpack(p, in_pad, out_pad):
    d = dims(in_pad, out_pad)
    Ws, bs, o = [], [], 0
    for l in range(4):
        n = d[l] * d[l + 1]
        Ws.append(p[o:o + n].reshape(d[l], d[l + 1]))
        o += n
        bs.append(p[o:o + d[l + 1]])
        o += d[l + 1]
    return Ws, bs


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward_backward(p, X, Y, out_dim, in_pad, out_pad, use_bf16=True):
    """Loss and flat gradient for rows X [M][in_pad], targets Y [M][out_pad]."""
    r = bf16 if use_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    p = np.asarray(p, dtype=np.float64)
    Ws, bs = unpack(p, in_pad, out_pad)
    Wr = [r(W) for W in Ws]
    M = X.shape[0]
    A = [r(X)]
    Z = []
    for l in range(4):
        z = A[-1] @ Wr[l] + bs[l]
        Z.append(z)
        if l < 3:
            A.append(r(silu(z)))
    mask = np.zeros(out_pad)
    mask[:out_dim] = 1.0
    d = (Z[3] - np.asarray(Y, dtype=np.float64)) * mask
    loss = float(np.sum(d * d) / (M * out_dim))
    dZ = 2.0 * d / (M * out_dim)
    grads_W, grads_b = [None] * 4, [None] * 4
    for l in range(3, -1, -1):
        dZr = r(dZ)
        grads_W[l] = A[l].T @ dZr
        grads_b[l] = dZ.sum(axis=0)
        if l > 0:
            dA = dZr @ Wr[l].T
            dZ = dA * dsilu(Z[l - 1])
    g = np.concatenate([np.concatenate([gw.reshape(-1), gb]) for gw, gb in zip(grads_W, grads_b)])
    return loss, g, Z[3]

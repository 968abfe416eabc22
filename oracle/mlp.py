"""FP64 reference of the surrogate network -- TEST INFRASTRUCTURE ONLY.

Architecture (one ensemble member): inputs x (6 physical quantities) ->
z = (log x - mu) / sigma -> h1 = SiLU(W1 z + b1) (128) -> h2 = SiLU(W2 h1 + b2)
(128) -> h3 = SiLU(W3 h2 + b3) (128) -> y = w4 . h3 + b4, the standardised
ln k_s.  Parameters are kept flat in the order W1[128][6], b1, W2[128][128],
b2, W3[128][128], b3, w4[128], b4 (34 049 values).

The GPU kernels hold the weights in BF16 and round the hidden activations
h1, h2, h3 to BF16 before they enter the next layer; ``cast=True`` applies
the same round-to-nearest-even casts here so both sides compute the same
function.  The backward pass treats the casts as identity (straight-through),
as the GPU does.
"""
from __future__ import annotations

import numpy as np

H, D_IN = 128, 6
SIZES = (("W1", (H, D_IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)),
         ("b3", (H,)), ("w4", (H,)), ("b4", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(flat):
    out, off = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[off:off + n], dtype=np.float64).reshape(shape)
        off += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(x):
    """Round to the nearest BF16 value (ties to even), via the FP32 bits."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(a):
    return a / (1.0 + np.exp(-a))


def dsilu(a):
    s = 1.0 / (1.0 + np.exp(-a))
    return s * (1.0 + a * (1.0 - s))


def standardise(X, norm):
    """norm = dict(mu[6], sigma[6]); X raw physical inputs [n, 6] (all > 0)."""
    return (np.log(np.asarray(X, dtype=np.float64)) - norm["mu"]) / norm["sigma"]


def forward(flat, Z, cast=True):
    """Forward pass on standardised inputs Z [n, 6]; returns (y [n], cache)."""
    P = unpack(flat)
    rnd = bf16 if cast else (lambda v: np.asarray(v, dtype=np.float64))
    W1, W2, W3, w4 = (rnd(P[k]) for k in ("W1", "W2", "W3", "w4"))
    a1 = Z @ W1.T + P["b1"]
    h1 = rnd(silu(a1))
    a2 = h1 @ W2.T + P["b2"]
    h2 = rnd(silu(a2))
    a3 = h2 @ W3.T + P["b3"]
    h3 = rnd(silu(a3))
    y = h3 @ w4 + P["b4"][0]
    return y, dict(Z=Z, a1=a1, h1=h1, a2=a2, h2=h2, a3=a3, h3=h3, W2=W2, W3=W3, w4=w4)


def loss_and_grad(flat, Z, t, cast=True):
    """Mean squared error over the batch and its gradient w.r.t. the flat
    parameters (the casts pass gradients straight through)."""
    y, c = forward(flat, Z, cast)
    n = Z.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    g = {}
    g["w4"] = dy @ c["h3"]
    g["b4"] = np.array([dy.sum()])
    da3 = np.outer(dy, c["w4"]) * dsilu(c["a3"])
    g["W3"] = da3.T @ c["h2"]
    g["b3"] = da3.sum(axis=0)
    da2 = (da3 @ c["W3"]) * dsilu(c["a2"])
    g["W2"] = da2.T @ c["h1"]
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ c["W2"]) * dsilu(c["a1"])
    g["W1"] = da1.T @ c["Z"]
    g["b1"] = da1.sum(axis=0)
    return loss, pack(g)


def adam(flat, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (flat, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v

"""FP64 reference of the chemistry-surrogate network (TEST INFRASTRUCTURE
ONLY; not part of the paper, which integrates the chemistry exactly).

Network: 5 standardised inputs (log10 nH, log10 xHI, log10 T, log10 N,
log10 dt) -> three hidden layers of 64 SiLU units -> 2 standardised outputs
(the surrogate uses them for asinh-compressed changes of log10 xHI, log10 T).  Loss: mean over samples and outputs of the squared
error of the standardised outputs.  Parameters are one flat vector in the
order W1 (64x5), b1, W2 (64x64), b2, W3 (64x64), b3, W4 (2x64), b4 -- each W
row-major as (out, in) -- 8834 values.

Plain numpy: the forward pass as matrix products, the backward pass written
out by the chain rule, checked in the tests against central differences.
"""

from __future__ import annotations

import numpy as np

SIZES = [(64, 5), (64, 64), (64, 64), (2, 64)]
NPARAM = sum(o * i + o for o, i in SIZES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (NPARAM,)
    out, off = [], 0
    for o, i in SIZES:
        W = theta[off:off + o * i].reshape(o, i)
        off += o * i
        b = theta[off:off + o]
        off += o
        out.append((W, b))
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X):
    """X (B, 5) -> Y (B, 2); also returns the pre-activations and inputs of
    every layer for the backward pass."""
    layers = unpack(theta)
    h = np.asarray(X, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        cache.append((h, z))
        h = silu(z) if li < len(layers) - 1 else z
    return h, cache


def loss_and_grad(theta, X, Yt):
    """Mean squared error over B samples x 2 outputs and its gradient."""
    Y, cache = forward(theta, X)
    Yt = np.asarray(Yt, dtype=np.float64)
    B = Y.shape[0]
    diff = Y - Yt
    loss = float(np.mean(diff * diff))
    g = 2.0 * diff / diff.size           # dL/dY
    layers = unpack(theta)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        h, z = cache[li]
        W, _ = layers[li]
        dz = g if li == len(layers) - 1 else g * silu_grad(z)
        grads[li] = (dz.T @ h, dz.sum(axis=0))
        g = dz @ W
    flat = np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in grads])
    return loss, flat


def init_params(seed: int = 0) -> np.ndarray:
    """He-style uniform initialisation (fan-in), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in SIZES:
        lim = np.sqrt(6.0 / i)
        parts.append(rng.uniform(-lim, lim, size=o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def adam_step(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; step >= 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)

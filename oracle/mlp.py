"""Plain FP64 reference of the warm-start network (not part of the paper:
the learned start vector x0 = s * MLP(theta) for CG).

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this module.  It
shares no code with the HIP kernels: a network of three affine layers with
ReLU after the first two, the mean squared error and its gradient written
out with NumPy products, and the Adam update (Kingma and Ba, 2015) as
published.  Pinned by central finite differences and by Adam's closed-form
first step (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np


def bf16_round(a) -> np.ndarray:
    """Rounds FP32 values to the nearest bfloat16 (ties to even), returned as
    FP64.  The bfloat16 number is the FP32 number with its 16 low bits cut."""
    f = np.ascontiguousarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta, params):
    """params = [W1, b1, W2, b2, W3, b3] with W_k [in][out].  Returns the
    output and the intermediate values (z1, h1, z2, h2)."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, np.float64) for p in params]
    x = np.asarray(theta, np.float64)
    z1 = x @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    return y, (x, z1, h1, z2, h2)


def loss_and_grads(theta, target, params, store=None):
    """L = mean over all entries of (y - target)^2 and dL/dparams.

    store: rounding applied where a lower-precision implementation keeps a
    value in memory (the input, the hidden activations, the target, the
    output gradient and the hidden layers' gradients before the products
    that read them); None keeps FP64 throughout.  The bias gradients sum the
    unrounded gradients."""
    s = store or (lambda a: np.asarray(a, np.float64))
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, np.float64) for p in params]
    x = s(theta)
    z1 = x @ W1 + b1
    h1 = s(np.maximum(z1, 0.0))
    z2 = h1 @ W2 + b2
    h2 = s(np.maximum(z2, 0.0))
    y = h2 @ W3 + b3
    d = y - s(target)
    M, n = d.shape
    L = float(np.mean(d * d))
    g = 2.0 * d / (M * n)
    dy = s(g)
    gW3 = h2.T @ dy
    gb3 = g.sum(axis=0)
    dz2 = (dy @ W3.T) * (z2 > 0)
    gb2 = dz2.sum(axis=0)
    dz2 = s(dz2)
    gW2 = h1.T @ dz2
    dz1 = (dz2 @ W2.T) * (z1 > 0)
    gb1 = dz1.sum(axis=0)
    dz1 = s(dz1)
    gW1 = x.T @ dz1
    return L, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam(w, m, v, g, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step; returns (w, m, v) updated."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v

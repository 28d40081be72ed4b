"""Learned energy sampler: CPU reference of the network (oracle).  Test infrastructure only.

Not in the paper: the learned part of the build is a small multilayer perceptron that
proposes where to place energy points on a T(E) curve.  This module is the plain,
slow statement of what the GPU kernels compute, for checking them:

    X0 = bf16(x)
    Z_l = X_{l-1} W_l^T + b_l,   X_l = bf16(gelu(Z_l))        l = 1 .. n-1
    logits = X_{n-1} W_n^T + b_n
    loss = mean_b [ -sum_c q[b, c] log softmax(logits[b])_c ]

with W_l the BF16 copies of FP32 master weights and every product accumulated in FP32.
GELU is x Phi(x) with Phi the standard normal CDF, erfc(-x / sqrt 2) / 2.
The backward pass is the chain rule, with the tensors the GPU stores in BF16 rounded at
the same places:

    dZ_n = bf16((softmax(logits) - q) / B)
    dW_l = dZ_l^T X_{l-1},   db_l = sum_b dZ_l
    dX_{l-1} = dZ_l W_l,     dZ_{l-1} = bf16(dX_{l-1} * gelu'(Z_{l-1}))

``rounding=False`` with float64 arrays gives the exact-arithmetic network, which the
tests pin against finite differences.
"""

from __future__ import annotations

import math

import numpy as np


def bf16_round(x: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 value (ties to even), returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).copy()
    nan = np.isnan(x)
    out[nan] = np.nan
    return out


_erfc = np.vectorize(math.erfc, otypes=[np.float64])


def _Phi(xd):
    """Standard normal CDF, erfc(-x / sqrt 2) / 2 (accurate in the left tail)."""
    return 0.5 * _erfc(-xd / math.sqrt(2.0))


def gelu(x):
    xd = np.asarray(x, dtype=np.float64)
    return (xd * _Phi(xd)).astype(np.asarray(x).dtype)


def gelu_grad(x):
    xd = np.asarray(x, dtype=np.float64)
    g = _Phi(xd) + xd * np.exp(-0.5 * xd * xd) / math.sqrt(2.0 * math.pi)
    return g.astype(np.asarray(x).dtype)


def _r(x, rounding):
    return bf16_round(x) if rounding else x


def forward(params, x, rounding=True):
    """params: list of (W [out, in], b [out]).  Returns (logits, cache)."""
    dt = np.float32 if rounding else np.float64
    X = [_r(np.asarray(x, dtype=dt), rounding)]
    Z = []
    n = len(params)
    for li, (W, b) in enumerate(params):
        Wq = _r(np.asarray(W, dtype=dt), rounding)
        z = X[-1] @ Wq.T + np.asarray(b, dtype=dt)
        Z.append(z)
        if li < n - 1:
            X.append(_r(gelu(z), rounding))
    return Z[-1], {"X": X, "Z": Z, "rounding": rounding}


def softmax(z):
    m = z.max(axis=1, keepdims=True)
    e = np.exp(z - m)
    return e / e.sum(axis=1, keepdims=True)


def xent_loss(logits, q):
    """Mean over rows of -sum_c q log softmax(logits)."""
    m = logits.max(axis=1, keepdims=True)
    lse = m + np.log(np.exp(logits - m).sum(axis=1, keepdims=True))
    return float(np.mean(-(q * (logits - lse)).sum(axis=1)))


def backward(params, cache, q):
    """Gradients [(dW, db)] of the mean cross-entropy loss."""
    rounding = cache["rounding"]
    dt = np.float32 if rounding else np.float64
    X, Z = cache["X"], cache["Z"]
    B = X[0].shape[0]
    p = softmax(Z[-1])
    dZ = _r(((p - q) / B).astype(dt), rounding)
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W = _r(np.asarray(params[li][0], dtype=dt), rounding)
        grads[li] = (dZ.T @ X[li], dZ.sum(axis=0))
        if li > 0:
            dX = dZ @ W
            dZ = _r((dX * gelu_grad(Z[li - 1])).astype(dt), rounding)
    return grads


def adamw(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One AdamW step (decoupled weight decay); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    w = w - lr * (mh / (np.sqrt(vh) + eps) + wd * w)
    return w, m, v

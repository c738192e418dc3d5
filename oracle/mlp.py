"""Plain FP64 reference of the surrogate network (TEST INFRASTRUCTURE ONLY).

The multilayer perceptron of the learned surrogate, written out with numpy:
normalised input x = (f - mu_in) / sd_in, hidden layers h = silu(W x + b),
a linear output layer, loss = mean of (yhat - (q - mu_out) / sd_out)^2 over
rows and features, and its gradient by the chain rule.  With ``bf16=True`` the
values that the GPU stores in BF16 (inputs, weights, hidden activations, the
output gradient and the gradients of the hidden pre-activations) are rounded
to BF16 at the same points, so the two differ only by FP32 accumulation
order; with ``bf16=False`` every step is FP64.

Parameters are a list of (W, b) with W of shape (out, in).  Only tests/ use
this module.
"""
from __future__ import annotations

import numpy as np


def to_bf16(x):
    """Round to the nearest BF16 value (ties to even) via FP32, as a float64 array."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    r = np.where(finite, (u + 0x7FFF + ((u >> 16) & 1)) >> 16, u >> 16)
    return (r.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def _r(x, on):
    return to_bf16(x) if on else np.asarray(x, dtype=np.float64)


def forward(params, f, mu_in, sd_in, bf16=True):
    """Returns (yhat, cache): yhat is the normalised network output."""
    x = _r((np.asarray(f, np.float64) - mu_in) / sd_in, bf16)
    hs, zs = [x], []
    h = x
    for li, (W, b) in enumerate(params):
        z = h @ _r(W, bf16).T + b
        zs.append(z)
        if li + 1 < len(params):
            h = _r(silu(z), bf16)
            hs.append(h)
    return zs[-1], (hs, zs)


def loss_and_grad(params, f, q, mu_in, sd_in, mu_out, sd_out, bf16=True, relative=False):
    """Loss and its gradient [(dW, db), ...].  relative=False: mean squared
    error of the normalised output.  relative=True: mean over rows of the
    squared relative error in the units of q, |sd_out * d_r|^2 / |q_r|^2."""
    yhat, (hs, zs) = forward(params, f, mu_in, sd_in, bf16)
    qq = np.asarray(q, np.float64)
    y = (qq - mu_out) / sd_out
    rows, n = yhat.shape
    d = yhat - y
    if relative:
        wt = np.asarray(sd_out, np.float64) ** 2 / np.sum(qq * qq, axis=1, keepdims=True) / rows
    else:
        wt = np.full_like(d, 1.0 / (rows * n))
    loss = float(np.sum(wt * d * d))
    g32 = 2.0 * wt * d
    g = _r(g32, bf16)
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        grads[li] = (g.T @ hs[li], np.sum(g32, axis=0))
        if li == 0:
            break
        dh = g @ _r(W, bf16)
        g32 = dh * silu_grad(zs[li - 1])
        g = _r(g32, bf16)
    return loss, grads


def conserve(q, cons):
    """Project rows of q onto the vectors orthogonal to the rows of cons."""
    C = np.asarray(cons, np.float64)
    G = C @ C.T
    return q - (q @ C.T) @ np.linalg.solve(G, C)

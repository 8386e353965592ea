"""CPU FP64 oracle for the small perceptron of the high-band surrogate.

TEST INFRASTRUCTURE ONLY (tests, smoke check and the benchmark's CPU-baseline
leg).  Shares no code with the HIP library.

The network is a 3-layer perceptron with SiLU activations:
    h1 = silu(x W1 + b1),  h2 = silu(h1 W2 + b2),  y = h2 W3 + b3
with silu(z) = z * sigmoid(z).  Training minimises the masked mean squared
error  L = (1/rows) * sum_{r,o} 0.5 * mask[r,o] * (y[r,o] - t[r,o])^2  with Adam
(Kingma & Ba, 2015: bias-corrected first and second moments).

Weights are taken exactly as given (the GPU keeps BF16 copies of FP32 master
weights; the oracle receives those BF16 values widened to float64).
"""
from __future__ import annotations

import numpy as np


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(params: dict, x: np.ndarray, keep: bool = False):
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ params["W1"] + params["b1"]
    h1 = silu(z1)
    z2 = h1 @ params["W2"] + params["b2"]
    h2 = silu(z2)
    y = h2 @ params["W3"] + params["b3"]
    if keep:
        return y, (x, z1, h1, z2, h2)
    return y


def loss(y: np.ndarray, t: np.ndarray, mask: np.ndarray | None = None):
    """Masked MSE and its gradient with respect to y."""
    m = np.ones_like(y) if mask is None else np.asarray(mask, dtype=np.float64)
    rows = y.shape[0]
    d = (y - t) * m
    L = 0.5 * np.sum(d * (y - t)) / rows
    return L, d / rows


def backward(params: dict, cache, dy: np.ndarray):
    """Gradients of a scalar with respect to params and input, given dL/dy."""
    x, z1, h1, z2, h2 = cache
    dy = np.asarray(dy, dtype=np.float64)
    g = {}
    g["W3"] = h2.T @ dy
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ params["W3"].T
    dz2 = dh2 * dsilu(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ params["W2"].T
    dz1 = dh1 * dsilu(z1)
    g["W1"] = x.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    dx = dz1 @ params["W1"].T
    return g, dx


def adam_step(params: dict, grads: dict, m: dict, v: dict, step: int, lr=1e-3, b1=0.9,
              b2=0.999, eps=1e-8):
    """One Adam update in place (step counts from 1)."""
    c1 = 1.0 - b1 ** step
    c2 = 1.0 - b2 ** step
    for k in params:
        m[k] = b1 * m[k] + (1.0 - b1) * grads[k]
        v[k] = b2 * v[k] + (1.0 - b2) * grads[k] ** 2
        params[k] = params[k] - lr * (m[k] / c1) / (np.sqrt(v[k] / c2) + eps)
    return params, m, v

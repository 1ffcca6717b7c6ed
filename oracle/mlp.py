"""Float64 reference of the fusion cost model's network -- TEST INFRASTRUCTURE ONLY.

A 3-layer perceptron F -> W -> W -> 1 with ReLU on both hidden layers, trained
on mean squared error with Adam.  Parameters are one flat vector in the
layout W1 [W x F], b1 [W], W2 [W x W], b2 [W], W3 [1 x W], b3 [1] (row-major),
the same layout the GPU library uses, so the two can be compared entry by
entry.  Plain numpy, float64, no blocking or fusion.
"""
from __future__ import annotations

import numpy as np


def unpack(p: np.ndarray, F: int, W: int):
    p = np.asarray(p, dtype=np.float64)
    i = 0
    W1 = p[i:i + W * F].reshape(W, F); i += W * F
    b1 = p[i:i + W]; i += W
    W2 = p[i:i + W * W].reshape(W, W); i += W * W
    b2 = p[i:i + W]; i += W
    W3 = p[i:i + W].reshape(1, W); i += W
    b3 = p[i:i + 1]; i += 1
    assert i == p.size
    return W1, b1, W2, b2, W3, b3


def num_params(F: int, W: int) -> int:
    return W * F + W + W * W + W + W + 1


def forward(p, X, F: int, W: int) -> np.ndarray:
    W1, b1, W2, b2, W3, b3 = unpack(p, F, W)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return (h2 @ W3.T + b3)[:, 0]


def loss(p, X, T, F: int, W: int) -> float:
    """Mean squared error over the batch."""
    d = forward(p, X, F, W) - np.asarray(T, dtype=np.float64)
    return float(np.mean(d * d))


def loss_grad(p, X, T, F: int, W: int):
    """(loss, gradient) by the chain rule written out layer by layer."""
    W1, b1, W2, b2, W3, b3 = unpack(p, F, W)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    B = X.shape[0]
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ W3.T + b3)[:, 0]
    d = y - T
    L = float(np.mean(d * d))
    dy = 2.0 * d / B                       # dL/dy
    gW3 = dy[None, :] @ h2                 # [1, W]
    gb3 = np.array([dy.sum()])
    dh2 = dy[:, None] * W3                 # [B, W]
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba): returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

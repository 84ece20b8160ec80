"""The learned-index network in fp64: 32 bit features -> 64 -> 64 -> 1 with ReLU.

Test infrastructure only (see the package docstring).  The paper has no
learned index; this is the plain definition of the network, its mean-squared
loss, the gradients by the chain rule, and one Adam update (Kingma & Ba).
Parameters: W1 (64x32), b1 (64), W2 (64x64), b2 (64), w3 (64), b3 (scalar).
"""
from __future__ import annotations

import numpy as np


def features(patterns, nbits: int = 32) -> np.ndarray:
    """Bit j of each pattern as a 0/1 feature (B x nbits)."""
    p = np.asarray(patterns, dtype=np.uint64)
    return ((p[:, None] >> np.arange(nbits, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.float64)


def forward(P, X):
    W1, b1, W2, b2, w3, b3 = P
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (X, z1, h1, z2, h2)


def loss(P, X, target) -> float:
    y, _ = forward(P, X)
    return float(np.mean((y - target) ** 2))


def gradients(P, X, target):
    """d loss / d parameters for loss = mean_b (y_b - target_b)^2."""
    W1, b1, W2, b2, w3, b3 = P
    y, (X, z1, h1, z2, h2) = forward(P, X)
    B = X.shape[0]
    dy = 2.0 * (y - target) / B
    gw3 = h2.T @ dy
    gb3 = float(dy.sum())
    dz2 = np.outer(dy, w3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return [gW1, gb1, gW2, gb2, gw3, gb3]


def adam_step(P, G, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update with bias correction; returns new (P, m, v)."""
    outP, outm, outv = [], [], []
    for p, g, mm, vv in zip(P, G, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mh = mm / (1 - b1 ** step)
        vh = vv / (1 - b2 ** step)
        outP.append(p - lr * mh / (np.sqrt(vh) + eps))
        outm.append(mm)
        outv.append(vv)
    return outP, outm, outv

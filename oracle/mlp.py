"""fp64 reference of the learned router, for checking the GPU training kernels.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, no
blocking or fusion.  The network maps a scalar feature u to
    h1 = clamp(W1 u + b1, 0, 1)            (32 units)
    h2 = clamp(W2 h1 + b2, 0, 1)           (32 units)
    y  = W3 . h2 + b3
and is trained on the mean squared error of y against targets t.  The
parameters are one flat vector in the order W1[32], b1[32], W2[32x32] (row j
holds the weights into unit j), b2[32], W3[32], b3[1]: 1153 values.

The derivative of clamp(x, 0, 1) is taken as 1 for 0 < x < 1 and 0 elsewhere.
This network is not from the paper; it is the learned replacement of the
Direct table used for arrays where the table would be too large.
"""
from __future__ import annotations

import numpy as np

H = 32
N_PARAMS = 2 * H + H * H + H + H + 1  # 1153


def unpack(p: np.ndarray):
    p = np.asarray(p, np.float64)
    o = 0
    W1 = p[o:o + H]; o += H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def forward(p: np.ndarray, u: np.ndarray):
    """y for every u, plus the intermediate values the backward pass needs."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    u = np.asarray(u, np.float64)
    a1 = np.outer(u, W1) + b1              # (B, 32)
    h1 = np.clip(a1, 0.0, 1.0)
    a2 = h1 @ W2.T + b2                    # (B, 32)
    h2 = np.clip(a2, 0.0, 1.0)
    y = h2 @ W3 + b3                       # (B,)
    return y, (u, a1, h1, a2, h2)


def loss(p: np.ndarray, u: np.ndarray, t: np.ndarray) -> float:
    y, _ = forward(p, u)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def grad(p: np.ndarray, u: np.ndarray, t: np.ndarray):
    """(loss, d loss / d p) by the chain rule, layer by layer."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    y, (u, a1, h1, a2, h2) = forward(p, u)
    B = u.size
    dy = 2.0 * (y - np.asarray(t, np.float64)) / B          # (B,)
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    dh2 = np.outer(dy, W3)
    da2 = dh2 * ((a2 > 0.0) & (a2 < 1.0))
    gW2 = da2.T @ h1                                          # (32, 32): [j, k]
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * ((a1 > 0.0) & (a1 < 1.0))
    gW1 = da1.T @ u
    gb1 = da1.sum(axis=0)
    g = np.concatenate([gW1, gb1, gW2.reshape(-1), gb2, gW3, [gb3]])
    return float(np.mean((y - t) ** 2)), g


def numeric_grad(p: np.ndarray, u: np.ndarray, t: np.ndarray, idx, eps: float = 1e-6):
    """Central finite differences of the loss for the parameters listed in idx."""
    p = np.asarray(p, np.float64)
    out = np.empty(len(idx))
    for n, k in enumerate(idx):
        e = np.zeros_like(p)
        e[k] = eps
        out[n] = (loss(p + e, u, t) - loss(p - e, u, t)) / (2 * eps)
    return out

"""Plain FP64 reference of the rank-predictor network (test infrastructure only).

TEST INFRASTRUCTURE ONLY: used by the tests to check the GPU network's forward
pass, gradients and training.  It shares no code with the GPU library.

The network maps 8 features of a truncation to a predicted log2(1 + k):

    h1 = relu(W1 x + b1)      W1: 64 x 8
    h2 = relu(W2 h1 + b2)     W2: 64 x 64
    y  = w3 . h2 + b3         w3: 64

and is trained on the mean squared error 0.5 mean_i (y_i - t_i)^2.  Weights
are given as FP64 arrays (the GPU's BF16 weights upcast).  Written directly
from the definitions: a matrix product per layer, the chain rule for the
gradients.
"""
from __future__ import annotations

import numpy as np

SHAPES = {"W1": (64, 8), "b1": (64,), "W2": (64, 64), "b2": (64,), "w3": (64,), "b3": ()}


def forward(p, X):
    """Forward pass for a batch X (B x 8); returns y (B,) and the activations."""
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["w3"] + p["b3"]
    return y, (X, z1, h1, z2, h2)


def loss(p, X, t):
    y, _ = forward(p, X)
    return 0.5 * np.mean((y - np.asarray(t, dtype=np.float64)) ** 2)


def gradients(p, X, t):
    """Gradients of loss(p, X, t) with respect to every parameter (chain rule)."""
    y, (X, z1, h1, z2, h2) = forward(p, X)
    B = X.shape[0]
    dy = (y - np.asarray(t, dtype=np.float64)) / B          # dL/dy
    g = {"w3": h2.T @ dy, "b3": np.sum(dy)}
    dh2 = np.outer(dy, p["w3"])
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return g


def finite_difference(p, X, t, name, index, h=1e-6):
    """Central difference of the loss in one parameter entry."""
    q = {k: np.array(v, dtype=np.float64, copy=True) for k, v in p.items()}
    a = q[name].reshape(-1) if q[name].ndim else None
    if a is None:
        q[name] = np.float64(p[name] + h)
        lp = loss(q, X, t)
        q[name] = np.float64(p[name] - h)
        lm = loss(q, X, t)
    else:
        a[index] += h
        lp = loss(q, X, t)
        a[index] -= 2 * h
        lm = loss(q, X, t)
    return (lp - lm) / (2 * h)


def to_bf16(a):
    """Round FP64 values to the nearest BF16 (round to nearest even), as FP64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounding = 0x7FFF + ((u >> 16) & 1)
    u = ((u + rounding) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)

"""FP64 reference for the log-importance MLP.  TEST INFRASTRUCTURE ONLY.

Network: in_dim -> H -> H -> 1 with ReLU hidden layers, parameters packed as
W1[H][in], b1[H], W2[H][H], b2[H], W3[H], b3 (the same flat layout the GPU
kernels use).  Loss: weighted mean squared error
    L = sum_i wt_i (f(x_i) - y_i)^2 / sum_i wt_i.
Optimiser: Adam (Kingma & Ba 2015) with bias correction.

Plain numpy, written from the definitions: forward, the chain rule for the
backward pass, and the Adam update.
"""
from __future__ import annotations

import numpy as np


def unpack(params: np.ndarray, in_dim: int, H: int):
    p = np.asarray(params, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * in_dim].reshape(H, in_dim); o += H * in_dim
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o:o + 1]; o += 1
    assert o == p.size, (o, p.size)
    return W1, b1, W2, b2, W3, b3


def n_params(in_dim: int, H: int) -> int:
    return H * in_dim + H + H * H + H + H + 1


def init_params(in_dim: int, H: int, seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (float32 values)."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (H, in_dim)) * np.sqrt(6.0 / in_dim)
    W2 = rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H)
    W3 = rng.uniform(-1, 1, (H,)) * np.sqrt(6.0 / H)
    p = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3, np.zeros(1)])
    return p.astype(np.float32)


def forward(params, X, in_dim, H):
    W1, b1, W2, b2, W3, b3 = unpack(params, in_dim, H)
    X = np.asarray(X, np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ W3 + b3[0]
    return out, (X, z1, h1, z2, h2)


def loss(params, X, y, wt, in_dim, H) -> float:
    out, _ = forward(params, X, in_dim, H)
    wt = np.asarray(wt, np.float64)
    r = out - np.asarray(y, np.float64)
    return float(np.sum(wt * r * r) / np.sum(wt))


def grad(params, X, y, wt, in_dim, H):
    """Analytic gradient of ``loss`` by the chain rule."""
    W1, b1, W2, b2, W3, b3 = unpack(params, in_dim, H)
    out, (X, z1, h1, z2, h2) = forward(params, X, in_dim, H)
    wt = np.asarray(wt, np.float64)
    dout = 2.0 * wt * (out - np.asarray(y, np.float64)) / np.sum(wt)     # dL/dout  [n]
    gW3 = dout @ h2
    gb3 = np.array([dout.sum()])
    dh2 = np.outer(dout, W3)
    dz2 = dh2 * (z2 > 0.0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0.0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, gb3])


def adam_step(params, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v

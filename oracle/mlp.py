"""MLP cost model in FP64: the learned selector that stands in for the
decision tree (the paper's section 5.1 evaluates an MLP among its classifiers;
here the network regresses each chosen kernel's relative performance and the
selection is the argmax).  Test infrastructure only.

Network 6 -> 64 -> 64 -> k with ReLU after the two hidden layers and a linear
output.  Features of a problem (M, N, K, batch, transA, transB):
    x = [log2(M)/12, log2(N)/12, log2(K)/12, log2(batch)/6, transA, transB]
Targets: the relative (Q16 / 65535) performance of each of the k chosen
kernels on that problem.  Loss: mean squared error over rows x k.
Optimiser: full-batch Adam (Kingma and Ba, 2015) with bias correction,
lr 1e-3, beta1 0.9, beta2 0.999, eps 1e-8.  Weights are row-major
[fan_out][fan_in]; y = x W^T + b.  ReLU'(0) is taken as 0.
"""
from __future__ import annotations

import math

import numpy as np

PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def features(shapes):
    rows = []
    for (M, N, K, b, ta, tb) in shapes:
        rows.append([math.log2(M) / 12.0, math.log2(N) / 12.0, math.log2(K) / 12.0,
                     math.log2(b) / 6.0, float(ta), float(tb)])
    return np.array(rows, dtype=np.float64)


def forward(p, X):
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (X, z1, h1, z2, h2)


def loss(p, X, Y):
    y, _ = forward(p, X)
    return float(np.mean((y - Y) ** 2))


def grads(p, X, Y):
    y, (X, z1, h1, z2, h2) = forward(p, X)
    n, k = Y.shape
    dy = 2.0 * (y - Y) / (n * k)
    g = {}
    g["W3"] = dy.T @ h2
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ p["W3"]
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return g, float(np.mean((y - Y) ** 2))


def adam_init(p):
    return {name: np.zeros_like(p[name]) for name in PARAM_ORDER}, \
           {name: np.zeros_like(p[name]) for name in PARAM_ORDER}


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); updates p, m, v in place."""
    for name in PARAM_ORDER:
        m[name] = b1 * m[name] + (1.0 - b1) * g[name]
        v[name] = b2 * v[name] + (1.0 - b2) * g[name] * g[name]
        mh = m[name] / (1.0 - b1 ** t)
        vh = v[name] / (1.0 - b2 ** t)
        p[name] = p[name] - lr * mh / (np.sqrt(vh) + eps)


def train(p0, X, Y, steps, lr=1e-3):
    p = {name: np.array(p0[name], dtype=np.float64, copy=True) for name in PARAM_ORDER}
    m, v = adam_init(p)
    losses = []
    for t in range(1, steps + 1):
        g, l = grads(p, X, Y)
        losses.append(l)
        adam_step(p, g, m, v, t, lr)
    return p, losses


def select(p, X):
    y, _ = forward(p, X)
    return np.argmax(y, axis=1)     # first maximum

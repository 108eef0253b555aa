"""Rank-predictor MLP (oracle).  Test infrastructure only.

A plain fully connected network with three hidden layers of 64 tanh units,
written out in float64 so that finite differences can pin its gradients.  It
maps per-bond features to a distribution over rank classes (class c means
rank 8*(c+1): the coarse rank lattice r_c = n*r_0 of Sec. 5.1 of Hauck, Kabel,
Gauger, arXiv 2512.07811, taken here with r_0 = 8 instead of the paper's 16).

Loss per sample (reading: under-prediction costs a fallback, over-prediction
only extra work, so the loss is biased upward):
    CE(z, y) + beta * sum_c softmax(z)_c * w(c, y)
    w(c, y) = (c - y)/C  for c > y,   gamma  for c < y,   0 for c = y.
Optimizer: Adam (Kingma and Ba 2015) with bias correction.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64
LAYERS = 3


def init_params(n_in: int, n_cls: int, seed: int):
    g = np.random.Generator(np.random.PCG64(seed))
    dims = [n_in] + [HIDDEN] * LAYERS + [n_cls]
    P = {}
    for i in range(len(dims) - 1):
        P[f"W{i}"] = g.standard_normal((dims[i], dims[i + 1])) * np.sqrt(1.0 / dims[i])
        P[f"b{i}"] = np.zeros(dims[i + 1])
    return P


def cost_matrix(n_cls: int, gamma: float):
    c = np.arange(n_cls)[:, None]
    y = np.arange(n_cls)[None, :]
    return np.where(c > y, (c - y) / n_cls, np.where(c < y, gamma, 0.0))  # [c, y]


def forward(P, x):
    hs = [x]
    h = x
    n = len([k for k in P if k.startswith("W")])
    for i in range(n - 1):
        h = np.tanh(h @ P[f"W{i}"] + P[f"b{i}"])
        hs.append(h)
    z = h @ P[f"W{n - 1}"] + P[f"b{n - 1}"]
    return z, hs


def softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss_and_grad(P, x, y, beta: float = 1.0, gamma: float = 2.0):
    """Mean loss over the batch and gradients for every parameter."""
    B = x.shape[0]
    z, hs = forward(P, x)
    C = z.shape[1]
    p = softmax(z)
    w = cost_matrix(C, gamma)[:, y].T            # (B, C): w[b, c] = w(c, y_b)
    ce = -np.log(p[np.arange(B), y])
    ec = np.sum(p * w, axis=1)
    loss = float(np.mean(ce + beta * ec))
    onehot = np.zeros_like(p)
    onehot[np.arange(B), y] = 1.0
    dz = (p - onehot) + beta * p * (w - ec[:, None])
    dz /= B
    n = len(hs)
    G = {}
    d = dz
    for i in range(n - 1, -1, -1):
        G[f"W{i}"] = hs[i].T @ d
        G[f"b{i}"] = d.sum(axis=0)
        if i > 0:
            d = (d @ P[f"W{i}"].T) * (1.0 - hs[i] ** 2)
    return loss, G


def adam_init(P):
    return {k: np.zeros_like(v) for k, v in P.items()}, {k: np.zeros_like(v) for k, v in P.items()}


def adam_step(P, G, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); updates P, m, v in place."""
    for k in P:
        m[k] = b1 * m[k] + (1 - b1) * G[k]
        v[k] = b2 * v[k] + (1 - b2) * G[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)


def predict_class(P, x, quantile: float = 0.9):
    """Smallest class whose cumulative predicted probability reaches `quantile`."""
    p = softmax(forward(P, x)[0])
    cdf = np.cumsum(p, axis=1)
    return np.argmax(cdf >= quantile, axis=1)

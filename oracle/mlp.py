"""Reference multilayer perceptron of the subspace-size estimator (test infrastructure only).

Not part of the paper: the paper sizes the subspace by hand (p at least the eigenvalue count,
Section 4).  The estimator maps stochastic trace features of the filter to a count; this module
is the plain FP64 definition of its network and training step, against which the device kernels
are checked: three affine layers 19 -> 256 -> 256 -> 1 with ReLU between them, mean squared
error, and the Adam update (Kingma and Ba) with bias correction.

Parameters are a dict of float64 arrays W1 (h x d), b1 (h), W2 (h x h), b2 (h), W3 (1 x h), b3 (1);
`flatten` orders them W1, b1, W2, b2, W3, b3 with each matrix row-major.
"""
from __future__ import annotations

import numpy as np

NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def shapes(n_in=19, hidden=256):
    return {"W1": (hidden, n_in), "b1": (hidden,), "W2": (hidden, hidden), "b2": (hidden,), "W3": (1, hidden),
            "b3": (1,)}


def init_params(rng, n_in=19, hidden=256):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (the usual default)."""
    P = {}
    for name, shp in shapes(n_in, hidden).items():
        fan_in = n_in if name in ("W1", "b1") else hidden
        a = 1.0 / np.sqrt(fan_in)
        P[name] = rng.uniform(-a, a, size=shp)
    return P


def flatten(P):
    return np.concatenate([np.asarray(P[k], dtype=np.float64).ravel() for k in NAMES])


def unflatten(v, n_in=19, hidden=256):
    P, o = {}, 0
    for k in NAMES:
        shp = shapes(n_in, hidden)[k]
        size = int(np.prod(shp))
        P[k] = np.asarray(v[o:o + size], dtype=np.float64).reshape(shp)
        o += size
    return P


def forward(P, X):
    """y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 for every row x of X; returns (y, cache)."""
    Z1 = X @ P["W1"].T + P["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ P["W2"].T + P["b2"]
    H2 = np.maximum(Z2, 0.0)
    y = (H2 @ P["W3"].T + P["b3"])[:, 0]
    return y, (X, Z1, H1, Z2, H2)


def mse(y, t):
    return float(np.mean((y - t) ** 2))


def backward(P, cache, y, t):
    """Gradients of the mean squared error mean((y - t)^2) with respect to every parameter."""
    X, Z1, H1, Z2, H2 = cache
    dy = 2.0 * (y - t) / len(t)
    G = {"W3": dy[None, :] @ H2, "b3": np.array([dy.sum()])}
    dZ2 = (dy[:, None] * P["W3"]) * (Z2 > 0)
    G["W2"] = dZ2.T @ H1
    G["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ P["W2"]) * (Z1 > 0)
    G["W1"] = dZ1.T @ X
    G["b1"] = dZ1.sum(axis=0)
    return G


def adam_init(P):
    return {"m": {k: np.zeros_like(v) for k, v in P.items()}, "v": {k: np.zeros_like(v) for k, v in P.items()}}


def adam_step(P, G, state, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step number `step` (1-based): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
    p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps)."""
    for k in NAMES:
        g = G[k]
        state["m"][k] = beta1 * state["m"][k] + (1 - beta1) * g
        state["v"][k] = beta2 * state["v"][k] + (1 - beta2) * g * g
        mh = state["m"][k] / (1 - beta1 ** step)
        vh = state["v"][k] / (1 - beta2 ** step)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return P

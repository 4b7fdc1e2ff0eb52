"""FP64 reference of the fusion cost model: a multilayer perceptron with three
ReLU hidden layers, a linear scalar output, mean-squared-error loss and Adam.

TEST INFRASTRUCTURE ONLY (the GPU library's MLP kernels are checked against it).

Parameter layout (shared with the GPU library's flat float array, in order):
W1 [F, H], b1 [H], W2 [H, H], b2 [H], W3 [H, H], b3 [H], W4 [H, 1], b4 [1].
Forward for one sample x: h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2),
h3 = relu(h2 W3 + b3), y = h3 W4 + b4.  Loss over a batch of B samples:
L = (1/B) sum_s (y_s - t_s)^2.  Adam (Kingma & Ba 2015) with bias correction:
m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2, theta <- theta - lr mhat / (sqrt(vhat) + eps),
mhat = m / (1 - b1^step), vhat = v / (1 - b2^step).
"""
from __future__ import annotations

import numpy as np


def shapes(n_in: int, hidden: int = 64):
    return [(n_in, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, 1), (1,)]


def n_params(n_in: int, hidden: int = 64) -> int:
    return int(sum(np.prod(s) for s in shapes(n_in, hidden)))


def unpack(theta: np.ndarray, n_in: int, hidden: int = 64):
    out, k = [], 0
    for s in shapes(n_in, hidden):
        size = int(np.prod(s))
        out.append(np.asarray(theta[k:k + size], dtype=np.float64).reshape(s))
        k += size
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def forward(theta, X, n_in: int, hidden: int = 64):
    """Returns (y [B], cache)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta, n_in, hidden)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0)
    z3 = h2 @ W3 + b3
    h3 = np.maximum(z3, 0)
    y = (h3 @ W4 + b4)[:, 0]
    return y, (X, z1, h1, z2, h2, z3, h3)


def loss(theta, X, t, n_in: int, hidden: int = 64) -> float:
    y, _ = forward(theta, X, n_in, hidden)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(theta, X, t, n_in: int, hidden: int = 64):
    """(loss, dL/dtheta) by the chain rule through the layers above."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta, n_in, hidden)
    y, (X, z1, h1, z2, h2, z3, h3) = forward(theta, X, n_in, hidden)
    t = np.asarray(t, dtype=np.float64)
    B = X.shape[0]
    dy = 2.0 * (y - t) / B                      # [B]
    dW4 = h3.T @ dy[:, None]
    db4 = np.array([dy.sum()])
    dz3 = (dy[:, None] * W4[:, 0][None, :]) * (z3 > 0)
    dW3 = h2.T @ dz3
    db3 = dz3.sum(0)
    dz2 = (dz3 @ W3.T) * (z2 > 0)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * (z1 > 0)
    dW1 = X.T @ dz1
    db1 = dz1.sum(0)
    return float(np.mean((y - t) ** 2)), pack([dW1, db1, dW2, db2, dW3, db3, dW4, db4])


def adam_step(theta, g, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update; returns (theta, m, v).  `step` counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v

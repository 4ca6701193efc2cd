"""fp64 reference of the level-selector network (forward, backward, Adam).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and never by the product
package.  Plain numpy in float64, written from the textbook definitions:

* network 16 -> 64 -> 64 -> 6, ReLU after the two hidden layers, softmax over
  the six error-bound levels of Sec. 3.7 (lossless, 1e-5 ... 1e-1);
* loss = mean over samples of the cross-entropy -log p[label];
* gradients by the chain rule (ReLU'(0) taken as 0);
* Adam (Kingma and Ba, 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and
  bias correction.

Parameter vector (float, 5638 entries), in this order: W1 (64 x 16, row
major, W1[j, i] multiplies input i into unit j), b1 (64), W2 (64 x 64), b2
(64), W3 (6 x 64), b3 (6).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 16, 64, 6
SHAPES = [(N_H, N_IN), (N_H,), (N_H, N_H), (N_H,), (N_OUT, N_H), (N_OUT,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)   # 5638
BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == N_PARAMS
    out, k = [], 0
    for s in SHAPES:
        m = int(np.prod(s))
        out.append(theta[k:k + m].reshape(s))
        k += m
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in parts])


def forward(theta, X):
    """Returns (probabilities N x 6, cache)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    zmax = z.max(axis=1, keepdims=True)
    e = np.exp(z - zmax)
    p = e / e.sum(axis=1, keepdims=True)
    return p, (X, a1, h1, a2, h2, z)


def loss(theta, X, y):
    p, _ = forward(theta, X)
    y = np.asarray(y, dtype=np.int64)
    return float(-np.mean(np.log(p[np.arange(len(y)), y])))


def grad(theta, X, y):
    """(loss, gradient vector) of the mean cross-entropy."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    p, (X, a1, h1, a2, h2, z) = forward(theta, X)
    y = np.asarray(y, dtype=np.int64)
    n = len(y)
    L = float(-np.mean(np.log(p[np.arange(n), y])))
    dz = p.copy()
    dz[np.arange(n), y] -= 1.0
    dz /= n
    gW3 = dz.T @ h2
    gb3 = dz.sum(axis=0)
    dh2 = dz @ W3
    da2 = dh2 * (a2 > 0.0)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (a1 > 0.0)
    gW1 = da1.T @ X
    gb1 = da1.sum(axis=0)
    return L, pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam(theta, m, v, g, lr, t):
    """One Adam step at step number t >= 1; returns (theta, m, v)."""
    m = BETA1 * m + (1.0 - BETA1) * g
    v = BETA2 * v + (1.0 - BETA2) * g * g
    mhat = m / (1.0 - BETA1 ** t)
    vhat = v / (1.0 - BETA2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + EPS), m, v


def predict(theta, X):
    """Level with the largest probability (lowest level on ties)."""
    p, _ = forward(theta, X)
    return np.argmax(p, axis=1).astype(np.uint8)

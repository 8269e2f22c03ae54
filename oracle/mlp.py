"""CPU reference of the learned cost model, in float64 (test infrastructure:
only tests, the smoke check and the benchmark's CPU leg use it).

The model is a plain multilayer perceptron 4 -> 64 -> 64 -> S with ReLU
hidden layers.  It maps a problem's features (log2 m, log2 n, density, rank
estimate / min(m, n), the first two scaled by 1/16) to predicted log run times
of S candidate schedules.  It is trained by minimising the masked mean squared
error with Adam (Kingma & Ba, "Adam: A Method for Stochastic Optimization",
Algorithm 1).  The cost model exists because the paper observes that
field-operation counts mispredict run time (Section 1).

Parameter layout (one flat array): W1[4][64] b1[64] W2[64][64] b2[64]
W3[64][S] b3[S], W[a][j] connecting input a to output j.

Pins: the analytic gradient is checked against central finite differences,
the forward pass against a hand-computed network, the Adam step against its
closed-form first step.
"""
from __future__ import annotations

import numpy as np

H = 64

# Planted mistakes for the tests that show the pins catch them (0 = none):
# 1 drops the ReLU mask of the second hidden layer in the backward pass,
# 2 uses W2 instead of its transpose, 3 loses the factor 2 of the square.
MUTATION = 0


def param_count(S: int) -> int:
    return 4 * H + H + H * H + H + H * S + S


def unpack(params: np.ndarray, S: int):
    p = np.asarray(params, dtype=np.float64)
    o = 0
    W1 = p[o:o + 4 * H].reshape(4, H); o += 4 * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H * S].reshape(H, S); o += H * S
    b3 = p[o:o + S]; o += S
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def scale(feats: np.ndarray) -> np.ndarray:
    x = np.asarray(feats, dtype=np.float64).reshape(-1, 4).copy()
    x[:, 0] /= 16.0
    x[:, 1] /= 16.0
    return x


def forward(params, S, feats):
    """Returns (x, h1, h2, y) for every problem (rows)."""
    W1, b1, W2, b2, W3, b3 = unpack(params, S)
    x = scale(feats)
    h1 = np.maximum(x @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    y = h2 @ W3 + b3
    return x, h1, h2, y


def loss(params, S, feats, target, mask, inv_count):
    y = forward(params, S, feats)[3]
    d = y - np.asarray(target, np.float64)
    return float(inv_count * np.sum(np.asarray(mask, np.float64) * d * d))


def grad(params, S, feats, target, mask, inv_count):
    """Gradient of loss() by backpropagation; returns (gradient, loss)."""
    W1, b1, W2, b2, W3, b3 = unpack(params, S)
    x, h1, h2, y = forward(params, S, feats)
    M = np.asarray(mask, np.float64)
    d = y - np.asarray(target, np.float64)
    L = float(inv_count * np.sum(M * d * d))
    dy = (1.0 if MUTATION == 3 else 2.0) * M * d * inv_count
    gW3 = h2.T @ dy
    gb3 = dy.sum(axis=0)
    dh2 = (dy @ W3.T) * (1.0 if MUTATION == 1 else (h2 > 0))
    gW2 = h1.T @ dh2
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ (W2 if MUTATION == 2 else W2.T)) * (h1 > 0)
    gW1 = x.T @ dh1
    gb1 = dh1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return g, L


def fd_grad(params, S, feats, target, mask, inv_count, idx, h=1e-6):
    """Central differences of loss() at the parameter indices idx."""
    p = np.asarray(params, np.float64).copy()
    out = []
    for i in idx:
        old = p[i]
        p[i] = old + h
        lp = loss(p, S, feats, target, mask, inv_count)
        p[i] = old - h
        lm = loss(p, S, feats, target, mask, inv_count)
        p[i] = old
        out.append((lp - lm) / (2 * h))
    return np.array(out)


def adam(params, g, m1, m2, lr, beta1, beta2, eps, step):
    """One Adam step (bias-corrected moments); returns new (params, m1, m2)."""
    g = np.asarray(g, np.float64)
    m1 = beta1 * np.asarray(m1, np.float64) + (1 - beta1) * g
    m2 = beta2 * np.asarray(m2, np.float64) + (1 - beta2) * g * g
    mh = m1 / (1 - beta1 ** step)
    vh = m2 / (1 - beta2 ** step)
    return np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + eps), m1, m2

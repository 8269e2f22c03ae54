"""Pins of the CPU reference cost-model network (oracle/mlp.py) against
things other than itself: finite differences, a network small enough to
evaluate by hand, and Adam's closed-form first step."""
import numpy as np
import pytest

from oracle import mlp


def random_problem(S, N, seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp.param_count(S))
    f = np.c_[rng.uniform(6, 16, (N, 2)), rng.uniform(0, 1, (N, 2))]
    t = rng.normal(0, 1, (N, S))
    M = (rng.random((N, S)) < 0.7).astype(float)
    M[0, 0] = 1.0
    return p, f, t, M, 1.0 / M.sum()


@pytest.mark.parametrize("S,N,seed", [(1, 3, 0), (5, 7, 1), (20, 40, 2), (64, 9, 3)])
def test_gradient_matches_finite_differences(S, N, seed):
    p, f, t, M, ic = random_problem(S, N, seed)
    g, L = mlp.grad(p, S, f, t, M, ic)
    assert abs(L - mlp.loss(p, S, f, t, M, ic)) <= 1e-12 * max(1.0, abs(L))
    idx = np.random.default_rng(seed + 10).choice(p.size, 60, replace=False)
    idx = np.unique(np.r_[idx, [0, 4 * 64, 4 * 64 + 64, p.size - 1]])
    fd = mlp.fd_grad(p, S, f, t, M, ic, idx)
    assert np.max(np.abs(fd - g[idx])) <= 1e-6 * max(1.0, np.max(np.abs(g)))


@pytest.mark.parametrize("mutation", [1, 2, 3])
def test_planted_gradient_mistakes_are_caught(mutation):
    S, N = 6, 12
    p, f, t, M, ic = random_problem(S, N, 5)
    idx = np.arange(p.size)[:: max(1, p.size // 300)]
    fd = mlp.fd_grad(p, S, f, t, M, ic, idx)
    old = mlp.MUTATION
    try:
        mlp.MUTATION = mutation
        g, _ = mlp.grad(p, S, f, t, M, ic)
    finally:
        mlp.MUTATION = old
    assert np.max(np.abs(fd - g[idx])) > 1e-3 * np.max(np.abs(fd))


def test_forward_by_hand():
    # S = 2; W1 passes feature a to hidden unit a (a < 4), b1 = 0; W2 = identity,
    # b2 = -0.25; W3 sums hidden units 0..3 into output 0 and takes unit 2
    # twice into output 1; b3 = (1, -1).
    S = 2
    W1 = np.zeros((4, 64)); W1[np.arange(4), np.arange(4)] = 1.0
    b1 = np.zeros(64)
    W2 = np.eye(64)
    b2 = np.full(64, -0.25)
    W3 = np.zeros((64, S)); W3[:4, 0] = 1.0; W3[2, 1] = 2.0
    b3 = np.array([1.0, -1.0])
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    f = np.array([[8.0, 12.0, 0.5, 0.1]])    # scaled: 0.5, 0.75, 0.5, 0.1
    y = mlp.forward(p, S, f)[3][0]
    h2 = np.maximum(np.array([0.5, 0.75, 0.5, 0.1]) - 0.25, 0.0)   # 0.25, 0.5, 0.25, 0
    assert np.allclose(y, [1.0 + h2.sum(), -1.0 + 2 * h2[2]])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    q, m1, m2 = mlp.adam(p, g, np.zeros(50), np.zeros(50), lr, b1, b2, eps, 1)
    # bias-corrected first moments equal g and g^2, so the step is lr * g / (|g| + eps)
    assert np.allclose(q, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-12)
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)

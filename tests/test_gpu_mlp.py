"""GPU parity of the cost-model kernels (fp32) against the float64 CPU
reference network: initialisation, forward, gradient, Adam, argmin."""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from oracle import mlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1006_1744_amd as g  # noqa: E402


def problem(S, N, seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp.param_count(S)).astype(np.float32)
    f = np.c_[rng.uniform(6, 16, (N, 2)), rng.uniform(0, 1, (N, 2))].astype(np.float32)
    t = rng.normal(0, 1, (N, S)).astype(np.float32)
    M = (rng.random((N, S)) < 0.7).astype(np.float32)
    return p, f, t, M


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("S", [1, 20, 200])
def test_init_matches_splitmix_definition(S):
    P = mlp.param_count(S)
    params = torch.empty(P, dtype=torch.float32, device="cuda")
    g.mlp_init(params, S, 1234)
    got = params.cpu().numpy().astype(np.float64)
    H = 64
    fans = np.zeros(P)
    fans[:4 * H] = 4
    o2 = 4 * H + H
    fans[o2:o2 + H * H] = H
    o3 = o2 + H * H + H
    fans[o3:o3 + H * S] = H
    idx = np.arange(P)[:: max(1, P // 400)]
    for i in idx:
        if fans[i] == 0:
            assert got[i] == 0.0
        else:
            u = (synth.splitmix(1234, int(i)) >> 40) / float(1 << 24)
            want = (2 * u - 1) * math.sqrt(6.0 / fans[i])
            assert abs(got[i] - want) <= 1e-6 * max(1.0, abs(want)), i


@pytest.mark.parametrize("S,N", [(1, 5), (20, 37), (64, 100), (200, 33)])
def test_forward_matches_reference(S, N):
    p, f, _, _ = problem(S, N, S + N)
    y = g.mlp_forward(dev(p), S, dev(f)).cpu().numpy()
    want = mlp.forward(p, S, f)[3]
    assert np.max(np.abs(y - want)) <= 1e-5 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("S,N", [(1, 3), (20, 300), (64, 77), (200, 50)])
def test_gradient_matches_reference(S, N):
    p, f, t, M = problem(S, N, 7 * S + N)
    ic = 1.0 / max(1.0, float(M.sum()))
    out = g.mlp_grad(dev(p), S, dev(f), dev(t), dev(M), ic).cpu().numpy().astype(np.float64)
    want, L = mlp.grad(p, S, f, t, M, ic)
    scale = max(1e-12, np.max(np.abs(want)))
    assert np.max(np.abs(out[:-1] - want)) <= 1e-4 * scale
    assert abs(out[-1] - L) <= 1e-5 * max(1.0, abs(L))


def test_adam_matches_reference():
    S = 20
    P = mlp.param_count(S)
    rng = np.random.default_rng(4)
    p = rng.normal(0, 0.3, P).astype(np.float32)
    gr = rng.normal(0, 1, P).astype(np.float32)
    # first moments with the gradient's sign: the update adds two same-signed terms,
    # so fp32 rounding stays relative to the result (no cancellation)
    m1 = (np.sign(gr) * np.abs(rng.normal(0, 0.1, P))).astype(np.float32)
    m2 = rng.uniform(0, 0.1, P).astype(np.float32)
    dp, dm1, dm2 = dev(p), dev(m1), dev(m2)
    g.mlp_adam(dp, S, dev(np.r_[gr, 0.0].astype(np.float32)), dm1, dm2, 1e-3, step=3)
    # the kernel receives fp32 hyperparameters: give the reference the same values
    f32 = lambda v: float(np.float32(v))  # noqa: E731
    wp, wm1, wm2 = mlp.adam(p, gr, m1, m2, f32(1e-3), f32(0.9), f32(0.999), f32(1e-8), 3)
    assert np.allclose(dp.cpu().numpy(), wp, rtol=1e-5, atol=1e-7)
    assert np.allclose(dm1.cpu().numpy(), wm1, rtol=1e-5, atol=1e-8)
    assert np.allclose(dm2.cpu().numpy(), wm2, rtol=1e-5, atol=1e-9)


def test_predict_is_argmin():
    S, N = 20, 500
    p, f, _, _ = problem(S, N, 11)
    table = np.array([[4 + s % 5, [1, 2, 4, 8][s // 5], 512, 1] for s in range(S)], np.int32)
    out = g.costmodel_predict(dev(p), S, dev(f), dev(table)).cpu().numpy()
    y = mlp.forward(p, S, f)[3]
    for i in range(N):
        srt = np.sort(y[i])
        j = int(np.argmin(y[i]))
        if srt[1] - srt[0] > 1e-3:
            assert np.array_equal(out[i], table[j]), i
        else:
            k = [s for s in range(S) if np.array_equal(table[s], out[i])][0]
            assert y[i, k] <= srt[0] + 1e-3

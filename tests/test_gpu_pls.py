"""GPU parity: the HIP path through the C-ABI against the CPU oracle, bit for bit.

Every comparison covers rank, P, Q and every word of the in-place matrix
(padding included), or every word of the RREF.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU runs deselect the marker anyway
    pytest.skip("no GPU", allow_module_level=True)

import paper_1006_1744_amd as g  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_pls(A: np.ndarray, m: int, n: int, s=None):
    dA = g.to_device(A)
    P, Q, rank = g.pls(dA, m, n, s)
    torch.cuda.synchronize()
    return int(rank.item()), P.cpu().numpy(), Q.cpu().numpy(), g.to_host(dA), dA, Q, rank


def assert_same_pls(A, m, n, s=None, label=""):
    say(f"[pls] {label} m={m} n={n} sched={s}")
    r, P, Q, Ap = oracle.pls(A, m, n)
    gr, gP, gQ, gAp, *_ = gpu_pls(A, m, n, s)
    assert gr == r, f"rank {gr} != {r}"
    assert np.array_equal(gQ[:n], Q), "Q differs"
    assert np.array_equal(gP[:m], P), "P differs"
    if not np.array_equal(gAp, Ap):
        bad = np.argwhere(gAp != Ap)
        raise AssertionError(f"A' differs at {len(bad)} words, first {bad[:5].tolist()}")


SCHEDS = {
    "default": None,
    "mmpf": g.Sched(8, 8, 1 << 20, g.SCHUR_MFMA),
    "rec64_xor": g.Sched(8, 8, 64, g.SCHUR_XOR),
    "rec64_mfma": g.Sched(8, 8, 64, g.SCHUR_MFMA),
    "k4t1_c128": g.Sched(4, 1, 128, g.SCHUR_XOR),
    "k5t2_c256": g.Sched(5, 2, 256, g.SCHUR_MFMA),
    "rec64_fp4": g.Sched(8, 8, 64, g.SCHUR_FP4),
    "k6t4_c128_fp4": g.Sched(6, 4, 128, g.SCHUR_FP4),
}


# ---------------------------------------------------------------- products
@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("m,k,n", [(1, 1, 1), (64, 64, 64), (100, 70, 130), (257, 300, 190),
                                   (512, 1024, 384), (1000, 129, 65), (1000, 700, 1000),
                                   (300, 4000, 300), (2100, 600, 1100), (257, 65, 4096),
                                   (300, 8200, 300), (520, 4160, 700), (256, 4608, 256)])
def test_addmul(variant, m, k, n):
    say(f"[addmul] variant={variant} m={m} k={k} n={n}")
    A = synth.random_half(m, k, 11 + m)
    B = synth.random_half(k, n, 12 + n)
    C = synth.random_half(m, n, 13 + k)
    want = oracle.pack_bits(oracle.unpack_bits(C, n) ^ oracle.gf2_matmul_bits(
        oracle.unpack_bits(A, k), oracle.unpack_bits(B, n)))
    dC, dA, dB = g.to_device(C), g.to_device(A), g.to_device(B)
    g.addmul(dC, dA, dB, m, k, n, variant)
    torch.cuda.synchronize()
    assert np.array_equal(g.to_host(dC), want)


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("m,k,n", [(4400, 4160, 4160), (20000, 2000, 1000)])
def test_addmul_multi_tile_sampled(variant, m, k, n):
    """More tiles than product blocks (each block walks several tiles' stages as
    one pipeline) with a K tail and partial edge tiles; sampled rows against the
    oracle's product."""
    say(f"[addmul sampled] variant={variant} m={m} k={k} n={n}")
    A = synth.random_half(m, k, 21 + m)
    B = synth.random_half(k, n, 22 + n)
    C = synth.random_half(m, n, 23 + k)
    dC, dA, dB = g.to_device(C), g.to_device(A), g.to_device(B)
    g.addmul(dC, dA, dB, m, k, n, variant)
    torch.cuda.synchronize()
    got = g.to_host(dC)
    rows = np.unique(np.concatenate([np.arange(0, m, 97), np.arange(m - 40, m)]))
    want = oracle.pack_bits(oracle.unpack_bits(C[rows], n) ^ oracle.gf2_matmul_bits(
        oracle.unpack_bits(A[rows], k), oracle.unpack_bits(B, n)))
    assert np.array_equal(got[rows][:, :want.shape[1]], want)


# ---------------------------------------------------------------- PLS
SHAPES = [(1, 1), (1, 100), (100, 1), (64, 64), (65, 63), (63, 130), (130, 200), (300, 257),
          (257, 300), (512, 512), (700, 1000), (1000, 700)]


@pytest.mark.parametrize("sname", list(SCHEDS))
@pytest.mark.parametrize("m,n", SHAPES)
def test_pls_dense(sname, m, n):
    A = synth.random_half(m, n, 7 * m + n)
    assert_same_pls(A, m, n, SCHEDS[sname], f"dense/{sname}")


@pytest.mark.parametrize("sname", ["default", "mmpf", "rec64_xor"])
@pytest.mark.parametrize("p", [0.1, 0.01, 0.002])
@pytest.mark.parametrize("m,n", [(130, 200), (600, 600), (1000, 700)])
def test_pls_sparse(sname, p, m, n):
    A = synth.random_bernoulli(m, n, p, 31 * m + n)
    assert_same_pls(A, m, n, SCHEDS[sname], f"p={p}/{sname}")


@pytest.mark.parametrize("sname", ["default", "mmpf", "rec64_mfma", "k4t1_c128", "rec64_fp4"])
@pytest.mark.parametrize("m,n,r", [(200, 300, 90), (512, 512, 300), (700, 900, 650),
                                   (1000, 1000, 999), (300, 300, 0), (800, 400, 130)])
def test_pls_planted(sname, m, n, r):
    A = synth.planted(m, n, r, 5 + r, p=0.5, unit=True)
    assert_same_pls(A, m, n, SCHEDS[sname], f"planted r={r}/{sname}")


def test_pls_special():
    m, n = 300, 400
    for name, X in [("zero", np.zeros((m, n), np.uint8)),
                    ("identity", np.eye(m, n, dtype=np.uint8)),
                    ("ones", np.ones((m, n), np.uint8))]:
        A = oracle.pack_bits(X)
        for sname in ("default", "mmpf", "rec64_xor"):
            assert_same_pls(A, m, n, SCHEDS[sname], f"{name}/{sname}")
    X = np.zeros((m, n), np.uint8)
    X[m - 1, 70] = 1
    X[m - 1, 5] = 1
    X[m - 2, 200] = 1
    A = oracle.pack_bits(X)
    for sname in ("default", "mmpf", "rec64_xor"):
        assert_same_pls(A, m, n, SCHEDS[sname], f"last-row/{sname}")
    # zero columns exactly at panel and split boundaries
    X = (np.random.default_rng(1).random((m, n)) < 0.5).astype(np.uint8)
    X[:, 64:70] = 0
    X[:, 128] = 0
    X[:, 255:258] = 0
    A = oracle.pack_bits(X)
    for sname in ("default", "mmpf", "rec64_xor", "k5t2_c256"):
        assert_same_pls(A, m, n, SCHEDS[sname], f"zero-cols/{sname}")


def test_pls_padded_stride():
    m, n = 333, 250
    A = synth.random_half(m, n, 3, stride=6)
    assert_same_pls(A, m, n, None, "stride6")


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_pls_4096(seed):
    n = 4096
    A = synth.random_half(n, n, seed)
    assert_same_pls(A, n, n, SCHEDS["mmpf"], f"4096 seed={seed} mmpf")
    assert_same_pls(A, n, n, None, f"4096 seed={seed} default")


# ---------------------------------------------------------------- RREF
@pytest.mark.parametrize("m,n,kind", [(64, 64, "half"), (300, 257, "half"), (257, 300, "half"),
                                      (500, 700, "planted"), (700, 500, "sparse"),
                                      (1, 50, "half"), (50, 1, "half"), (200, 200, "zero"),
                                      (600, 3000, "half"), (1500, 1400, "planted1200"),
                                      (1300, 4000, "half"), (300, 64, "half"), (1000, 640, "half")])
def test_rref(m, n, kind):
    if kind == "half":
        A = synth.random_half(m, n, m + 2 * n)
    elif kind == "planted":
        A = synth.planted(m, n, 333, 9, p=0.5)
    elif kind == "planted1200":
        A = synth.planted(m, n, 1200, 9, p=0.5)
    elif kind == "sparse":
        A = synth.random_bernoulli(m, n, 0.01, 4)
    else:
        A = synth.empty(m, n)
    say(f"[rref] {kind} m={m} n={n}")
    r, R, piv = oracle.rref(A, m, n)
    gr, gP, gQ, gAp, dAp, dQ, drank = gpu_pls(A, m, n)
    dR = g.rref(dAp, m, n, dQ, drank)
    torch.cuda.synchronize()
    assert gr == r
    assert np.array_equal(g.to_host(dR), R)


def test_rref_4096():
    n = 4096
    A = synth.random_half(n, n, 1)
    say("[rref] 4096")
    r, R, piv = oracle.rref(A, n, n)
    gr, gP, gQ, gAp, dAp, dQ, drank = gpu_pls(A, n, n)
    dR = g.rref(dAp, n, n, dQ, drank)
    torch.cuda.synchronize()
    assert gr == r and np.array_equal(g.to_host(dR), R)


# ---------------------------------------------------------------- unpack
@pytest.mark.parametrize("m,n,kind", [(1, 1, "half"), (300, 257, "half"), (257, 300, "half"),
                                      (500, 700, "planted"), (700, 130, "sparse"), (200, 200, "zero")])
def test_pls_unpack(m, n, kind):
    if kind == "half":
        A = synth.random_half(m, n, 3 * m + n)
    elif kind == "planted":
        A = synth.planted(m, n, 321, 4, p=0.5)
    elif kind == "sparse":
        A = synth.random_bernoulli(m, n, 0.01, 6)
    else:
        A = synth.empty(m, n)
    say(f"[unpack] {kind} m={m} n={n}")
    r, P, Q, Ap = oracle.pls(A, m, n)
    L0, S0 = oracle.unpack_LS(Ap, m, n, r, Q)
    gr, gP, gQ, gAp, dAp, dQ, drank = gpu_pls(A, m, n)
    dL, dS = g.pls_unpack(dAp, m, n, dQ, drank)
    torch.cuda.synchronize()
    rmax = min(m, n)
    L = oracle.unpack_bits(g.to_host(dL), rmax)
    S = oracle.unpack_bits(g.to_host(dS), n)
    assert np.array_equal(L[:, :r], L0) and not L[:, r:].any()
    assert np.array_equal(S[:r], S0)

"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (one gf2_pls call with the default schedule, then gf2_rref), against the
CPU oracle run on the same input: rank, P, Q and every word of the in-place
result bit for bit.  The RREF is checked through properties that pin it at any
size (rows past the rank are zero, the pivot columns form the identity, and
S = U_Q R by Freivalds' test with random vectors), because forming it on the
host by Gauss-Jordan at these sizes would take minutes."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1006_1744_amd as g  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def matvec(M: np.ndarray, v: np.ndarray, rows: int, chunk: int = 4096) -> np.ndarray:
    """Parity of popcount(M[i] & v) for i < rows (packed rows and vector)."""
    out = np.empty(rows, dtype=np.uint8)
    for a in range(0, rows, chunk):
        b = min(rows, a + chunk)
        out[a:b] = np.bitwise_count(M[a:b] & v[None, :]).sum(axis=1, dtype=np.int64) & 1
    return out


def scatter_bits(y: np.ndarray, Q: np.ndarray, n: int) -> np.ndarray:
    """Packed n-bit vector with bit Q[j] = y[j]."""
    z = np.zeros((n + 63) // 64, dtype=np.uint64)
    on = Q[y.astype(bool)].astype(np.int64)
    np.bitwise_or.at(z, on // 64, np.left_shift(np.uint64(1), (on % 64).astype(np.uint64)))
    return z


def s_rows(Ap: np.ndarray, r: int, Q: np.ndarray, n: int) -> np.ndarray:
    """S (r x n, packed) from the in-place result: stored bits right of Q[i], one at Q[i]."""
    W = (n + 63) // 64
    S = np.ascontiguousarray(Ap[:r, :W]).copy()
    q = Q[:r].astype(np.int64)
    cols = np.arange(W, dtype=np.int64)[None, :]
    w = (q // 64)[:, None]
    S[cols < w] = 0
    lo = (q % 64).astype(np.uint64)
    # bits at or below the pivot in its word are cleared (all of them when lo == 63)
    low = np.where(lo == 63, ~np.uint64(0),
                   np.left_shift(np.uint64(1), np.minimum(lo + np.uint64(1), np.uint64(63))) - np.uint64(1))
    keep = ~low
    idx = np.arange(r)
    S[idx, q // 64] = (S[idx, q // 64] & keep) | np.left_shift(np.uint64(1), lo)
    return S


def check_rref_properties(R: np.ndarray, S: np.ndarray, r: int, Q: np.ndarray, n: int,
                          trials: int = 16):
    W = (n + 63) // 64
    assert not R[r:, :W].any(), "rows past the rank must be zero"
    rng = np.random.default_rng(99)
    for _ in range(trials):
        # R[:, Q] = I:  R z(y) = y for a random r-vector y
        y = rng.integers(0, 2, r, dtype=np.uint8)
        assert np.array_equal(matvec(R, scatter_bits(y, Q[:r], n), r), y), "R[:, Q] != I"
        # S = U_Q R with U_Q = S[:, Q]:  S v = S z(R v)
        v = rng.integers(0, np.iinfo(np.uint64).max, W, dtype=np.uint64, endpoint=True)
        if n % 64:
            v[-1] &= np.uint64((1 << (n % 64)) - 1)
        Rv = matvec(R, v, r)
        assert np.array_equal(matvec(S, v, r), matvec(S, scatter_bits(Rv, Q[:r], n), r)), \
            "S != U_Q R"


def run_full(A, m, n, s=None, rref=True):
    dA = g.to_device(A)
    P, Q, rank = g.pls(dA, m, n, s)
    R = g.rref(dA, m, n, Q, rank) if rref else None
    torch.cuda.synchronize()
    return (int(rank.item()), P.cpu().numpy(), Q.cpu().numpy(), g.to_host(dA),
            g.to_host(R) if rref else None)


def compare(label, got, want):
    gr, gP, gQ, gAp = got[:4]
    r, P, Q, Ap = want
    assert gr == r, f"{label}: rank {gr} != {r}"
    assert np.array_equal(gQ, Q), f"{label}: Q differs"
    assert np.array_equal(gP, P), f"{label}: P differs"
    assert np.array_equal(gAp, Ap), f"{label}: A' differs"


def test_full_65536_dense_all_schur_variants():
    m = n = 65536
    A = synth.random_half(m, n, 1)
    say("[full] 65536^2 p=1/2 seed 1: GPU (fp4 MFMA Schur, default schedule)")
    got = run_full(A, m, n)
    say("[full] oracle")
    want = oracle.pls(A, m, n)
    compare("65536 fp4 MFMA", got, want)
    r = want[0]
    if r == n:   # full rank: the RREF is the identity
        I = np.zeros_like(got[4])
        idx = np.arange(n)
        I[idx, idx // 64] = np.left_shift(np.uint64(1), (idx % 64).astype(np.uint64))
        assert np.array_equal(got[4], I)
    else:
        check_rref_properties(got[4], s_rows(want[3], r, want[2], n), r, want[2], n)
    say("[full] GPU with the int8 MFMA Schur product")
    got_i = run_full(A, m, n, g.Sched(8, 8, 512, g.SCHUR_MFMA), rref=False)
    compare("65536 int8 MFMA", got_i, want)
    del got_i
    say("[full] GPU with the XOR-popcount Schur product")
    got_x = run_full(A, m, n, g.Sched(8, 8, 512, g.SCHUR_XOR), rref=False)
    compare("65536 XOR", got_x, want)


def test_full_65536_sparse():
    m = n = 65536
    A = synth.random_bernoulli(m, n, 0.01, 2)
    say("[full] 65536^2 p=0.01 seed 2")
    got = run_full(A, m, n)
    want = oracle.pls(A, m, n)
    compare("65536 sparse", got, want)
    r, P, Q, Ap = want
    check_rref_properties(got[4], s_rows(Ap, r, Q, n), r, Q, n)


def test_full_32768x131072():
    m, n = 32768, 131072
    A = synth.random_half(m, n, 3)
    say("[full] 32768x131072 p=1/2 seed 3")
    got = run_full(A, m, n)
    want = oracle.pls(A, m, n)
    compare("32768x131072", got, want)
    r, P, Q, Ap = want
    check_rref_properties(got[4], s_rows(Ap, r, Q, n), r, Q, n)


def test_full_32768_planted_rank_mmpf_and_recursive():
    m = n = 32768
    A = synth.planted(m, n, 24576, 4, p=0.5, unit=False)
    say("[full] 32768^2 planted rank 24576 (B C, Bernoulli(1/2) factors)")
    want = oracle.pls(A, m, n)
    assert want[0] == 24576
    got = run_full(A, m, n)
    compare("32768 planted, recursive", got, want)
    r, P, Q, Ap = want
    check_rref_properties(got[4], s_rows(Ap, r, Q, n), r, Q, n)
    say("[full] the same matrix by MMPF alone")
    got_m = run_full(A, m, n, g.Sched(8, 8, 1 << 20, g.SCHUR_MFMA), rref=False)
    compare("32768 planted, MMPF", got_m, want)

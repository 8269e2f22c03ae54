"""GPU parity of M4RI (Section 3.1, algorithm "M4RI") and of the M+P hybrid
(Section 6: M4RI until the approximated density of the remaining part reaches a
threshold, then PLS-based elimination) against the oracle's Gauss-Jordan
reduction, word for word: the reduced row echelon form is unique, so every
schedule, threshold and switch point must give the same bits, the same rank and
the same pivot columns."""
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


def make_input(kind, m, n, seed):
    w = max((n + 63) // 64, 1)
    if kind == "half":
        return synth.random_half(m, n, seed)
    if kind.startswith("p="):
        return synth.random_bernoulli(m, n, float(kind[2:]), seed)
    if kind == "zero":
        return np.zeros((m, w), dtype=np.uint64)
    if kind == "ones":
        A = np.zeros((m, w), dtype=np.uint64)
        A[:, : n // 64] = np.uint64(0xFFFFFFFFFFFFFFFF)
        if n % 64:
            A[:, n // 64] = np.uint64((1 << (n % 64)) - 1)
        return A
    if kind == "identity":
        A = np.zeros((m, w), dtype=np.uint64)
        for i in range(min(m, n)):
            A[i, i // 64] |= np.uint64(1) << np.uint64(i % 64)
        return A
    if kind == "lastrow":
        # a single one in the last row: the far search reaches the end
        A = np.zeros((m, w), dtype=np.uint64)
        A[m - 1, (n - 1) // 64] = np.uint64(1) << np.uint64((n - 1) % 64)
        return A
    if kind.startswith("planted"):
        return synth.planted(m, n, int(kind[7:]), seed, p=0.5)
    if kind == "sparse_dense":
        # left half Bernoulli(0.01), right half Bernoulli(1/2): density rises as
        # the elimination moves right
        h = (n // 2) // 64 * 64
        L = synth.random_bernoulli(m, h, 0.01, seed)
        Rr = synth.random_half(m, n - h, seed + 1)
        return np.ascontiguousarray(np.concatenate([L[:, : h // 64], Rr], axis=1))
    raise ValueError(kind)


_cache = {}


def oracle_rref(A, m, n, key):
    if key not in _cache:
        _cache[key] = oracle.rref(A, m, n)
    return _cache[key]


def check(label, got_A, got_Q, got_r, want, n):
    r, R, piv = want
    assert got_r == r, f"{label}: rank {got_r} != {r}"
    assert np.array_equal(got_Q[:r], piv), f"{label}: pivot columns differ"
    assert np.array_equal(got_Q[r:], np.arange(r, n, dtype=np.int32)), f"{label}: Q tail"
    assert np.array_equal(got_A, R), f"{label}: RREF differs"


CASES = [
    (1, 1, "half", 1), (1, 1, "zero", 1), (1, 200, "half", 2), (200, 1, "half", 3),
    (64, 64, "half", 4), (65, 130, "half", 5), (200, 200, "zero", 6), (300, 300, "identity", 7),
    (300, 200, "ones", 8), (500, 700, "lastrow", 9), (700, 500, "half", 10),
    (1000, 1000, "planted600", 11), (1500, 1200, "p=0.01", 12), (1200, 1800, "p=0.002", 13),
    (2000, 2000, "planted1999", 14), (1300, 3000, "half", 15), (4096, 4096, "half", 1),
    (4096, 4096, "half", 2), (4096, 4096, "p=0.01", 16), (3000, 2000, "planted1700", 17),
    # many rows and words: the update's grid takes the rows in several chunks per
    # block, so a row's column tiles run in blocks far apart in time (regression:
    # its panel word must not change under them)
    (12307, 13508, "half", 25), (9000, 13508, "p=0.05", 26),
]

SCHEDS = [g.Sched(8, 8, 512, g.SCHUR_FP4), g.Sched(4, 1, 512, g.SCHUR_FP4),
          g.Sched(6, 2, 512, g.SCHUR_FP4), g.Sched(7, 4, 512, g.SCHUR_FP4)]


@pytest.mark.parametrize("m,n,kind,seed", CASES)
def test_m4ri_matches_oracle(m, n, kind, seed):
    A = make_input(kind, m, n, seed)
    want = oracle_rref(A, m, n, (m, n, kind, seed))
    scheds = SCHEDS if m * n <= 4_000_000 else SCHEDS[:2]
    for s in scheds:
        say(f"[m4ri] {kind} {m}x{n} seed {seed} {s}")
        dA = g.to_device(A)
        Q, rank = g.m4ri(dA, m, n, s)
        torch.cuda.synchronize()
        check(f"m4ri {s}", g.to_host(dA), Q.cpu().numpy(), int(rank.item()), want, n)


@pytest.mark.parametrize("m,n,kind,seed", [c for c in CASES if c[0] * c[1] >= 40000])
@pytest.mark.parametrize("threshold", [0.0, 0.05, 0.15, 0.2, 2.0])
def test_rref_mp_matches_oracle(m, n, kind, seed, threshold):
    A = make_input(kind, m, n, seed)
    want = oracle_rref(A, m, n, (m, n, kind, seed))
    dA = g.to_device(A)
    Q, rank, sw = g.rref_mp(dA, m, n, threshold)
    torch.cuda.synchronize()
    say(f"[m+p {threshold}] {kind} {m}x{n}: switched at panel {sw}")
    if threshold == 0.0 and m > 0:
        assert sw == 0
    if threshold > 1.0:
        assert sw == -1
    check(f"m+p {threshold}", g.to_host(dA), Q.cpu().numpy(), int(rank.item()), want, n)


@pytest.mark.parametrize("m,n,threshold,seed", [(3000, 4096, 0.4, 21), (2048, 3000, 0.35, 22)])
@pytest.mark.parametrize("schur", [g.SCHUR_FP4, g.SCHUR_MFMA, g.SCHUR_XOR])
def test_rref_mp_switches_midway(m, n, threshold, seed, schur):
    A = make_input("sparse_dense", m, n, seed)
    want = oracle_rref(A, m, n, (m, n, "sparse_dense", seed))
    dA = g.to_device(A)
    Q, rank, sw = g.rref_mp(dA, m, n, threshold, s=g.Sched(8, 8, 512, schur))
    torch.cuda.synchronize()
    nb = (n + 63) // 64
    say(f"[m+p {threshold}] sparse|dense {m}x{n}: switched at panel {sw} of {nb}")
    assert 0 < sw < nb, "the hybrid should switch between its first and last strip"
    check("m+p midway", g.to_host(dA), Q.cpu().numpy(), int(rank.item()), want, n)


def test_m4ri_padded_stride():
    m, n = 700, 900
    A = make_input("planted500", m, n, 31)
    want = oracle_rref(A, m, n, (m, n, "planted500", 31))
    Ap = np.zeros((m, 20), dtype=np.uint64)
    Ap[:, : A.shape[1]] = A
    dA = g.to_device(Ap)
    Q, rank = g.m4ri(dA, m, n)
    torch.cuda.synchronize()
    got = g.to_host(dA)
    assert not np.any(got[:, A.shape[1]:]), "padding words must stay zero"
    check("m4ri padded", got[:, : A.shape[1]], Q.cpu().numpy(), int(rank.item()), want, n)


def test_m4ri_graph_replay():
    m, n = 2000, 2500
    A = make_input("planted1500", m, n, 41)
    want = oracle_rref(A, m, n, (m, n, "planted1500", 41))
    src = g.to_device(A)
    work = torch.empty_like(src)
    Q = torch.empty(n, dtype=torch.int32, device="cuda")
    rank = torch.empty(1, dtype=torch.int32, device="cuda")
    ws = g.workspace(int(g.get_lib().gf2_m4ri_workspace_bytes(m, n)))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        work.copy_(src)
        g.m4ri(work, m, n, Q=Q, rank=rank, ws=ws, stream=stream)
    stream.synchronize()
    eager = g.to_host(work).copy()
    check("eager", eager, Q.cpu().numpy(), int(rank.item()), want, n)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        g.m4ri(work, m, n, Q=Q, rank=rank, ws=ws, stream=stream)
    for rep in range(3):
        work.copy_(src)
        Q.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        check(f"replay {rep}", g.to_host(work), Q.cpu().numpy(), int(rank.item()), want, n)

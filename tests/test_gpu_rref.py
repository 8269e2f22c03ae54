"""GPU parity of the reduced row echelon form (Definition "Reduced Row Echelon
Form", Section 2; computed from the PLS as in Table 1) against the oracle's
independent Gauss-Jordan elimination, word for word, for every Schur variant the
triangular solve can use; and PLS + RREF captured in one HIP graph (the RREF
reads the rank on the device, so the pair enqueues without waiting)."""
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


VARIANTS = {"fp4": g.SCHUR_FP4, "int8": g.SCHUR_MFMA, "xor": g.SCHUR_XOR}


def make_input(kind, m, n, seed):
    if kind == "half":
        return synth.random_half(m, n, seed)
    if kind.startswith("planted"):
        return synth.planted(m, n, int(kind[7:]), seed, p=0.5)
    if kind == "sparse":
        return synth.random_bernoulli(m, n, 0.01, seed)
    raise ValueError(kind)


# Wide cases whose upper triangular solve reaches the 256 x 256-tile product
# (inner dimension above 2048 at the top of the solve: rank above about 4100
# with non-pivot columns), and smaller ones on the 128 x 128 tiles and the
# blocked table solve alone.
CASES = [
    (5000, 6000, "half", 31),          # rank 5000, top product K = 2560
    (8192, 32768, "half", 32),         # rank 8192, K = 4096, 384 non-pivot words
    (8192, 8192, "planted6144", 33),   # rank 6144, non-pivot columns spread over the width
    (3000, 2000, "planted1700", 34),   # m > n, rank deficient
    (1200, 1800, "sparse", 35),
    (2100, 2300, "half", 36),          # K <= 2048: small tiles only
]


@pytest.fixture(scope="module")
def oracle_rrefs():
    cache = {}

    def get(m, n, kind, seed):
        key = (m, n, kind, seed)
        if key not in cache:
            A = make_input(kind, m, n, seed)
            r, R, piv = oracle.rref(A, m, n)
            cache[key] = (A, r, R)
        return cache[key]
    return get


@pytest.mark.parametrize("m,n,kind,seed", CASES)
def test_rref_all_variants(oracle_rrefs, m, n, kind, seed):
    A, r, R = oracle_rrefs(m, n, kind, seed)
    dA = g.to_device(A)
    P, Q, rank = g.pls(dA, m, n)
    torch.cuda.synchronize()
    assert int(rank.item()) == r
    for name, v in VARIANTS.items():
        say(f"[rref] {kind} {m}x{n} rank {r}, solve products {name}")
        dR = g.rref(dA, m, n, Q, rank, s=g.Sched(8, 8, 512, v))
        torch.cuda.synchronize()
        got = g.to_host(dR)
        if not np.array_equal(got, R):
            bad = np.argwhere(got != R)
            raise AssertionError(f"{name}: R differs at {len(bad)} words, first {bad[:5].tolist()}")


def test_rref_stale_output_and_workspace(oracle_rrefs):
    """R and the workspace hold garbage on entry: every word of R is written."""
    m, n = 1500, 2600
    A, r, R = oracle_rrefs(m, n, "planted1100", 37)
    dA = g.to_device(A)
    P, Q, rank = g.pls(dA, m, n)
    dR = torch.full_like(dA, -1)
    ws = torch.full((g.rref_workspace_bytes(m, n),), 0x5A, dtype=torch.uint8, device="cuda")
    g.rref(dA, m, n, Q, rank, R=dR, ws=ws)
    torch.cuda.synchronize()
    assert np.array_equal(g.to_host(dR), R)


@pytest.mark.parametrize("m,n,kind,seed", [(3000, 5000, "planted2000", 41), (2048, 2048, "half", 42),
                                           (700, 300, "sparse", 43)])
def test_pls_rref_graph_replay(oracle_rrefs, m, n, kind, seed):
    """gf2_pls followed by gf2_rref captured in one HIP graph and replayed three
    times (the input restored between replays by eager copies): every replay
    equals the eager result and the oracle."""
    A, r, R = oracle_rrefs(m, n, kind, seed)
    rp, Pw, Qw, Apw = oracle.pls(A, m, n)
    say(f"[graph] pls + rref {kind} {m}x{n}")
    pristine = g.to_device(A)
    dA = pristine.clone()
    P = torch.empty(m, dtype=torch.int32, device="cuda")
    Q = torch.empty(n, dtype=torch.int32, device="cuda")
    rank = torch.empty(1, dtype=torch.int32, device="cuda")
    dR = torch.empty_like(dA)
    ws = g.workspace(g.pls_workspace_bytes(m, n))
    wsr = g.workspace(g.rref_workspace_bytes(m, n))
    g.pls(dA, m, n, ws=ws, P=P, Q=Q, rank=rank)
    g.rref(dA, m, n, Q, rank, R=dR, ws=wsr)
    torch.cuda.synchronize()
    want_A, want_R = dA.clone(), dR.clone()
    assert np.array_equal(g.to_host(want_R), R)
    assert np.array_equal(g.to_host(want_A), Apw)
    dA.copy_(pristine)
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=stream):
        g.pls(dA, m, n, ws=ws, P=P, Q=Q, rank=rank)
        g.rref(dA, m, n, Q, rank, R=dR, ws=wsr)
    for rep in range(3):
        dA.copy_(pristine)
        dR.fill_(-1)
        rank.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert int(rank.item()) == r, f"replay {rep}: rank"
        assert torch.equal(dA, want_A), f"replay {rep}: A'"
        assert torch.equal(dR, want_R), f"replay {rep}: R"
        assert np.array_equal(P.cpu().numpy(), Pw) and np.array_equal(Q.cpu().numpy(), Qw)

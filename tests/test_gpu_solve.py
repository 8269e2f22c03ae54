"""GPU parity of the linear-system solver and the null-space basis built on the
PLS (abstract and Section 1: the decomposition as the building block for solving
systems), through the C ABI, against the oracle's ``solve_from_pls`` and
``kernel_basis`` (pinned in test_oracle_solve.py by brute force over every x).

The solution with every non-pivot entry zero is unique when it exists, and a
null-space basis with prescribed non-pivot coordinates is unique, so the GPU
results are compared word for word.  At the benchmark's size the oracle's
per-entry loops would take too long; there the result is checked by the
properties that pin it: non-pivot entries zero plus A X = B exactly (64 packed
right-hand sides at once), and for the basis the non-pivot coordinates (the
identity) plus A v = 0 for 64 random combinations v of the basis vectors."""
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
    if kind == "half":
        return synth.random_half(m, n, seed)
    if kind == "sparse":
        return synth.random_bernoulli(m, n, 0.01, seed)
    if kind == "zero":
        return np.zeros((m, max((n + 63) // 64, 1)), dtype=np.uint64)
    if kind == "identity":
        A = np.zeros((m, max((n + 63) // 64, 1)), dtype=np.uint64)
        for i in range(min(m, n)):
            A[i, i // 64] |= np.uint64(1) << np.uint64(i % 64)
        return A
    if kind.startswith("planted"):
        return synth.planted(m, n, int(kind[7:]), seed, p=0.5)
    raise ValueError(kind)


def rhs_block(A, m, n, nrhs, seed, stride=None):
    """nrhs right-hand sides as an m x nrhs packed matrix: even columns A x for a
    random x (consistent), odd columns random (inconsistent unless rank = m)."""
    rng = np.random.default_rng(seed)
    Ab = oracle.unpack_bits(A, n).astype(np.float32)
    cols = np.zeros((m, nrhs), dtype=np.uint8)
    for t in range(nrhs):
        if t % 2 == 0:
            x = rng.integers(0, 2, size=n).astype(np.float32)
            cols[:, t] = (Ab @ x).astype(np.int64) & 1 if n else 0
        else:
            cols[:, t] = rng.integers(0, 2, size=m)
    return oracle.pack_bits(cols, stride), cols


def gpu_pls(A, m, n):
    dA = g.to_device(A)
    P, Q, rank = g.pls(dA, m, n)
    return dA, P, Q, rank


SOLVE_CASES = [
    (1, 1, "half", 1), (1, 1, "zero", 1), (5, 3, "half", 2), (3, 5, "half", 3),
    (64, 64, "half", 64), (65, 63, "half", 65), (200, 200, "zero", 7), (300, 300, "identity", 9),
    (700, 500, "half", 5), (500, 700, "half", 130), (1500, 1500, "planted900", 33),
    (2000, 1300, "sparse", 64), (1300, 2600, "planted1100", 63), (2500, 2500, "half", 12),
]


@pytest.mark.parametrize("m,n,kind,nrhs", SOLVE_CASES)
@pytest.mark.parametrize("variant", [g.SCHUR_FP4, g.SCHUR_MFMA, g.SCHUR_XOR])
def test_solve_matches_oracle(m, n, kind, nrhs, variant):
    if variant != g.SCHUR_FP4 and m * n > 2_000_000:
        pytest.skip("other product variants covered on the smaller cases")
    seed = 500 + m + 3 * n
    A = make_input(kind, m, n, seed)
    Bp, cols = rhs_block(A, m, n, nrhs, seed + 1)
    r, P, Q, Ap = oracle.pls(A, m, n)
    say(f"[solve] {kind} {m}x{n} rank {r} nrhs {nrhs} variant {variant}")
    dA, dP, dQ, drank = gpu_pls(A, m, n)
    X, bad = g.solve(dA, m, n, dP, dQ, drank, g.to_device(Bp), nrhs, s=g.Sched(8, 8, 512, variant))
    torch.cuda.synchronize()
    Xb = oracle.unpack_bits(g.to_host(X), nrhs)
    badbits = oracle.unpack_bits(g.to_host(bad)[None, :], nrhs)[0]
    for t in range(nrhs):
        want = oracle.solve_from_pls(cols[:, t], m, n, r, P, Q, Ap)
        if want is None:
            assert badbits[t] == 1, f"rhs {t}: inconsistent system not flagged"
        else:
            assert badbits[t] == 0, f"rhs {t}: consistent system flagged"
            assert np.array_equal(Xb[:, t], want), f"rhs {t}: solution differs"
    # padding bits past nrhs stay zero
    if nrhs % 64:
        assert not np.any(g.to_host(X)[:, -1] >> np.uint64(nrhs % 64))


def test_solve_padded_strides():
    m, n, nrhs = 900, 800, 70
    A = make_input("planted600", m, n, 77)
    Bp, cols = rhs_block(A, m, n, nrhs, 78, stride=5)
    r, P, Q, Ap = oracle.pls(A, m, n)
    dA, dP, dQ, drank = gpu_pls(A, m, n)
    Xd = torch.full((n, 4), -1, dtype=torch.int64, device="cuda")
    X, bad = g.solve(dA, m, n, dP, dQ, drank, g.to_device(Bp), nrhs, X=Xd)
    torch.cuda.synchronize()
    Xh = g.to_host(X)
    assert not np.any(Xh[:, 2:]), "padding words of X must be zeroed"
    Xb = oracle.unpack_bits(Xh, nrhs)
    badbits = oracle.unpack_bits(g.to_host(bad)[None, :], nrhs)[0]
    for t in range(nrhs):
        want = oracle.solve_from_pls(cols[:, t], m, n, r, P, Q, Ap)
        assert (want is None) == bool(badbits[t])
        if want is not None:
            assert np.array_equal(Xb[:, t], want)


KERNEL_CASES = [
    (1, 1, "zero"), (1, 5, "half"), (5, 1, "half"), (64, 130, "half"), (200, 200, "zero"),
    (300, 300, "identity"), (500, 700, "half"), (900, 900, "planted700"), (700, 1300, "sparse"),
    (1500, 1500, "planted1000"), (1200, 3000, "half"),
]


@pytest.mark.parametrize("m,n,kind", KERNEL_CASES)
@pytest.mark.parametrize("variant", [g.SCHUR_FP4, g.SCHUR_XOR])
def test_kernel_basis_matches_oracle(m, n, kind, variant):
    A = make_input(kind, m, n, 900 + m + n)
    r, P, Q, Ap = oracle.pls(A, m, n)
    say(f"[kernel] {kind} {m}x{n} rank {r} variant {variant}")
    want = oracle.kernel_basis(m, n, r, Q, Ap)
    dA, dP, dQ, drank = gpu_pls(A, m, n)
    K = g.kernel_basis(dA, m, n, dQ, drank, s=g.Sched(8, 8, 512, variant))
    torch.cuda.synchronize()
    Kb = oracle.unpack_bits(g.to_host(K), n)
    assert np.array_equal(Kb[:n - r], want), "basis differs"
    assert not np.any(Kb[n - r:]), "rows past the nullity must be zero"


@pytest.mark.slow
def test_solve_full_size_by_properties():
    m = n = 65536
    nrhs = 64
    A = synth.random_half(m, n, 1)
    rng = np.random.default_rng(3)
    # 64 right-hand sides B = A Xr for random Xr (consistent), packed one word a row
    Xr = rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)
    B = oracle.mul64(A, m, n // 64, Xr)
    say("[solve] 65536^2 p=1/2: PLS then 64 right-hand sides")
    dA, dP, dQ, drank = gpu_pls(A, m, n)
    X, bad = g.solve(dA, m, n, dP, dQ, drank, g.to_device(B[:, None]), nrhs)
    torch.cuda.synchronize()
    r = int(drank.item())
    Xh = g.to_host(X)[:, 0].copy()
    assert int(g.to_host(bad)[0]) == 0
    if r == n:
        # full rank: the solution is unique, so it is Xr itself
        assert np.array_equal(Xh, Xr)
    # A X = B exactly
    assert np.array_equal(oracle.mul64(A, m, n // 64, Xh), B)


@pytest.mark.slow
def test_kernel_basis_full_size_by_properties():
    m = n = 32768
    A = synth.planted(m, n, 24576, 4, p=0.5, unit=False)
    say("[kernel] 32768^2 planted rank 24576")
    dA, dP, dQ, drank = gpu_pls(A, m, n)
    K = g.kernel_basis(dA, m, n, dQ, drank)
    torch.cuda.synchronize()
    r = int(drank.item())
    assert r == 24576
    Q = dQ.cpu().numpy()
    Kh = g.to_host(K)
    assert not np.any(Kh[n - r:])
    basis = Kh[:n - r]
    # non-pivot coordinates: row j has exactly the j-th non-pivot column among them
    piv = np.zeros(n, dtype=bool)
    piv[Q[:r]] = True
    free = np.flatnonzero(~piv)
    Kfree = oracle.unpack_bits(basis, n)[:, free]
    assert np.array_equal(Kfree, np.eye(n - r, dtype=np.uint8))
    # A v = 0 for 64 random combinations v of the basis rows (a nonzero A K^T
    # survives each with probability at most 1/2)
    combos = rng_combos(basis, 64, seed=11)
    V = np.zeros(n, dtype=np.uint64)
    for t, v in enumerate(combos):
        bits = oracle.unpack_bits(v[None, :], n)[0].astype(np.uint64)
        V |= bits << np.uint64(t)
    assert not np.any(oracle.mul64(A, m, n // 64, V))


def rng_combos(rows, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        sel = rng.integers(0, 2, size=rows.shape[0]).astype(bool)
        out.append(np.bitwise_xor.reduce(rows[sel], axis=0) if sel.any()
                   else np.zeros(rows.shape[1], np.uint64))
    return out

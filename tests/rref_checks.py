"""Checks that pin a reduced row echelon form at any size without forming it on
the host (test helper; used by the full-size GPU tests and checked on the CPU in
test_rref_checks.py).

With S the echelon rows of a PLS (pivot i at column Q[i]) and U = S[:, Q], the
RREF R is the unique matrix with rows past the rank zero, R[:, Q] = I and
S = U R (Definition "Reduced Row Echelon Form", Section 2).  The two identities
are tested by Freivalds' method (Freivalds 1977) with 64 random vectors each, so
a wrong R passes with probability at most 2^-64."""
from __future__ import annotations

import numpy as np

import oracle


def s_rows(Ap: np.ndarray, r: int, Q: np.ndarray, n: int) -> np.ndarray:
    """S (r x n, packed) from the in-place result: stored bits right of Q[i], one at Q[i]."""
    W = (n + 63) // 64
    S = np.ascontiguousarray(Ap[:r, :W]).copy()
    if r == 0:
        return S
    q = Q[:r].astype(np.int64)
    cols = np.arange(W, dtype=np.int64)[None, :]
    w = (q // 64)[:, None]
    S[cols < w] = 0
    lo = (q % 64).astype(np.uint64)
    # bits at or below the pivot in its word are cleared (all of them when lo == 63)
    low = np.where(lo == 63, ~np.uint64(0),
                   np.left_shift(np.uint64(1), np.minimum(lo + np.uint64(1), np.uint64(63))) - np.uint64(1))
    idx = np.arange(r)
    S[idx, q // 64] = (S[idx, q // 64] & ~low) | np.left_shift(np.uint64(1), lo)
    return S


def _spread(Y: np.ndarray, Q: np.ndarray, W: int) -> np.ndarray:
    """Vectors z with z[Q[j]] = y[j], zero elsewhere, 64 at a time (bit t of each word)."""
    Z = np.zeros(64 * W, dtype=np.uint64)
    Z[Q.astype(np.int64)] = Y
    return Z


def rref_violations(R: np.ndarray, S: np.ndarray, r: int, Q: np.ndarray, n: int,
                    seed: int = 99) -> list[str]:
    """The identities R fails (empty when it is the RREF, up to probability 2^-64)."""
    W = (n + 63) // 64
    bad = []
    if R[r:, :W].any():
        bad.append("rows past the rank are not zero")
    if r == 0:
        return bad
    rng = np.random.default_rng(seed)
    q = Q[:r]
    # R[:, Q] = I:  R z(y) = y for 64 random r-vectors y
    Y = rng.integers(0, np.iinfo(np.uint64).max, r, dtype=np.uint64, endpoint=True)
    if not np.array_equal(oracle.mul64(R, r, W, _spread(Y, q, W)), Y):
        bad.append("R[:, Q] != I")
    # S = U R:  S v = S z(R v) for 64 random n-vectors v
    V = rng.integers(0, np.iinfo(np.uint64).max, 64 * W, dtype=np.uint64, endpoint=True)
    V[n:] = 0
    RV = oracle.mul64(R, r, W, V)
    if not np.array_equal(oracle.mul64(S, r, W, V), oracle.mul64(S, r, W, _spread(RV, q, W))):
        bad.append("S != U_Q R")
    return bad


def check_rref_properties(R, S, r, Q, n):
    bad = rref_violations(R, S, r, Q, n)
    assert not bad, "; ".join(bad)

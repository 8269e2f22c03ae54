"""CPU oracle for PLS / RREF over GF(2).  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU path (``paper_1006_1744_amd``)
never imports it, and the two share no code; only the seeded input generator
(``synth``), which holds none of the method's arithmetic, serves both.

Contents
* ``pls(A, m, n)``   -- Gaussian PLS, Appendix A of Albrecht & Pernet (C, gcc,
  OpenMP over the rows one pivot updates).  The unique result the MMPF and the
  recursive PLS must reproduce bit for bit: rank r, transposition vectors P and
  Q, and the in-place matrix (L below the diagonal, S on and above it, after the
  "compress L" column swaps).
* ``rref(A, m, n)``  -- Gauss-Jordan reduction (Definition of the reduced row
  echelon form, Section 2), written independently of ``pls``.
* checkers: unpacking L and S from the in-place result, applying P,
  reconstruction A = P L S, echelon-form checks, Freivalds' randomized product
  check (Freivalds 1977).
* ``solve_from_pls`` / ``kernel_basis``: A x = b and a basis of the null space
  from the PLS (forward substitution with L, back substitution with S).
* ``pyref``: pure-Python statements of the paper's algorithms for tiny inputs.

Parity status: every function here is pinned by tests in
``tests/test_oracle_pins.py`` (brute force on tiny inputs, the Figure 1 table,
the Section 4.1 "[1 0 1]" example, reconstruction, rank(A) = rank(A^T),
planted ranks, agreement of independent statements of the algorithm); the
solving functions by ``tests/test_oracle_solve.py`` (brute force over every x
on tiny systems, consistency, null-space dimension and independence).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import pyref  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gf2_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.oracle_pls.restype = i64
        lib.oracle_pls.argtypes = [p, i64, i64, i64, p, p]
        lib.oracle_rref.restype = i64
        lib.oracle_rref.argtypes = [p, i64, i64, i64, p]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        lib.oracle_mul64.restype = None
        lib.oracle_mul64.argtypes = [p, i64, i64, i64, p, p]
        _lib = lib
    return _lib


def threads() -> int:
    return int(_load().oracle_threads())


def _check(A: np.ndarray, m: int, n: int) -> None:
    if A.dtype != np.uint64 or A.ndim != 2 or A.shape[0] != m:
        raise ValueError("A must be uint64 of shape (m, stride)")
    if A.shape[1] < (n + 63) // 64:
        raise ValueError("stride too small")


def pls(A: np.ndarray, m: int, n: int):
    """Gaussian PLS of a copy of A.  Returns (r, P[int32 m], Q[int32 n], A')."""
    _check(A, m, n)
    a = np.ascontiguousarray(A.copy())
    P = np.arange(m, dtype=np.int32)
    Q = np.arange(n, dtype=np.int32)
    if m == 0 or n == 0:
        return 0, P, Q, a
    r = _load().oracle_pls(a.ctypes.data, m, n, a.shape[1], P.ctypes.data, Q.ctypes.data)
    return int(r), P, Q, a


def rref(A: np.ndarray, m: int, n: int):
    """Gauss-Jordan RREF of a copy of A.  Returns (r, R, pivot_columns[int32 r])."""
    _check(A, m, n)
    a = np.ascontiguousarray(A.copy())
    piv = np.zeros(max(min(m, n), 1), dtype=np.int32)
    if m == 0 or n == 0:
        return 0, a, piv[:0]
    r = _load().oracle_rref(a.ctypes.data, m, n, a.shape[1], piv.ctypes.data)
    return int(r), a, piv[:r].copy()


def mul64(M: np.ndarray, rows: int, W: int, V: np.ndarray) -> np.ndarray:
    """64 GF(2) matrix-vector products at once (checker for Freivalds' test):
    bit t of out[i] = parity of popcount(M[i, :W] AND v_t), with bit t of V[j]
    entry j of v_t (V: uint64[64 W])."""
    if M.dtype != np.uint64 or M.ndim != 2 or M.shape[0] < rows or M.shape[1] < W:
        raise ValueError("M must be uint64 (>= rows, >= W)")
    V = np.ascontiguousarray(V, dtype=np.uint64)
    if V.shape[0] < 64 * W:
        raise ValueError("V needs 64 W entries")
    M = np.ascontiguousarray(M)
    out = np.zeros(max(rows, 1), dtype=np.uint64)
    if rows > 0:
        _load().oracle_mul64(M.ctypes.data, rows, W, M.shape[1], V.ctypes.data, out.ctypes.data)
    return out[:rows]


# ---------------------------------------------------------------- conversions
def to_rows(A: np.ndarray, n: int) -> list[int]:
    """numpy packed rows -> list of Python ints (column j = bit j)."""
    out = []
    w = (n + 63) // 64
    for i in range(A.shape[0]):
        v = 0
        for k in range(w - 1, -1, -1):
            v = (v << 64) | int(A[i, k])
        out.append(v)
    return out


def from_rows(rows: list[int], n: int, stride: int | None = None) -> np.ndarray:
    w = (n + 63) // 64
    stride = w if stride is None else stride
    a = np.zeros((len(rows), stride), dtype=np.uint64)
    for i, v in enumerate(rows):
        for k in range(w):
            a[i, k] = (v >> (64 * k)) & 0xFFFFFFFFFFFFFFFF
    return a


def unpack_bits(A: np.ndarray, n: int) -> np.ndarray:
    """(m, stride) uint64 -> (m, n) uint8 of 0/1."""
    m = A.shape[0]
    if m == 0 or n == 0:
        return np.zeros((m, n), dtype=np.uint8)
    b = np.unpackbits(np.ascontiguousarray(A).view(np.uint8), axis=1, bitorder="little")
    return b[:, :n].copy()


def pack_bits(B: np.ndarray, stride: int | None = None) -> np.ndarray:
    """(m, n) 0/1 -> (m, stride) uint64."""
    m, n = B.shape
    w = (n + 63) // 64
    stride = w if stride is None else stride
    out = np.zeros((m, stride), dtype=np.uint64)
    if m == 0 or n == 0:
        return out
    padded = np.zeros((m, w * 64), dtype=np.uint8)
    padded[:, :n] = B & 1
    packed = np.packbits(padded, axis=1, bitorder="little").view(np.uint64)
    out[:, :w] = packed
    return out


# ------------------------------------------------------------------- checkers
def unpack_LS(Ap: np.ndarray, m: int, n: int, r: int, Q: np.ndarray):
    """From the compressed in-place result: L (m x r, unit lower trapezoidal) and
    S (r x n, S[i, Q[i]] = 1, zero left of it, the stored bits right of it)."""
    B = unpack_bits(Ap, n)
    L = np.zeros((m, r), dtype=np.uint8)
    S = np.zeros((r, n), dtype=np.uint8)
    for i in range(m):
        k = min(i, r)
        L[i, :k] = B[i, :k]
        if i < r:
            L[i, i] = 1
    for i in range(r):
        q = int(Q[i])
        S[i, q] = 1
        S[i, q + 1:] = B[i, q + 1:]
    return L, S


def apply_P(A_bits: np.ndarray, P: np.ndarray) -> np.ndarray:
    """Row i swapped with row P[i], for i = 0, 1, ... in order (on a 0/1 array)."""
    X = A_bits.copy()
    for i in range(X.shape[0]):
        p = int(P[i])
        if p != i:
            X[[i, p]] = X[[p, i]]
    return X


def gf2_matmul_bits(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Plain product of 0/1 matrices reduced mod 2 (int64 accumulation)."""
    if X.shape[1] == 0:
        return np.zeros((X.shape[0], Y.shape[1]), dtype=np.uint8)
    return ((X.astype(np.int64) @ Y.astype(np.int64)) & 1).astype(np.uint8)


def reconstruct_ok(A: np.ndarray, m: int, n: int, r: int, P, Q, Ap) -> bool:
    """A with rows permuted by P equals L*S exactly (small sizes)."""
    L, S = unpack_LS(Ap, m, n, r, Q)
    lhs = apply_P(unpack_bits(A, n), P)
    return bool(np.array_equal(lhs, gf2_matmul_bits(L, S)))


def is_row_echelon(S: np.ndarray, Q: np.ndarray) -> bool:
    """Leading one of row i at Q[i], strictly increasing."""
    r = S.shape[0]
    last = -1
    for i in range(r):
        nz = np.flatnonzero(S[i])
        if nz.size == 0 or nz[0] != Q[i] or nz[0] <= last:
            return False
        last = nz[0]
    return True


def is_rref(R_bits: np.ndarray, r: int) -> bool:
    """Rows < r in echelon form with each leading one alone in its column; rows >= r zero."""
    m = R_bits.shape[0]
    if np.any(R_bits[r:]):
        return False
    last = -1
    for i in range(r):
        nz = np.flatnonzero(R_bits[i])
        if nz.size == 0 or nz[0] <= last:
            return False
        last = nz[0]
        if R_bits[:, last].sum() != 1:
            return False
    return True


def freivalds(A: np.ndarray, m: int, n: int, r: int, P, Q, Ap, trials: int = 64,
              seed: int = 12345) -> bool:
    """Randomized check of (P applied to A) = L S, Freivalds (1977): both sides are
    multiplied by `trials` random 0/1 vectors; a wrong factorisation passes with
    probability <= 2^-trials.  Works on packed rows (np.bitwise_count), so it runs
    at sizes where L and S cannot be formed as byte matrices."""
    rng = np.random.default_rng(seed)
    W = (n + 63) // 64
    Wr = (r + 63) // 64
    order = np.arange(m)
    for i in range(m):
        p = int(P[i])
        if p != i:
            order[[i, p]] = order[[p, i]]
    Aperm = np.ascontiguousarray(A[order, :W])
    # S rows: stored bits right of Q[i], a one at Q[i], zeros left of it
    Sp = np.ascontiguousarray(Ap[:r, :W].copy())
    for i in range(r):
        q = int(Q[i])
        w, lo = q // 64, q % 64
        Sp[i, :w] = 0
        keep = ((1 << 64) - 1) ^ ((1 << (lo + 1)) - 1)
        Sp[i, w] = np.uint64((int(Sp[i, w]) & keep) | (1 << lo))
    # L rows: bits < min(i, r) of the stored row, plus the unit diagonal
    Lp = np.zeros((m, max(Wr, 1)), dtype=np.uint64)
    if r:
        Lp[:, :Wr] = Ap[:, :Wr]
        if r % 64:
            Lp[:, Wr - 1] &= np.uint64((1 << (r % 64)) - 1)
        for i in range(min(r, m)):
            w, lo = i // 64, i % 64
            Lp[i, w + 1:] = 0
            Lp[i, w] = np.uint64((int(Lp[i, w]) & ((1 << lo) - 1)) | (1 << lo))

    def parity(M: np.ndarray, x: np.ndarray) -> np.ndarray:
        return (np.bitwise_count(M & x[None, :]).sum(axis=1) & 1).astype(np.uint8)

    for _ in range(trials):
        x = rng.integers(0, np.iinfo(np.uint64).max, size=W, dtype=np.uint64, endpoint=True)
        if n % 64:
            x[W - 1] &= np.uint64((1 << (n % 64)) - 1)
        lhs = parity(Aperm, x) if W else np.zeros(m, np.uint8)
        if r:
            y = parity(Sp, x)
            ypk = pack_bits(y[None, :])[0]
            rhs = parity(Lp[:, :Wr], ypk[:Wr])
        else:
            rhs = np.zeros(m, np.uint8)
        if not np.array_equal(lhs, rhs):
            return False
    return True


# ---------------------------------------------------------------- solving
# The decomposition as the building block for solving linear systems over GF(2)
# (the abstract and Section 1): with P A = L S, a system A x = b becomes
# L S x = P b, one forward substitution with L's unit lower triangle, a
# consistency test on L's remaining rows, and one back substitution with the
# echelon rows of S.  Written out on 0/1 arrays, for test sizes.

def solve_from_pls(b: np.ndarray, m: int, n: int, r: int, P, Q, Ap):
    """A solution x (0/1, length n, non-pivot entries 0) of A x = b, from A's PLS
    (r, P, Q, A' as returned by ``pls``); None if the system is inconsistent.
    b: 0/1 vector of length m."""
    L, S = unpack_LS(Ap, m, n, r, Q)
    c = apply_P(np.asarray(b, dtype=np.uint8).reshape(m, 1), P).reshape(m)
    # L y = c on the first r rows (unit lower triangle)
    y = np.zeros(r, dtype=np.uint8)
    for i in range(r):
        y[i] = c[i] ^ (int(L[i, :i].astype(np.int64) @ y[:i].astype(np.int64)) & 1)
    # the remaining rows of L y must reproduce the remaining entries of c
    if r < m:
        rest = (L[r:].astype(np.int64) @ y.astype(np.int64)) & 1
        if not np.array_equal(rest.astype(np.uint8), c[r:]):
            return None
    # S x = y: pivot columns Q[0] < Q[1] < ... from the last row up, others 0
    x = np.zeros(n, dtype=np.uint8)
    for i in range(r - 1, -1, -1):
        q = int(Q[i])
        x[q] = y[i] ^ (int(S[i, q + 1:].astype(np.int64) @ x[q + 1:].astype(np.int64)) & 1)
    return x


def kernel_basis(m: int, n: int, r: int, Q, Ap) -> np.ndarray:
    """A basis of {x : A x = 0} as the rows of an (n - r) x n 0/1 array, one per
    non-pivot column f: x[f] = 1, the other non-pivot entries 0, the pivot entries
    from S x = 0 (L and P are invertible on the rows that matter, so A x = 0
    exactly when S x = 0)."""
    _, S = unpack_LS(Ap, m, n, r, Q)
    piv = {int(q) for q in Q[:r]}
    basis = []
    for f in range(n):
        if f in piv:
            continue
        x = np.zeros(n, dtype=np.uint8)
        x[f] = 1
        for i in range(r - 1, -1, -1):
            q = int(Q[i])
            x[q] = int(S[i, q + 1:].astype(np.int64) @ x[q + 1:].astype(np.int64)) & 1
        basis.append(x)
    return np.array(basis, dtype=np.uint8).reshape(len(basis), n)

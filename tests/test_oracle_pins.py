"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

None of these tests needs a GPU.  Each pin is chosen so that a plausible mistake
in the oracle fails it; ``test_planted_mistakes_are_caught`` rebuilds the oracle
with such mistakes planted and checks exactly that.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from oracle import pyref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------- brute force
def brute_rank(rows: list[int]) -> int:
    """log2 of the size of the row space, by enumerating every combination."""
    span = {0}
    for x in rows:
        span |= {s ^ x for s in span}
    return len(span).bit_length() - 1


def brute_profile(rows: list[int], n: int) -> list[int]:
    """Column rank profile: Q[t] = first j with rank(A[:, :j+1]) = t + 1."""
    prof = []
    last = 0
    for j in range(n):
        msk = (1 << (j + 1)) - 1
        rk = brute_rank([x & msk for x in rows])
        if rk > last:
            prof.append(j)
            last = rk
    return prof


def check_pls_contract(A: np.ndarray, m: int, n: int, res, rows=None) -> None:
    r, P, Q, Ap = res
    assert 0 <= r <= min(m, n)
    assert oracle.reconstruct_ok(A, m, n, r, P, Q, Ap)
    L, S = oracle.unpack_LS(Ap, m, n, r, Q)
    assert oracle.is_row_echelon(S, Q[:r])
    for i in range(r):
        assert i <= P[i] < m
    assert list(P[r:]) == list(range(r, m))
    assert list(Q[r:]) == list(range(r, n))
    # in-place layout after compressing L: row i < r has a one at column i and
    # zeros on (i, Q[i]]; rows >= r are zero from column r on
    B = oracle.unpack_bits(Ap, n)
    for i in range(r):
        assert B[i, i] == 1
        assert not B[i, i + 1:Q[i] + 1].any()
    assert not B[r:, r:].any()
    if rows is not None:
        assert r == brute_rank(rows)
        assert list(Q[:r]) == brute_profile(rows, n)


# ------------------------------------------------------- Figure 1 and MakeTable1
def _parse_bits(s: str) -> int:
    s = s.replace("|", "").strip()
    return sum(int(ch) << j for j, ch in enumerate(s))


def _golden_sections(name):
    sec, out = None, {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                sec = line.strip("[]")
                out[sec] = []
            else:
                out[sec].append(line)
    return out


def test_figure1_make_table():
    """Section 3.1, Figure 1: the table of all 2^3 combinations of the three
    reduced rows, listed by the id read MSB-first from the strip."""
    g = _golden_sections("figure1_m4ri_table.txt")
    U = [_parse_bits(s) for s in g["U"]]
    T_printed = [_parse_bits(s) for s in g["T"]]
    T, L = pyref.make_table(U, 0, 0, 3)
    assert [T[L[i]] for i in range(8)] == T_printed
    for line in g["CLEAR"]:
        before, after = (x.strip() for x in line.split("->"))
        rows = [_parse_bits(before)]
        pyref.add_rows_from_table(rows, 0, 1, 0, 3, T, L)
        assert rows[0] == _parse_bits(after)
    # 2^k - 1 additions build the table (Section 3.1): T holds the whole span
    assert sorted(T) == sorted({a ^ b ^ c for a in (0, U[0]) for b in (0, U[1])
                                for c in (0, U[2])})


def test_make_table1_fix_101_example():
    """Section 4.1, "Preserving L": with kbar = 3 and the first U row starting
    [1 0 1], a row starting [1 0 1] is cleared by that row alone, so its strip
    must read [1 0 0] afterwards (the multipliers of the U rows)."""
    U = [_parse_bits("101|1101"), _parse_bits("011|0110"), _parse_bits("001|1011")]
    T, L = pyref.make_table1(U, 0, 3)
    x = _parse_bits("101|0000")
    rows = [x]
    pyref.add_rows_from_table(rows, 0, 1, 0, 3, T, L)
    assert rows[0] & 0b111 == _parse_bits("100")
    assert rows[0] >> 3 == (x ^ U[0]) >> 3
    # every strip pattern is cleared into its multipliers, rest reduced
    for strip in range(8):
        y = 0
        for j in range(3):
            y |= ((strip >> (2 - j)) & 1) << j
        rows = [y | (0b1010 << 3)]
        pyref.add_rows_from_table(rows, 0, 1, 0, 3, T, L)
        mult = [(rows[0] >> j) & 1 for j in range(3)]
        comb = 0
        for j in range(3):
            if mult[j]:
                comb ^= U[j]
        assert (comb & 0b111) == y
        assert rows[0] >> 3 == ((0b1010 << 3) ^ comb) >> 3


# -------------------------------------------------------------- exhaustive
@pytest.mark.parametrize("m,n", [(1, 8), (8, 1), (2, 6), (6, 2), (3, 4), (4, 3)])
def test_exhaustive_tiny(m, n):
    """Every m x n matrix with m*n <= 12: rank and column profile by brute force,
    reconstruction A = P L S, echelon form, transposition form, layout."""
    for bits in range(1 << (m * n)):
        rows = [(bits >> (i * n)) & ((1 << n) - 1) for i in range(m)]
        A = oracle.from_rows(rows, n)
        check_pls_contract(A, m, n, oracle.pls(A, m, n), rows)


def test_random_4x4_to_8x8_brute():
    rng = np.random.default_rng(3)
    for _ in range(400):
        m, n = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        rows = [int(rng.integers(0, 1 << n)) for _ in range(m)]
        A = oracle.from_rows(rows, n)
        check_pls_contract(A, m, n, oracle.pls(A, m, n), rows)


# ---------------------------------------------- independent statements agree
def _inputs_small(count, seed):
    rng = np.random.default_rng(seed)
    for t in range(count):
        m, n = int(rng.integers(1, 41)), int(rng.integers(1, 41))
        kind = t % 4
        if kind == 0:
            A = synth.random_half(m, n, 1000 + t)
        elif kind == 1:
            A = synth.random_bernoulli(m, n, 0.1, 1000 + t)
        elif kind == 2:
            A = synth.planted(m, n, int(rng.integers(0, min(m, n) + 1)), 1000 + t)
        else:
            A = synth.random_bernoulli(m, n, 0.03, 1000 + t)
        yield m, n, A


def test_c_oracle_matches_paper_statements():
    """The C oracle, the literal Gaussian PLS, MMPF (k = 1..8) and the recursive
    PLS (Section 5) reach the same (r, P, Q, A') -- this pins P, which only the
    pivot rule fixes."""
    for m, n, A in _inputs_small(160, 7):
        r, P, Q, Ap = oracle.pls(A, m, n)
        check_pls_contract(A, m, n, (r, P, Q, Ap))
        rows = oracle.to_rows(A, n)
        want = (r, list(P), list(Q), oracle.to_rows(Ap, n))
        got = pyref.gaussian_pls(rows, m, n)
        assert (got[0], got[1], got[2], got[3]) == want
        for k in (1, 3, 8):
            got = pyref.mmpf(rows, m, n, k)
            assert (got[0], got[1], got[2], got[3]) == want
        for base in (1, 4):
            got = pyref.pls_recursive(rows, m, n, base)
            assert (got[0], got[1], got[2], got[3]) == want


def test_rank_of_transpose():
    rng = np.random.default_rng(11)
    for t in range(30):
        m, n = int(rng.integers(1, 150)), int(rng.integers(1, 200))
        A = synth.planted(m, n, int(rng.integers(0, min(m, n) + 1)), 77 + t, unit=True)
        At = oracle.pack_bits(oracle.unpack_bits(A, n).T.copy())
        assert oracle.pls(A, m, n)[0] == oracle.pls(At, n, m)[0]


def test_planted_rank_exact():
    for (m, n, r, p) in [(50, 70, 20, 0.5), (64, 64, 64, 0.5), (100, 40, 40, 0.1),
                         (300, 500, 123, 0.01), (129, 65, 1, 0.5), (10, 10, 0, 0.5)]:
        A = synth.planted(m, n, r, 5, p=p, unit=True)
        assert oracle.pls(A, m, n)[0] == r


# ---------------------------------------------------------------------- RREF
def test_rref_oracle():
    """RREF is unique (Definition, Section 2): Gauss-Jordan (C) equals M4RI
    (Section 3.1) and Python Gauss-Jordan; its rank and pivots equal the PLS
    rank and column profile; rank([A; R]) = rank(A)."""
    for m, n, A in _inputs_small(80, 19):
        r, R, piv = oracle.rref(A, m, n)
        rp, P, Q, _ = oracle.pls(A, m, n)
        assert r == rp and list(piv) == list(Q[:r])
        assert oracle.is_rref(oracle.unpack_bits(R, n), r)
        rows = oracle.to_rows(A, n)
        for k in (1, 2, 5):
            r4, rows4 = pyref.m4ri(rows, m, n, k)
            assert r4 == r and rows4 == oracle.to_rows(R, n)
        rg, rowsg, pivg = pyref.gauss_jordan(rows, m, n)
        assert rowsg == oracle.to_rows(R, n)
        stacked = np.vstack([A, R])
        assert oracle.pls(stacked, 2 * m, n)[0] == r


# ------------------------------------------------------------- special cases
def test_special_cases():
    m, n = 70, 130
    Z = synth.empty(m, n)
    r, P, Q, Ap = oracle.pls(Z, m, n)
    assert r == 0 and not Ap.any()
    assert list(P) == list(range(m)) and list(Q) == list(range(n))
    I = oracle.pack_bits(np.eye(m, n, dtype=np.uint8))
    r, P, Q, Ap = oracle.pls(I, m, n)
    assert r == m and np.array_equal(Ap, I)
    ones = oracle.pack_bits(np.ones((m, n), dtype=np.uint8))
    r, P, Q, Ap = oracle.pls(ones, m, n)
    assert r == 1
    B = oracle.unpack_bits(Ap, n)
    assert (B[:, 0] == 1).all() and B[0, 1:].all() and not B[1:, 1:].any()
    # pivot only in the last row, first columns zero
    X = np.zeros((m, n), dtype=np.uint8)
    X[m - 1, 5] = 1
    X[m - 1, 9] = 1
    A = oracle.pack_bits(X)
    r, P, Q, Ap = oracle.pls(A, m, n)
    assert r == 1 and P[0] == m - 1 and Q[0] == 5
    check_pls_contract(A, m, n, (r, P, Q, Ap))
    # one row, one column
    for (mm, nn) in [(1, 100), (100, 1), (1, 1)]:
        A = synth.random_half(mm, nn, 4)
        check_pls_contract(A, mm, nn, oracle.pls(A, mm, nn), oracle.to_rows(A, nn)
                           if mm * nn <= 16 else None)


def test_padding_and_stride():
    m, n = 37, 100
    A = synth.random_half(m, n, 9, stride=5)
    r, P, Q, Ap = oracle.pls(A, m, n)
    assert not Ap[:, 2:].any()                      # padding words stay zero
    assert not (Ap[:, 1] >> np.uint64(36)).any()    # bits past column n stay zero
    r2, P2, Q2, Ap2 = oracle.pls(np.ascontiguousarray(A[:, :2]), m, n)
    assert r == r2 and np.array_equal(Ap[:, :2], Ap2)


# ---------------------------------------------------------------- Freivalds
def test_freivalds_matches_exact_and_detects_errors():
    for (m, n) in [(300, 500), (513, 257)]:
        A = synth.random_half(m, n, 21)
        r, P, Q, Ap = oracle.pls(A, m, n)
        assert oracle.reconstruct_ok(A, m, n, r, P, Q, Ap)
        assert oracle.freivalds(A, m, n, r, P, Q, Ap)
        bad = Ap.copy()
        bad[m // 2, 3] ^= np.uint64(1 << 7)
        assert not oracle.reconstruct_ok(A, m, n, r, P, Q, bad)
        assert not oracle.freivalds(A, m, n, r, P, Q, bad)


@pytest.mark.slow
def test_oracle_medium_freivalds():
    m = n = 2048
    A = synth.random_bernoulli(m, n, 0.01, 3)
    r, P, Q, Ap = oracle.pls(A, m, n)
    assert oracle.freivalds(A, m, n, r, P, Q, Ap, trials=32)


# ------------------------------------------------------- planted mistakes
def _pin_battery(pls_fn) -> bool:
    """True iff the PLS function passes the pins above on a fixed input set."""
    try:
        for bits in range(1 << 12):
            m, n = 3, 4
            rows = [(bits >> (i * n)) & 15 for i in range(m)]
            A = oracle.from_rows(rows, n)
            check_pls_contract(A, m, n, pls_fn(A, m, n), rows)
        for m, n, A in _inputs_small(40, 5):
            res = pls_fn(A, m, n)
            check_pls_contract(A, m, n, res)
            got = pyref.gaussian_pls(oracle.to_rows(A, n), m, n)
            if (got[0], got[1], got[2], got[3]) != (res[0], list(res[1]), list(res[2]),
                                                    oracle.to_rows(res[3], n)):
                return False
    except AssertionError:
        return False
    return True


def _variant(path):
    lib = ctypes.CDLL(path)
    lib.oracle_pls.restype = ctypes.c_int64
    lib.oracle_pls.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                               ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]

    def fn(A, m, n):
        a = A.copy()
        P = np.arange(m, dtype=np.int32)
        Q = np.arange(n, dtype=np.int32)
        r = lib.oracle_pls(a.ctypes.data, m, n, a.shape[1], P.ctypes.data, Q.ctypes.data)
        return int(r), P, Q, a
    return fn


def test_planted_mistakes_are_caught(tmp_path):
    src = os.path.join(os.path.dirname(oracle.__file__), "gf2_oracle.c")
    assert _pin_battery(oracle.pls)
    for k in range(1, 6):
        so = str(tmp_path / f"mut{k}.so")
        subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", "-std=c99",
                               f"-DORACLE_MUTATION={k}", src, "-o", so])
        assert not _pin_battery(_variant(so)), f"mutation {k} not caught"


def test_brute_force_helpers():
    assert brute_rank([1, 2, 4, 8]) == 4
    assert brute_rank([3, 3, 0]) == 1
    assert brute_rank([]) == 0
    assert brute_profile([0b0110, 0b0100], 4) == [1, 2]

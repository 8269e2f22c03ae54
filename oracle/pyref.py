"""Pure-Python statements of the paper's algorithms, for tiny inputs.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Rows are Python ints: column ``j`` is bit ``j``.  Every function follows the
algorithm it names in Albrecht & Pernet, "Efficient Decomposition of Dense
Matrices over GF(2)", in the paper's order of steps and notation, written from
its description rather than copied from the printed pseudo-code:

* ``gaussian_pls``        -- Appendix A, "Gaussian PLS Decomposition".
* ``pls_submatrix``       -- Appendix A, "PlsSubmatrix".
* ``make_table1``         -- Section 4.1, "MakeTable1" (Gray-code table, the
                             translation array L and the a-priori-id fix).
* ``add_rows_from_table`` -- Appendix A, "AddRowsFromTable".
* ``mmpf``                -- Section 4.1, "MMPF".
* ``make_table``          -- Appendix A, "MakeTable" (the M4RI table, no fix).
* ``gauss_submatrix``     -- Appendix A, "GaussSubmatrix".
* ``m4ri``                -- Section 3.1, "M4RI" (reduced row echelon form).
* ``pls_recursive``       -- Section 5, "PLS Decomposition" (asymptotically fast
                             recursion with a Gaussian base case).

Readings where the printed text is ambiguous (all documented with the design):
indices are 0-based and ranges half-open; the table index reads the k bits
starting at column c with column c as the most significant bit (the "0 1 1 -> 3"
example of Section 3.1); the k-th Gray code is g(i) = i ^ (i >> 1), its bit b
selecting row k-1-b of the k source rows; "the a-priori id" of table row i is
g(i).
"""
from __future__ import annotations


def bit(x: int, j: int) -> int:
    return (x >> j) & 1


def mask_from(c: int) -> int:
    """All columns >= c (as an int with unbounded high bits, masked later)."""
    return ~((1 << c) - 1)


def add_row_from(rows: list[int], dst: int, src: int, c: int) -> None:
    """row dst += row src, starting at column c."""
    rows[dst] ^= rows[src] & mask_from(c)


def swap_rows(rows: list[int], a: int, b: int) -> None:
    rows[a], rows[b] = rows[b], rows[a]


def swap_cols_from(rows: list[int], a: int, b: int, start: int) -> None:
    """Swap columns a and b in rows start..end."""
    if a == b:
        return
    for i in range(start, len(rows)):
        x = rows[i]
        if bit(x, a) != bit(x, b):
            rows[i] = x ^ (1 << a) ^ (1 << b)


def compress_l(rows: list[int], Q: list[int], r: int) -> None:
    """Swap columns j and Q[j] starting at row j, for j < r."""
    for j in range(r):
        swap_cols_from(rows, j, Q[j], j)


# ---------------------------------------------------------------- Gaussian PLS
def gaussian_pls(rows_in: list[int], m: int, n: int):
    """Appendix A, "Gaussian PLS Decomposition".  Returns (r, P, Q, rows)."""
    A = list(rows_in)
    P = list(range(m))
    Q = list(range(n))
    r = c = 0
    while r < m and c < n:
        found = False
        for j in range(c, n):              # search for some pivot, column by column
            for i in range(r, m):
                if bit(A[i], j):
                    found = True
                    break
            if found:
                break
        if not found:
            break
        P[r], Q[r] = i, j
        swap_rows(A, r, i)
        if j + 1 < n:                       # clear below, keeping L in column j
            for l in range(r + 1, m):
                if bit(A[l], j):
                    add_row_from(A, l, r, j + 1)
        r, c = r + 1, j + 1
    for i in range(r, m):
        P[i] = i
    for i in range(r, n):
        Q[i] = i
    compress_l(A, Q, r)
    return r, P, Q, A


# ------------------------------------------------------------------ MMPF pieces
def pls_submatrix(A: list[int], m: int, n: int, s_r: int, s_c: int, k: int,
                  P: list[int], Q: list[int]):
    """Appendix A, "PlsSubmatrix": find up to k pivots in the k columns starting
    at s_c, searching rows from s_r in the current order; lazily clear earlier
    strip columns (done[] bookkeeping); finish the touched rows.
    Returns (kbar, d_r)."""
    done = [0] * k
    kbar = 0
    for r in range(k):
        found = False
        i = s_r + r
        while i < m:
            for l in range(r):             # clear before
                if done[l] < i:
                    if bit(A[i], s_c + l):
                        add_row_from(A, i, s_r + l, s_c + l + 1)
                    done[l] = i
            if bit(A[i], s_c + r):
                found = True
                break
            i += 1
        if not found:
            break
        P[s_r + r], Q[s_r + r] = i, s_c + r
        swap_rows(A, s_r + r, i)
        done[r] = i
        kbar = r + 1
    d_r = max(done[:kbar]) if kbar else s_r
    for c2 in range(kbar):                 # finish submatrix
        if s_c + c2 < n - 1:
            for r2 in range(done[c2] + 1, d_r + 1):
                if bit(A[r2], s_c + c2):
                    add_row_from(A, r2, s_r + c2, s_c + c2 + 1)
    return kbar, d_r


def gray(i: int) -> int:
    return i ^ (i >> 1)


def table_id(x: int, c: int, k: int) -> int:
    """The k bits of x starting at column c, column c as the most significant."""
    v = 0
    for j in range(k):
        v = (v << 1) | bit(x, c + j)
    return v


def make_table1(U: list[int], c: int, kbar: int):
    """Section 4.1, "MakeTable1".  U holds kbar rows; returns (T, L).

    T[i] is the sum of the rows of U selected by the Gray code g(i), from column
    c on (bit b of g(i) selects row kbar-1-b); L maps the k-bit id read at column
    c of T[i] to i; finally the bits of the a-priori id g(i) are added onto the
    kbar columns starting at c, so that adding T[L[id]] to a row whose strip
    reads id leaves the multipliers of the U rows in the strip."""
    size = 1 << kbar
    T = [0] * size
    for i in range(1, size):
        flipped = (gray(i) ^ gray(i - 1)).bit_length() - 1
        j = kbar - 1 - flipped
        T[i] = T[i - 1] ^ (U[j] & mask_from(c))
    L = [0] * size
    for i in range(1, size):
        L[table_id(T[i], c, kbar)] = i
    for i in range(1, size):
        g = gray(i)
        for j in range(kbar):
            b_j = (g >> (kbar - 1 - j)) & 1
            if b_j:
                T[i] ^= 1 << (c + j)
    return T, L


def make_table(A: list[int], r: int, c: int, k: int):
    """Appendix A, "MakeTable" (M4RI): Gray-code table of the k rows starting at
    row r, from column c, and the array L indexing it by the k bits at column c."""
    size = 1 << k
    T = [0] * size
    for i in range(1, size):
        flipped = (gray(i) ^ gray(i - 1)).bit_length() - 1
        j = r + (k - 1 - flipped)
        T[i] = T[i - 1] ^ (A[j] & mask_from(c))
    L = [0] * size
    for i in range(size):
        L[table_id(T[i], c, k)] = i
    return T, L


def add_rows_from_table(A: list[int], r_start: int, r_end: int, c: int, k: int,
                        T: list[int], L: list[int]) -> None:
    """Appendix A, "AddRowsFromTable"."""
    for i in range(r_start, r_end):
        idx = table_id(A[i], c, k)
        A[i] ^= T[L[idx]] & mask_from(c)


def mmpf(rows_in: list[int], m: int, n: int, k: int):
    """Section 4.1, "MMPF".  Returns (r, P, Q, rows)."""
    A = list(rows_in)
    P = list(range(m))
    Q = list(range(n))
    r = c = 0
    while r < m and c < n:
        kk = min(k, n - c)
        kbar, d_r = pls_submatrix(A, m, n, r, c, kk, P, Q)
        if kbar > 0:
            U = []
            for t in range(kbar):          # zero everything before the triangle
                U.append(A[r + t] & mask_from(c + t))
            T, L = make_table1(U, c, kbar)
            add_rows_from_table(A, d_r + 1, m, c, kbar, T, L)
            r, c = r + kbar, c + kbar
        else:
            c += 1                         # skip zero column
    for i in range(r, m):
        P[i] = i
    for i in range(r, n):
        Q[i] = i
    compress_l(A, Q, r)
    return r, P, Q, A


# ------------------------------------------------------------------------ M4RI
def gauss_submatrix(A: list[int], r: int, c: int, k: int, r_end: int) -> int:
    """Appendix A, "GaussSubmatrix": reduced echelon form of the k-column strip
    at (r, c), searching pivot rows up to r_end.  Returns the rank found."""
    r_s = r
    for j in range(c, c + k):
        found = False
        for i in range(r_s, r_end):
            for l in range(j - c):         # clear the first columns
                if bit(A[i], c + l):
                    add_row_from(A, i, r + l, c + l)
            if bit(A[i], j):
                swap_rows(A, i, r_s)
                for l in range(r, r_s):    # clear above
                    if bit(A[l], j):
                        add_row_from(A, l, r_s, j)
                r_s += 1
                found = True
                break
        if not found:
            return j - c
    return k


def m4ri(rows_in: list[int], m: int, n: int, k: int):
    """Section 3.1, "M4RI": returns (r, rows) with rows in reduced echelon form."""
    A = list(rows_in)
    r = c = 0
    while c < n:
        kk = min(k, n - c)
        kbar = gauss_submatrix(A, r, c, kk, m)
        if kbar > 0:
            T, L = make_table(A, r, c, kbar)
            add_rows_from_table(A, 0, r, c, kbar, T, L)
            add_rows_from_table(A, r + kbar, m, c, kbar, T, L)
        r, c = r + kbar, c + kbar
        if kk != kbar:
            c += 1
    return r, A


# -------------------------------------------------------------- recursive PLS
def pls_recursive(rows_in: list[int], m: int, n: int, base: int = 2):
    """Section 5, "PLS Decomposition", on a column view [0, n) of all m rows.

    n0 is a positive split below n (about n/2); widths <= base fall back to
    Gaussian PLS.  P_1 and Q_1 are fresh vectors for the second call, and the
    final column swaps move the second call's L columns next to the first's.
    Returns (r, P, Q, rows)."""
    A = list(rows_in)
    P = list(range(m))
    Q = list(range(n))
    r = _pls_rec(A, 0, m, 0, n, P, Q, base)
    return r, P, Q, A


def _view_get(A, r0, c0, w, i):
    return (A[r0 + i] >> c0) & ((1 << w) - 1)


def _view_set(A, r0, c0, w, i, v):
    msk = ((1 << w) - 1) << c0
    A[r0 + i] = (A[r0 + i] & ~msk) | ((v << c0) & msk)


def _pls_rec(A, rs, re, cs, ce, P, Q, base):
    """PLS of the view rows [rs, re) x columns [cs, ce); P, Q relative."""
    m, n = re - rs, ce - cs
    if m == 0 or n == 0:
        return 0
    if n <= base:
        sub = [_view_get(A, rs, cs, n, i) for i in range(m)]
        r, Pv, Qv, sub = gaussian_pls(sub, m, n)
        for i in range(m):
            _view_set(A, rs, cs, n, i, sub[i])
        P[:] = Pv
        Q[:] = Qv
        return r
    n0 = n // 2
    P0 = list(range(m))
    Q0 = list(range(n0))
    r0 = _pls_rec(A, rs, re, cs, cs + n0, P0, Q0, base)
    # P*A_1: apply the first call's transpositions to the right columns
    for i in range(r0):
        if P0[i] != i:
            a, b = _view_get(A, rs, cs + n0, n - n0, i), _view_get(A, rs, cs + n0, n - n0, P0[i])
            _view_set(A, rs, cs + n0, n - n0, i, b)
            _view_set(A, rs, cs + n0, n - n0, P0[i], a)
    if r0 > 0:
        # A_NE <- L_NW^{-1} A_NE  (unit lower triangular forward substitution)
        for i in range(r0):
            x = _view_get(A, rs, cs + n0, n - n0, i)
            lrow = _view_get(A, rs, cs, r0, i)
            for j in range(i):
                if bit(lrow, j):
                    x ^= _view_get(A, rs, cs + n0, n - n0, j)
            _view_set(A, rs, cs + n0, n - n0, i, x)
        # A_SE <- A_SE + A_SW * A_NE
        for i in range(r0, m):
            lrow = _view_get(A, rs, cs, r0, i)
            x = _view_get(A, rs, cs + n0, n - n0, i)
            for j in range(r0):
                if bit(lrow, j):
                    x ^= _view_get(A, rs, cs + n0, n - n0, j)
            _view_set(A, rs, cs + n0, n - n0, i, x)
    P1 = list(range(m - r0))
    Q1 = list(range(n - n0))
    r1 = _pls_rec(A, rs + r0, re, cs + n0, ce, P1, Q1, base)
    # A_SW <- P_1 * A_SW
    for i in range(r1):
        if P1[i] != i:
            a = _view_get(A, rs + r0, cs, r0, i)
            b = _view_get(A, rs + r0, cs, r0, P1[i])
            _view_set(A, rs + r0, cs, r0, i, b)
            _view_set(A, rs + r0, cs, r0, P1[i], a)
    for i in range(r0):
        P[i] = P0[i]
    for i in range(m - r0):
        P[r0 + i] = P1[i] + r0
    for i in range(n0):
        Q[i] = Q0[i]
    for i in range(n - n0):
        Q[n0 + i] = Q1[i] + n0
    j = r0
    for i in range(n0, n0 + r1):
        Q[j] = Q[i]
        j += 1
    for i in range(r0 + r1, n):
        Q[i] = i
    # compress L: move the second call's L columns to [r0, r0 + r1)
    for t in range(r1):
        ci, cj = cs + r0 + t, cs + n0 + t
        if ci != cj:
            for row in range(rs + r0 + t, re):
                x = A[row]
                if bit(x, ci) != bit(x, cj):
                    A[row] = x ^ (1 << ci) ^ (1 << cj)
    return r0 + r1


# ------------------------------------------------------------------ RREF, rank
def gauss_jordan(rows_in: list[int], m: int, n: int):
    """Plain Gauss-Jordan; returns (r, rows, pivot_columns)."""
    A = list(rows_in)
    r = 0
    piv = []
    for j in range(n):
        if r >= m:
            break
        pi = next((i for i in range(r, m) if bit(A[i], j)), None)
        if pi is None:
            continue
        swap_rows(A, r, pi)
        for i in range(m):
            if i != r and bit(A[i], j):
                A[i] ^= A[r]
        piv.append(j)
        r += 1
    return r, A, piv

"""Pure-Python statements of the paper's algorithms, for tiny inputs.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Rows are Python ints: column ``j`` is bit ``j``.  Each function computes what the
algorithm it names in Albrecht & Pernet, "Efficient Decomposition of Dense
Matrices over GF(2)", computes, following the algorithm's steps in the paper's
order, but organised around what each step means rather than around the printed
pseudo-code (different loop structure and bookkeeping), so that its agreement
with the C oracle is a check between two codes written independently:

* ``gaussian_pls``        -- Appendix A, Gaussian PLS: the pivot rule applied
                             pivot by pivot, then the in-place layout built
                             directly from its definition.
* ``pls_submatrix``       -- Appendix A, PlsSubmatrix: pivots of one strip, rows
                             brought up to date with a per-row counter.
* ``make_table1``         -- Section 4.1, MakeTable1: every combination of the
                             strip rows, the index map, the multiplier fix.
* ``add_rows_from_table`` -- Appendix A, AddRowsFromTable.
* ``mmpf``                -- Section 4.1, MMPF.
* ``make_table``          -- Appendix A, MakeTable (the M4RI table, no fix).
* ``gauss_submatrix``     -- Appendix A, GaussSubmatrix.
* ``m4ri``                -- Section 3.1, M4RI (reduced row echelon form).
* ``pls_recursive``       -- Section 5, PLS Decomposition (asymptotically fast
                             recursion with a Gaussian base case).

Readings where the printed text is ambiguous (all documented with the design):
indices are 0-based and ranges half-open; the table index reads the k bits
starting at column c with column c as the most significant bit (the "0 1 1 -> 3"
example of Section 3.1); a table entry's selection pattern has the first of the
k source rows as its most significant bit; the "a priori id" of a table entry is
that selection pattern.  Tables are built by doubling (entry idx from entry idx
without its lowest set bit) instead of in Gray-code order: the paper allows any
construction with 2^k - 1 additions, and only the entry selected by an index is
ever read.
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


def lowest_one_at_or_after(x: int, c: int) -> int:
    """Column of the lowest set bit of x at or after column c, or -1."""
    y = x & mask_from(c)
    return (y & -y).bit_length() - 1 if y else -1


def compressed_row(x: int, i: int, Q: list[int], r: int) -> int:
    """Row i of the in-place result, from its state after elimination (the
    multiplier of pivot s in column Q[s], the echelon row itself for i < r):
    columns s < min(i, r) take the multipliers, and for i < r column i takes the
    unit diagonal, columns (i, Q[i]] are zero and the columns right of Q[i] keep
    the row of S."""
    out = 0
    for s in range(min(i, r)):
        out |= bit(x, Q[s]) << s
    if i < r:
        q = Q[i]
        out |= (1 << i) | ((x >> (q + 1)) << (q + 1))
    return out


def finish_pls(A: list[int], P: list[int], Q: list[int], m: int, n: int, r: int):
    for i in range(r, m):
        P[i] = i
    for i in range(r, n):
        Q[i] = i
    return r, P, Q, [compressed_row(A[i], i, Q, r) for i in range(m)]


# ---------------------------------------------------------------- Gaussian PLS
def gaussian_pls(rows_in: list[int], m: int, n: int):
    """Appendix A, Gaussian PLS.  Pivot r is the leftmost column (right of the
    previous pivot) holding a one in some row r.., taken from the first such row
    in the current order, which is exchanged with row r; every later row with a
    one in that column keeps it (its multiplier) and adds the pivot row's columns
    to its right.  Returns (r, P, Q, rows)."""
    A = list(rows_in)
    P = list(range(m))
    Q = list(range(n))
    full = (1 << n) - 1
    r = 0
    start = 0                       # first column a new pivot may take
    while r < m and start < n:
        seen = 0
        for x in A[r:]:
            seen |= x
        j = lowest_one_at_or_after(seen & full, start)
        if j < 0:
            break
        i = next(t for t in range(r, m) if bit(A[t], j))
        P[r], Q[r] = i, j
        swap_rows(A, r, i)
        right = A[r] & mask_from(j + 1)
        for t in range(r + 1, m):
            if bit(A[t], j):
                A[t] ^= right
        r += 1
        start = j + 1
    return finish_pls(A, P, Q, m, n, r)


# ------------------------------------------------------------------ MMPF pieces
def pls_submatrix(A: list[int], m: int, n: int, s_r: int, s_c: int, k: int,
                  P: list[int], Q: list[int]):
    """Appendix A, PlsSubmatrix: up to k pivots of the strip of k columns at
    s_c, among the rows from s_r in the current order.  A row is reduced by the
    strip pivots lazily: a counter per row says how many of them it has seen,
    and the row catches up when the scan reaches it again.  The scan for strip
    column s_c + t looks at rows s_r + t.. and stops at the first one left with
    a one there; a column with no such row ends the strip.  Every row the scan
    reached is then brought up to date with all pivots.  Returns (kbar, first
    row never reached)."""
    seen = {}                       # row position -> pivots applied to it

    def catch_up(i: int, t: int) -> None:
        for s in range(seen.get(i, 0), t):
            if bit(A[i], s_c + s):
                A[i] ^= A[s_r + s] & mask_from(s_c + s + 1)
        seen[i] = t

    t = 0
    reached = s_r
    while t < k:
        col = s_c + t
        hit = -1
        for i in range(s_r + t, m):
            catch_up(i, t)
            reached = max(reached, i + 1)
            if bit(A[i], col):
                hit = i
                break
        if hit < 0:
            break
        dst = s_r + t
        P[dst], Q[dst] = hit, col
        swap_rows(A, dst, hit)
        seen[dst], seen[hit] = seen.get(hit, 0), seen.get(dst, 0)
        t += 1
    for i in range(s_r + t, reached):
        catch_up(i, t)
    return t, reached


def table_id(x: int, c: int, k: int) -> int:
    """The k bits of x starting at column c, column c as the most significant."""
    v = 0
    for j in range(k):
        v = (v << 1) | bit(x, c + j)
    return v


def _combination_table(U: list[int], c: int, k: int) -> list[int]:
    """Entry idx = sum of the rows U[k-1-b] over the set bits b of idx, from
    column c on; each entry from the entry without its lowest set bit."""
    T = [0] * (1 << k)
    for idx in range(1, 1 << k):
        low = idx & -idx
        T[idx] = T[idx ^ low] ^ (U[k - low.bit_length()] & mask_from(c))
    return T


def make_table1(U: list[int], c: int, kbar: int):
    """Section 4.1, MakeTable1.  U holds the kbar strip rows (echelon, columns
    left of each row's diagonal cleared); returns (T, L): T lists every
    combination of them, L maps the kbar-bit pattern a combination shows at
    columns c.. to its entry, and each entry also carries its own selection
    pattern in the strip (the multiplier fix of "Preserving L"), so adding
    T[L[pattern]] to a row leaves the rows' multipliers in its strip."""
    T = _combination_table(U, c, kbar)
    L = [0] * len(T)
    for idx, v in enumerate(T):
        L[table_id(v, c, kbar)] = idx
    for idx in range(len(T)):
        for j in range(kbar):
            if (idx >> (kbar - 1 - j)) & 1:
                T[idx] ^= 1 << (c + j)
    return T, L


def make_table(A: list[int], r: int, c: int, k: int):
    """Appendix A, MakeTable (M4RI): every combination of the k rows starting at
    row r, from column c on, and the map L from the pattern at columns c.. to
    the entry."""
    T = _combination_table(A[r:r + k], c, k)
    L = [0] * len(T)
    for idx, v in enumerate(T):
        L[table_id(v, c, k)] = idx
    return T, L


def add_rows_from_table(A: list[int], r_start: int, r_end: int, c: int, k: int,
                        T: list[int], L: list[int]) -> None:
    """Appendix A, AddRowsFromTable: each row adds the entry its pattern selects."""
    for i in range(r_start, r_end):
        A[i] ^= T[L[table_id(A[i], c, k)]] & mask_from(c)


def mmpf(rows_in: list[int], m: int, n: int, k: int):
    """Section 4.1, MMPF: strips of k columns; each strip's pivots from
    PlsSubmatrix, its echelon rows tabulated by MakeTable1, and the rows the
    strip search never reached updated through the table.  A strip without a
    pivot in its first column moves on by one column.  Returns (r, P, Q, rows)."""
    A = list(rows_in)
    P = list(range(m))
    Q = list(range(n))
    r = c = 0
    while r < m and c < n:
        kbar, reached = pls_submatrix(A, m, n, r, c, min(k, n - c), P, Q)
        if kbar == 0:
            c += 1
            continue
        U = [A[r + t] & mask_from(c + t) for t in range(kbar)]
        T, L = make_table1(U, c, kbar)
        add_rows_from_table(A, reached, m, c, kbar, T, L)
        r += kbar
        c += kbar
    return finish_pls(A, P, Q, m, n, r)


# ------------------------------------------------------------------------ M4RI
def gauss_submatrix(A: list[int], r: int, c: int, k: int, r_end: int) -> int:
    """Appendix A, GaussSubmatrix: the strip of k columns at (r, c) brought to
    reduced echelon form.  For each strip column in turn, rows r + kbar .. in the
    current order are reduced by the strip's pivot rows and tested; the first
    with a one there is moved to slot r + kbar and cleared from the pivot rows
    above it.  Stops at the first strip column without a pivot.  Returns kbar."""
    kbar = 0
    for col in range(c, c + k):
        hit = -1
        for i in range(r + kbar, r_end):
            for s in range(kbar):
                if bit(A[i], c + s):
                    A[i] ^= A[r + s]
            if bit(A[i], col):
                hit = i
                break
        if hit < 0:
            break
        swap_rows(A, r + kbar, hit)
        for s in range(kbar):
            if bit(A[r + s], col):
                A[r + s] ^= A[r + kbar]
        kbar += 1
    return kbar


def m4ri(rows_in: list[int], m: int, n: int, k: int):
    """Section 3.1, M4RI: returns (r, rows) with rows in reduced echelon form."""
    A = list(rows_in)
    r = c = 0
    while c < n:
        width = min(k, n - c)
        kbar = gauss_submatrix(A, r, c, width, m)
        if kbar > 0:
            T, L = make_table(A, r, c, kbar)
            add_rows_from_table(A, 0, r, c, kbar, T, L)
            add_rows_from_table(A, r + kbar, m, c, kbar, T, L)
        r += kbar
        c += kbar + (1 if kbar < width else 0)
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

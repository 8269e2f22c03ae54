/*
 * CPU oracle for PLS and RREF over GF(2).  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  The GPU product path never links or calls it, and shares
 * no code with it.
 *
 * Matrices are bit-packed row-major: column j of row i is bit (j mod 64) of
 * A[i * stride + j / 64].  Bits past column n are zero and stay zero.
 *
 * oracle_pls   -- "Gaussian PLS Decomposition", Appendix A of Albrecht & Pernet,
 *                 "Efficient Decomposition of Dense Matrices over GF(2)".
 *                 Its output is the unique PLS reached by the pivot rule "smallest
 *                 column with a non-zero entry below the current row, first such
 *                 row in the current row order, transposition swap"; the MMPF and
 *                 recursive algorithms (Sections 4 and 5) reach the same result.
 * oracle_rref  -- textbook Gauss-Jordan elimination (Definition "Reduced Row
 *                 Echelon Form", Section 2), written independently of oracle_pls.
 *
 * Plain loops; OpenMP only over the independent rows updated by one pivot.
 */
#include <stdint.h>
#include <string.h>

/* Mutation testing: the pin tests rebuild this file with ORACLE_MUTATION set to
 * 1..5 to plant one plausible mistake each and check that some pin fails.
 * 0 (the default) is the oracle. */
#ifndef ORACLE_MUTATION
#define ORACLE_MUTATION 0
#endif

static inline int bit(const uint64_t *A, int64_t stride, int64_t i, int64_t j)
{
    return (int)((A[i * stride + (j >> 6)] >> (j & 63)) & 1);
}

static inline void swap_rows(uint64_t *A, int64_t stride, int64_t a, int64_t b)
{
    if (a == b) return;
    uint64_t *ra = A + a * stride, *rb = A + b * stride;
    for (int64_t w = 0; w < stride; w++) {
        uint64_t t = ra[w]; ra[w] = rb[w]; rb[w] = t;
    }
}

/* row dst ^= row src on columns [c, n) (words past n are zero in both rows). */
static inline void add_row_from(uint64_t *A, int64_t stride, int64_t n, int64_t dst,
                                int64_t src, int64_t c)
{
    if (c >= n) return;
    uint64_t *d = A + dst * stride;
    const uint64_t *s = A + src * stride;
    int64_t w0 = c >> 6, W = (n + 63) >> 6;
    d[w0] ^= s[w0] & (~0ULL << (c & 63));
    for (int64_t w = w0 + 1; w < W; w++) d[w] ^= s[w];
}

/*
 * Gaussian PLS (Appendix A, algorithm "Gaussian PLS Decomposition").
 * On return A holds L strictly below the diagonal and S on and above it after
 * the final "compress L" column swaps; P (length m) and Q (length n) are in
 * transposition form: step i swapped row i with row P[i], and pivot i sits in
 * column Q[i].  Entries P[i] = i for i >= r and Q[i] = i for i >= r.
 * Returns the rank r.
 */
int64_t oracle_pls(uint64_t *A, int64_t m, int64_t n, int64_t stride, int32_t *P, int32_t *Q)
{
    int64_t r = 0, c = 0;
    while (r < m && c < n) {
        /* pivot choice (Appendix A, Gaussian PLS): the leftmost column j >= c with a
           one in any of the rows r..m-1, and the first of those rows in the order
           they stand in now */
        int64_t pi = -1, pj = -1;
#if ORACLE_MUTATION == 4
        /* planted mistake: row-major search (first row, then its lowest column) */
        for (int64_t i = r; i < m && pi < 0; i++)
            for (int64_t j = c; j < n; j++)
                if (bit(A, stride, i, j)) { pi = i; pj = j; break; }
#else
        for (int64_t j = c; j < n && pi < 0; j++) {
            for (int64_t i = r; i < m; i++) {
                if (bit(A, stride, i, j)) {
                    pi = i; pj = j;
#if ORACLE_MUTATION == 2
                    continue; /* planted mistake: last row with a one */
#endif
                    break;
                }
            }
        }
#endif
        if (pi < 0) break;
        P[r] = (int32_t)pi;
        Q[r] = (int32_t)pj;
#if ORACLE_MUTATION == 5
        /* planted mistake: rotate rows r..pi instead of swapping r and pi */
        for (int64_t i = pi; i > r; i--) swap_rows(A, stride, i, i - 1);
#else
        swap_rows(A, stride, r, pi);
#endif
        /* eliminate column j from the rows below; the one at A[l][j] is kept,
           since it is the multiplier L[l][r], so the row sum starts at j + 1 */
        if (pj + 1 < n) {
            const int64_t rr = r, jj = pj;
#pragma omp parallel for schedule(static) if ((m - rr) * (n - jj) > (1 << 22))
            for (int64_t l = rr + 1; l < m; l++) {
#if ORACLE_MUTATION == 1
                /* planted mistake: add from column j, which erases the L bit */
                if (bit(A, stride, l, jj)) add_row_from(A, stride, n, l, rr, jj);
#else
                if (bit(A, stride, l, jj)) add_row_from(A, stride, n, l, rr, jj + 1);
#endif
            }
        }
        r += 1;
        c = pj + 1;
    }
    for (int64_t i = r; i < m; i++) P[i] = (int32_t)i;
    for (int64_t i = r; i < n; i++) Q[i] = (int32_t)i;
    /* in-place layout: pivot j's multipliers were left in its column Q[j]; for
       j = 0, 1, ... trade the contents of columns j and Q[j] in rows j..m-1, so
       that L ends up in the first r columns (a no-op when Q[j] = j) */
    for (int64_t j = 0; j < r; j++) {
        int64_t q = Q[j];
        if (q == j) continue;
#if ORACLE_MUTATION == 3
        continue; /* planted mistake: L left uncompressed */
#endif
        const int64_t jj = j;
#pragma omp parallel for schedule(static) if ((m - jj) > (1 << 14))
        for (int64_t i = jj; i < m; i++) {
            uint64_t *row = A + i * stride;
            int a = (int)((row[jj >> 6] >> (jj & 63)) & 1);
            int b = (int)((row[q >> 6] >> (q & 63)) & 1);
            if (a != b) {
                row[jj >> 6] ^= 1ULL << (jj & 63);
                row[q >> 6] ^= 1ULL << (q & 63);
            }
        }
    }
    return r;
}

/*
 * Gauss-Jordan reduction to the reduced row echelon form, in place.
 * For each column in order: take any row at or below the current row with a one
 * there, move it up, and clear that column in every other row.  Rows r..m-1 end
 * zero.  Returns r.  Writes the pivot columns to piv (length >= r) if non-null.
 */
int64_t oracle_rref(uint64_t *A, int64_t m, int64_t n, int64_t stride, int32_t *piv)
{
    int64_t r = 0;
    for (int64_t j = 0; j < n && r < m; j++) {
        int64_t pi = -1;
        for (int64_t i = r; i < m; i++)
            if (bit(A, stride, i, j)) { pi = i; break; }
        if (pi < 0) continue;
        swap_rows(A, stride, r, pi);
        const int64_t rr = r, jj = j;
#pragma omp parallel for schedule(static) if (m * (n - jj) > (1 << 22))
        for (int64_t i = 0; i < m; i++) {
            if (i != rr && bit(A, stride, i, jj)) add_row_from(A, stride, n, i, rr, jj);
        }
        if (piv) piv[r] = (int32_t)j;
        r += 1;
    }
    return r;
}

/*
 * Checker for randomized tests (Freivalds 1977), 64 random vectors at once:
 * out[i] bit t = parity of popcount(M[i] AND v_t) over words [0, W) of row i,
 * where bit t of V[j] is entry j of vector v_t (V has 64 W entries).
 */
void oracle_mul64(const uint64_t *M, int64_t rows, int64_t W, int64_t stride, const uint64_t *V,
                  uint64_t *out)
{
#pragma omp parallel for schedule(static) if (rows * W > (1 << 16))
    for (int64_t i = 0; i < rows; i++) {
        const uint64_t *row = M + i * stride;
        uint64_t acc = 0;
        for (int64_t w = 0; w < W; w++) {
            uint64_t x = row[w];
            while (x) {
                acc ^= V[64 * w + __builtin_ctzll(x)];
                x &= x - 1;
            }
        }
        out[i] = acc;
    }
}

/* Number of OpenMP threads the oracle would use (1 when built without OpenMP). */
int oracle_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

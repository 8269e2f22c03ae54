/*
 * Seeded synthetic GF(2) inputs, bit-packed row-major into 64-bit words.
 *
 * This module is shared by the CPU oracle's tests and the GPU path's tests and
 * benchmarks.  It produces inputs only: it contains no step of the PLS method.
 *
 * Storage convention: column j of row i is bit (j mod 64) of word
 * A[i * stride + j / 64] (least significant bit first).  Bits at columns >= n
 * and words at index >= ceil(n/64) inside a row are zero.
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used as a counter-based
 * generator: value(seed, i) = mix64(seed + (i + 1) * 0x9E3779B97F4A7C15), where
 * mix64 is the published SplitMix64 output function.
 */
#include <stdint.h>
#include <string.h>
#include <stdlib.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t synth_splitmix(uint64_t seed, uint64_t i)
{
    return mix64(seed + (i + 1) * GOLDEN);
}

/* Independent stream derived from (seed, tag). */
uint64_t synth_substream(uint64_t seed, uint64_t tag)
{
    return mix64(mix64(seed ^ (tag * 0xD1B54A32D192ED03ULL)) + GOLDEN);
}

static inline uint64_t row_mask_last(int64_t n)
{
    int r = (int)(n & 63);
    return r ? ((1ULL << r) - 1) : ~0ULL;
}

/* p = 1/2: word w of row i is value(seed, i * ceil(n/64) + w), masked to n bits. */
void synth_fill_half(uint64_t *A, int64_t m, int64_t n, int64_t stride, uint64_t seed)
{
    int64_t W = (n + 63) / 64;
#pragma omp parallel for schedule(static) if (m * W > (1 << 16))
    for (int64_t i = 0; i < m; i++) {
        uint64_t *row = A + i * stride;
        for (int64_t w = 0; w < W; w++)
            row[w] = synth_splitmix(seed, (uint64_t)(i * W + w));
        if (W > 0) row[W - 1] &= row_mask_last(n);
        for (int64_t w = W; w < stride; w++) row[w] = 0;
    }
}

/* General density: bit (i, j) = [ (value(seed, i*n + j) >> 32) < thresh ],
 * thresh = round(p * 2^32) computed by the caller (integer test, no floating point). */
void synth_fill_bernoulli(uint64_t *A, int64_t m, int64_t n, int64_t stride, uint64_t seed,
                          uint64_t thresh)
{
    int64_t W = (n + 63) / 64;
#pragma omp parallel for schedule(static) if (m * n > (1 << 20))
    for (int64_t i = 0; i < m; i++) {
        uint64_t *row = A + i * stride;
        memset(row, 0, (size_t)stride * 8);
        for (int64_t j = 0; j < n; j++) {
            uint64_t v = synth_splitmix(seed, (uint64_t)(i * n + j));
            if ((v >> 32) < thresh) row[j >> 6] |= 1ULL << (j & 63);
        }
        (void)W;
    }
}

/* Seeded choice of `count` distinct indices out of [0, range): partial Fisher-Yates
 * driven by value(seed, t).  `perm` must hold `range` ints. */
static void distinct_choice(int64_t *out, int64_t count, int64_t range, uint64_t seed)
{
    int64_t *perm = (int64_t *)malloc((size_t)range * sizeof(int64_t));
    for (int64_t i = 0; i < range; i++) perm[i] = i;
    for (int64_t t = 0; t < count; t++) {
        uint64_t v = synth_splitmix(seed, (uint64_t)t);
        int64_t j = t + (int64_t)(v % (uint64_t)(range - t));
        int64_t tmp = perm[t]; perm[t] = perm[j]; perm[j] = tmp;
        out[t] = perm[t];
    }
    free(perm);
}

/*
 * Planted-rank input A = B * C over GF(2), B (m x r), C (r x n).
 * thresh == 0 selects p = 1/2 word filling, otherwise Bernoulli(thresh / 2^32).
 * If unit != 0, r seeded distinct rows of B are replaced by the unit vectors e_t and
 * r seeded distinct columns of C by e_t, which makes rank(A) = r exactly.
 * The product is the plain definition: row i of A is the XOR of the rows k of C
 * with B[i][k] = 1.
 * Returns 0, or -1 if r > min(m, n) with unit set or allocation fails.
 */
int synth_fill_planted(uint64_t *A, int64_t m, int64_t n, int64_t stride, int64_t r,
                       uint64_t seed, uint64_t thresh, int unit)
{
    if (r < 0 || (unit && (r > m || r > n))) return -1;
    int64_t Wb = (r + 63) / 64, Wc = (n + 63) / 64;
    if (Wb == 0) Wb = 1;
    uint64_t *B = (uint64_t *)calloc((size_t)(m * Wb), 8);
    uint64_t *C = (uint64_t *)calloc((size_t)((r ? r : 1) * Wc), 8);
    if (!B || !C) { free(B); free(C); return -1; }
    uint64_t sB = synth_substream(seed, 0xB), sC = synth_substream(seed, 0xC);
    if (r > 0) {
        if (thresh == 0) {
            synth_fill_half(B, m, r, Wb, sB);
            synth_fill_half(C, r, n, Wc, sC);
        } else {
            synth_fill_bernoulli(B, m, r, Wb, sB, thresh);
            synth_fill_bernoulli(C, r, n, Wc, sC, thresh);
        }
    }
    if (unit && r > 0) {
        int64_t *rows = (int64_t *)malloc((size_t)r * sizeof(int64_t));
        int64_t *cols = (int64_t *)malloc((size_t)r * sizeof(int64_t));
        distinct_choice(rows, r, m, synth_substream(seed, 0xB0));
        distinct_choice(cols, r, n, synth_substream(seed, 0xC0));
        for (int64_t t = 0; t < r; t++) {
            uint64_t *brow = B + rows[t] * Wb;
            memset(brow, 0, (size_t)Wb * 8);
            brow[t >> 6] = 1ULL << (t & 63);
        }
        for (int64_t t = 0; t < r; t++) {
            int64_t c = cols[t];
            for (int64_t k = 0; k < r; k++) C[k * Wc + (c >> 6)] &= ~(1ULL << (c & 63));
            C[t * Wc + (c >> 6)] |= 1ULL << (c & 63);
        }
        free(rows); free(cols);
    }
#pragma omp parallel for schedule(dynamic, 16) if (m * r > (1 << 16))
    for (int64_t i = 0; i < m; i++) {
        uint64_t *out = A + i * stride;
        memset(out, 0, (size_t)stride * 8);
        const uint64_t *brow = B + i * Wb;
        for (int64_t k = 0; k < r; k++) {
            if ((brow[k >> 6] >> (k & 63)) & 1) {
                const uint64_t *crow = C + k * Wc;
                for (int64_t w = 0; w < Wc; w++) out[w] ^= crow[w];
            }
        }
    }
    free(B); free(C);
    return 0;
}

// Internal declarations of the gfx950 kernels and their host-side launchers.
//
// Dynamic extents.  The recursion of Section 5 splits columns at fixed word
// boundaries, so the sequence of kernel launches is known on the host; only the
// ranks found so far are data-dependent.  They live in a device array `rk` with
// one entry per 64-column panel: rk[b] is the rank of columns [0, 64*b).  Every
// row range a kernel touches is an affine function of a few rk entries, given
// as a RowRange and evaluated on the device, so no launch waits on the host.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gf2pls.h"

namespace gf2 {

// Row range [start, end) with start = rk[ib] + a and
// end = min(ie >= 0 ? rk[ie] : m, start + s)   (empty when end <= start).
struct RowRange {
    int32_t ib;
    int32_t ie;
    int32_t a;
    int32_t s;
};

__host__ __device__ inline RowRange row_range(int ib, int ie, int a, int s) {
    RowRange r;
    r.ib = ib; r.ie = ie; r.a = a; r.s = s;
    return r;
}

#ifdef __HIPCC__
__device__ inline void eval_range(const int32_t *rk, int m, RowRange r, int &start, int &end) {
    int base = r.ib >= 0 ? rk[r.ib] : 0;
    start = base + r.a;
    int hi = r.ie >= 0 ? rk[r.ie] : m;
    long long lim = (long long)start + r.s;
    end = (long long)hi < lim ? hi : (int)lim;
    if (end < start) end = start;
}
#endif

// Pairs of moved rows produced by a panel factorisation: count, then
// (destination offset, source offset) pairs relative to the panel's first row.
constexpr int kMaxMoved = 128;
constexpr int kMovedInts = 1 + 2 * kMaxMoved;

// ---------------------------------------------------------------- launchers
// All return hipError_t of the launch.
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t st);

// The words [blk_lo, blk_hi) of every row may live in a separate array (Ab, row
// stride sb, indexed by the same row and word numbers); the search, the final
// pass and the staging of the pivot rows use it, the moves of the other words
// use (A, stride).  Pass Ab = A, sb = stride and the whole width to work in place.
// Panel factorisation of the 64-column panel at word column wc, rows
// [rk[b], m): pivots, row swaps inside the panel, L of every row, compressed.
// Writes rk[b + 1], P and Q at the pivot slots, and the moved-row list.
// Also moves the other words of the pivot rows (the full-row swaps).
// `info` is a device scratch record of panel_info_bytes() bytes.
// The pivot rows' words on [bw_lo, bw_hi) are copied (after the swaps) into
// Bbuf (row t at Bbuf + t * bstride) when Bbuf is non-null.
hipError_t launch_leaf(uint64_t *A, int64_t stride, uint64_t *Ab, int64_t sb, int blk_lo,
                       int blk_hi, int m, int n, int wc, int32_t *rk, int b, int32_t *P, int32_t *Q,
                       int32_t *info, uint64_t *Bbuf, int64_t bstride, int bw_lo, int bw_hi,
                       uint64_t *linv_store, hipStream_t st);
// The two halves of launch_leaf: the search (one block; P, Q, rk[b + 1], *info)
// and the pass after it (final pass, moves, staging, L^{-1}); lazy: the search
// was launch_table_update_search's, and the final pass also adds the previous
// panel's update (info->unext) to the rows the search did not reach.
hipError_t launch_leaf_search(uint64_t *Ab, int64_t sb, int m, int n, int wc, int32_t *rk, int b,
                              int32_t *P, int32_t *Q, int32_t *info, hipStream_t st);
hipError_t launch_panel_post(uint64_t *A, int64_t stride, uint64_t *Ab, int64_t sb, int blk_lo,
                             int blk_hi, int m, int n, int wc, int32_t *rk, int b, int32_t *info,
                             uint64_t *Bbuf, int64_t bstride, int bw_lo, int bw_hi,
                             uint64_t *linv_store, bool lazy, hipStream_t st);
size_t panel_info_bytes();
size_t panel_info_linv_offset();

// X <- T^{-1} X for up to nbmax (<= trsm_block_max_rows() / 64) blocks of 64 rows
// `rows` of A; T's rows are the same rows of Lm, the block of 64 columns starting
// at word lw0 (diagonal block b at word lw0 + b).  lower = 0: unit upper.
// Bt (nullable): the solved rows are also written transposed for a following
// product whose K rows start nbmax-block-aligned at this call's first row: word
// kw0 + v of Bt rows 64 (w - w_lo) + c (row stride sbt words) receives bit c of
// word w of rows 64 v .. 64 v + 63, for v < nbmax (rows past the range as zero).
hipError_t launch_trsm_block(uint64_t *A, int64_t stride, const uint64_t *Lm, int64_t sl, int m,
                             RowRange rows, int lw0, int w_lo, int w_hi, const int32_t *rk,
                             int lower, int nbmax, const uint64_t *linv_store, uint64_t *Bt,
                             int64_t sbt, int kw0, hipStream_t st, const int32_t *nwd = nullptr);
int trsm_block_max_rows();

// Table-driven update after a panel (Section 4.1: MakeTable1 / AddRowsFromTable)
// on word columns [w_lo, w_hi): the panel's pivot rows become U = L^{-1} B and
// every row below adds l U, l its compressed panel word; B (the pivot rows as
// staged by launch_leaf) is read from Bbuf, L^{-1} from `linv` (64 rows).
// k bits per table, `tables` tables per pass over the rows.
// The same update (w_hi > w_lo = wc + 1) fused with the search of the next panel
// (word wc + 1, rows [rk[b + 1], m); writes rk[b + 2], P, Q and *info as
// launch_leaf_search does).  The rows the search does not reach (offsets >= F of
// *info) are left without the update of word wc + 1: the post pass of panel
// wc + 1 must run with lazy = true.
hipError_t launch_table_update_search(uint64_t *A, int64_t stride, int m, int n, int wc, int32_t *rk,
                                      int b, int w_lo, int w_hi, int k, int tables,
                                      const uint64_t *linv, const uint64_t *Bbuf, int64_t bstride,
                                      int32_t *P, int32_t *Q, int32_t *info, int target_blocks,
                                      hipStream_t st);

// Move the second block's L columns next to the first block's (Section 5,
// final "compress L"): node at column c0 (multiple of 64), split n0 columns,
// ranks r0 = rk[b1] - rk[b0], r1 = rk[b2] - rk[b1].
hipError_t launch_compress_shift(uint64_t *A, int64_t stride, int m, int c0, int n0,
                                 const int32_t *rk, int b0, int b1, int b2, hipStream_t st);

// All shifts of an MMPF block of nwd panels at word wb (splits after each panel),
// innermost first.
hipError_t launch_compress_chain_out(uint64_t *A, int64_t stride, uint64_t *Ab, int m, int wb,
                                     int nwd, const int32_t *rk, hipStream_t st);
hipError_t launch_compress_chain(uint64_t *A, int64_t stride, int m, int wb, int nwd,
                                 const int32_t *rk, int64_t wlim, hipStream_t st);

// P[i] = i for i >= r, Q[i] = i for r <= i < n, *rank = r, with r = rk[nb].
hipError_t launch_finalize(int32_t *P, int32_t *Q, int32_t *rank, const int32_t *rk, int nb,
                           int m, int n, hipStream_t st);

// Bit transpose: Bt (rows = 64 * nw bits of B's columns, words = ceil(kmax/64))
// from B rows `brows` (K = their count), word columns [w_lo, w_lo + nw).
// Rows of B beyond K read as zero.
// nwd (nullable, device): a dynamic word count; the launch covers
// min(nw, *nwd) words (the same in the products and the blocked solve below).
hipError_t launch_transpose(const uint64_t *B, int64_t sb, int m, RowRange brows, int w_lo,
                            int nw, int kmax, uint64_t *Bt, int64_t sbt, const int32_t *rk,
                            hipStream_t st, const int32_t *nwd = nullptr);

// C[rows, words w_lo..w_lo+nw) ^= A[rows, K bits from word aw] * B, with B given
// transposed in Bt (64*nw rows of kmax bits, zero past K).  K is the length of
// krows evaluated with kmrows as the default end.
// prof (nullable): the kernel stores its M, K and column count there (timing
// diagnostics).
hipError_t launch_gemm_xor(uint64_t *C, int64_t sc, const uint64_t *A, int64_t sa, int m,
                           RowRange rows, int aw, int w_lo, int nw, const uint64_t *Bt,
                           int64_t sbt, int kmax, RowRange krows, int kmrows, const int32_t *rk,
                           int32_t *prof, hipStream_t st, const int32_t *nwd = nullptr);
hipError_t launch_gemm_mfma(uint64_t *C, int64_t sc, const uint64_t *A, int64_t sa, int m,
                            RowRange rows, int aw, int w_lo, int nw, const uint64_t *Bt,
                            int64_t sbt, int kmax, RowRange krows, int kmrows, const int32_t *rk,
                            int32_t *prof, bool fp4, hipStream_t st,
                            const int32_t *nwd = nullptr);

// RREF helpers (k_rref.hip).  rr (device int32[3]) = {0, r, ceil((n - r) / 64)}
// is written by launch_rref_masks from *rank; the others read r from it.
hipError_t launch_zero_rows(uint64_t *X, int64_t sx, int rows, int words, hipStream_t st);
hipError_t launch_rref_masks(uint64_t *PM, uint64_t *NM, int32_t *prefP, int32_t *prefN,
                             const int32_t *Q, const int32_t *rank, int n, int rmax, int32_t *rr,
                             hipStream_t st);
hipError_t launch_rref_zero(uint64_t *Uc, int64_t su, uint64_t *Xc, int64_t sx, int rmax,
                            const int32_t *rr, hipStream_t st);
hipError_t launch_rref_gather(const uint64_t *Ap, int64_t sap, const int32_t *Q, int rmax, int n,
                              const uint64_t *PM, const uint64_t *NM, const int32_t *prefP,
                              const int32_t *prefN, uint64_t *Uc, int64_t su, uint64_t *Xc,
                              int64_t sx, const int32_t *rr, hipStream_t st);
hipError_t launch_rref_scatter(uint64_t *R, int64_t sr, int m, int n, const int32_t *Q,
                               const int32_t *rr, const uint64_t *NM, const int32_t *prefN,
                               const uint64_t *Xc, int64_t sx, hipStream_t st);

// Solver and null-space kernels (k_solve.hip).
// perm[i] = the original row at position i after the transpositions P[0, r)
// (r = *rank clamped to [0, rmax]); cnt, fill: int32[m], off: int32[m + 1],
// list: int32[rmax] scratch.
hipError_t launch_perm_from_swaps(const int32_t *P, const int32_t *rank, int m, int rmax,
                                  int32_t *cnt, int32_t *off, int32_t *fill, int32_t *list,
                                  int32_t *perm, hipStream_t st);
// Y[i] <- B[perm[i]], m rows of nrw words.
hipError_t launch_gather_rows(uint64_t *Y, int64_t sy, const uint64_t *B, int64_t sb,
                              const int32_t *perm, int m, int nrw, hipStream_t st);
// ext = {0, r, nrw}.
hipError_t launch_solve_extents(const int32_t *rank, int rmax, int nrw, int32_t *ext,
                                hipStream_t st);
// bad[0, nrw) <- OR of Y rows [ext[1], m).
hipError_t launch_consistency(const uint64_t *Y, int64_t sy, int m, int nrw, const int32_t *ext,
                              uint64_t *bad, hipStream_t st);
// X row j <- Y row i when j is the i-th pivot column (PM, prefP), else zero.
hipError_t launch_solve_scatter(uint64_t *X, int64_t sx, int n, int nrw, const uint64_t *Y,
                                int64_t sy, const uint64_t *PM, const int32_t *prefP,
                                hipStream_t st);
// Null-space basis rows from the transposed solved block XT (rows n x n).
hipError_t launch_kernel_scatter(uint64_t *K, int64_t sk, int n, const uint64_t *XT, int64_t sxt,
                                 const uint64_t *PM, const uint64_t *NM, const int32_t *prefP,
                                 const int32_t *prefN, const int32_t *ext, hipStream_t st);

// M4RI and the hybrid (k_m4ri.hip).  rec: m4ri_rec_bytes() of device scratch.
size_t m4ri_rec_bytes();
hipError_t launch_m4ri_prep(const int32_t *info, const int32_t *rk, int b, void *rec,
                            hipStream_t st);
// cbuf: m words of device scratch (the rows' multipliers).
hipError_t launch_m4ri_update(uint64_t *A, int64_t stride, int m, int wc, const int32_t *rk, int b,
                              int w_lo, int w_hi, int k, int tables, const uint64_t *linv,
                              const void *rec, uint64_t *cbuf, const uint64_t *Bbuf,
                              int64_t bstride, int target_blocks, hipStream_t st);
// out[0] = estimated density of rows [rk[b], m) x words [w0, nw) (float bits), out[1] = rk[b].
hipError_t launch_m4ri_density(const uint64_t *A, int64_t stride, int m, int n, int w0,
                               const int32_t *rk, int b, int32_t *out, hipStream_t st);
// C rows [0, rows) <- the columns of X selected by PM, packed (C zero on entry).
hipError_t launch_gather_cols(const uint64_t *X, int64_t sx, int rows, int nw, const uint64_t *PM,
                              const int32_t *prefP, uint64_t *C, int64_t sc, hipStream_t st);
hipError_t launch_mp_finish(int32_t *Q, int32_t *rank, int32_t *ext, const int32_t *Q2,
                            const int32_t *rank2, int R, int c0, int n, hipStream_t st);

// Learned cost model (k_mlp.hip): per problem the table row of the smallest
// predicted log time.
hipError_t launch_costmodel_predict(const float *params, int S, const float *feats, int N,
                                    const gf2_sched *table, gf2_sched *out, hipStream_t st);

// Batched PLS (k_batch.hip): queue order, then one persistent launch of `grid`
// blocks.  ws holds batch_ws_bytes(count) bytes.
size_t batch_ws_bytes(int64_t count);
hipError_t mlp_prepare();
// Rows [rk[ib], m) x nw words: dst word (i, dw0 + j) <- src word (i, sw0 + j).
hipError_t launch_copy_rows(uint64_t *dst, int64_t sd, int dw0, const uint64_t *src, int64_t ss,
                            int sw0, int nw, const int32_t *rk, int ib, int m, hipStream_t st);
hipError_t launch_unpack(const uint64_t *A, int64_t sa, int m, int n, const int32_t *Q,
                         const int32_t *rank, uint64_t *L, int64_t sl, int lwords, uint64_t *S,
                         int64_t ss, int swords, int64_t max_words, hipStream_t st);
hipError_t launch_batch_copy(const gf2_batch_item *src, const gf2_batch_item *dst, int count,
                             hipStream_t st);
// Plain copy of an m x nw-word block between two strided matrices.
hipError_t launch_copy_words(uint64_t *dst, int64_t sd, const uint64_t *src, int64_t ss, int64_t m,
                             int64_t nw, hipStream_t st);
int batch_blocks_per_cu();
hipError_t launch_pls_batched(const gf2_batch_item *items, int count, int32_t *ranks,
                              const gf2_sched *per, gf2_sched def, int32_t *ws, int grid,
                              hipStream_t st);
}  // namespace gf2

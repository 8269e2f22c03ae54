// Table-driven updates of the MMPF base case and the small pieces of the
// recursive driver.
//
// trsm_block_kernel  X <- T^{-1} X for up to 16 blocks of 64 rows (unit lower or
//                    unit upper T): 64 x 64 inverses of the diagonal blocks, then
//                    block substitution with tables of 16 combinations of 4 rows
//                    (MakeTable with k = 4, Section 3.1; AddRowsFromTable,
//                    Appendix A).
// table_update_search_kernel  Schur update after one panel (every row below the
//                    panel's pivot rows adds L[i] * U on the target columns, with
//                    L[i] the row's (final, compressed) panel word and U the
//                    pivot rows; one table per k multipliers, `tables` tables per
//                    pass over the rows), with the next panel's search in its
//                    first block.
// compress_shift_kernel  final "compress L" of Section 5.
// finalize_kernel    P, Q tails and the rank.
#include <algorithm>

#include "gf2_device.h"
#include "gf2_internal.h"
#include "gf2_panel.h"

namespace gf2 {

__global__ void fill_i32_kernel(int32_t *p, int32_t v, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, v, count);
    return hipGetLastError();
}

__global__ void copy_words_kernel(uint64_t *dst, int64_t sd, const uint64_t *src, int64_t ss,
                                  int64_t m, int64_t nw) {
    const int64_t total = m * nw;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / nw, w = e % nw;
        dst[i * sd + w] = src[i * ss + w];
    }
}

hipError_t launch_copy_words(uint64_t *dst, int64_t sd, const uint64_t *src, int64_t ss, int64_t m,
                             int64_t nw, hipStream_t st) {
    const int64_t total = m * nw;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(copy_words_kernel, dim3((unsigned)blocks), dim3(256), 0, st, dst, sd, src, ss,
                       m, nw);
    return hipGetLastError();
}

// Rows [rk[ib], m) x nw words: dst word (i, dw0 + j) <- src word (i, sw0 + j).
__global__ void copy_rows_kernel(uint64_t *dst, int64_t sd, int dw0, const uint64_t *src,
                                 int64_t ss, int sw0, int nw, const int32_t *rk, int ib, int m) {
    const int r0 = rk[ib];
    const int64_t total = (int64_t)(m - r0) * nw;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = r0 + e / nw;
        const int j = (int)(e % nw);
        dst[i * sd + dw0 + j] = src[i * ss + sw0 + j];
    }
}

hipError_t launch_copy_rows(uint64_t *dst, int64_t sd, int dw0, const uint64_t *src, int64_t ss,
                            int sw0, int nw, const int32_t *rk, int ib, int m, hipStream_t st) {
    if (nw <= 0 || m <= 0) return hipSuccess;
    int64_t blocks = ((int64_t)m * nw + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(copy_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, dst, sd, dw0, src,
                       ss, sw0, nw, rk, ib, m);
    return hipGetLastError();
}

// ------------------------------------------------------- blocked TRSM
// X <- T^{-1} X for up to TB_NB blocks of 64 rows in one launch (unit lower or
// unit upper T, its rows in Lm), one thread per row, two words of X per block.
// Each diagonal block's 64 x 64 inverse is formed by one wave (or, for a lower
// block that is exactly the 64 pivots of a full-rank panel, read from the
// inverse the panel search stored).  The blocks are then solved in order
// (forward for lower, backward for upper), right-looking: block b is
// multiplied by its diagonal inverse (tables of all 16 combinations of each 4
// of its rows, MakeTable with k = 4, and one table row per group of 4
// multipliers, AddRowsFromTable), the solved rows are tabulated the same way,
// and every row of the blocks still to come adds their combination selected
// by its L word of block column b.  A thread loads its row's L words once, in
// solve order, so no step waits on memory.  One launch replaces the bottom
// levels of the recursive solve (Section 5 reduces it to products), whose
// products would be too small to fill the device.
constexpr int TB_THREADS = 1024;
constexpr int TB_NB = 16;

// TW words of X per block: 2 when there are enough word pairs to fill the
// chip, else 1 (twice the blocks, half the LDS traffic per block and step;
// every step is bound by the LDS reads of its table lookups).
template <int TW>
__global__ __launch_bounds__(TB_THREADS) void trsm_block_kernel(
    uint64_t *A, int64_t stride, const uint64_t *Lm, int64_t sl, int m, RowRange rows, int lw0,
    int w_lo, int w_hi, const int32_t *rk, int lower, int nbmax, const uint64_t *linv_store,
    uint64_t *Bt, int64_t sbt, int kw0, const int32_t *nwd) {
    __shared__ __attribute__((aligned(16))) uint64_t sX[TB_NB * 64 * TW];
    __shared__ __attribute__((aligned(16))) uint64_t sT[256 * TW];
    __shared__ uint64_t sInv[TB_NB * 64];
    __shared__ uint64_t sIT[TB_NB * 256];   // per diagonal block: 16 groups x 16 combinations of its inverse rows
    int r0, r1;
    eval_range(rk, m, rows, r0, r1);
    const int nr = min(r1 - r0, nbmax * 64);
    // at most one row: nothing to solve, but a transposed copy is still owed
    if (nr <= 1 && Bt == nullptr) return;
    const int nb = max(nr + 63, 0) / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (nwd) w_hi = min(w_hi, w_lo + *nwd);
    const int w0 = w_lo + blockIdx.x * TW;
    const int tw_n = min(TW, w_hi - w0);
    if (tw_n <= 0) return;
    const int row = tid, rb = row >> 6;
    const bool have = row < nr;
    // every load of this thread at once: its X words, its diagonal word and its
    // L words in solve order (step s uses block column lower ? s : nb - 1 - s)
    uint64_t x[TW];
#pragma unroll
    for (int w = 0; w < TW; w++) x[w] = 0ull;
    uint64_t dg = 0, lw[TB_NB];
    if (have) {
        const uint64_t *pa = A + (int64_t)(r0 + row) * stride + w0;
#pragma unroll
        for (int w = 0; w < TW; w++)
            if (w < tw_n) x[w] = pa[w];
        const uint64_t *pl = Lm + (int64_t)(r0 + row) * sl + lw0;
        const int valid = nr - 64 * rb;
        dg = pl[rb] & (valid >= 64 ? ~0ull : ((1ull << valid) - 1));
    }
#pragma unroll
    for (int st = 0; st < TB_NB; st++) {
        const int c = lower ? st : nb - 1 - st;
        const bool later = lower ? rb > c : rb < c;
        // columns past the triangle (a partial last block) are not part of L
        const int cv = nr - 64 * c;
        const uint64_t cmask = cv >= 64 ? ~0ull : ((1ull << max(cv, 0)) - 1);
        lw[st] = (have && st < nb && later) ? Lm[(int64_t)(r0 + row) * sl + lw0 + c] & cmask : 0ull;
    }
#pragma unroll
    for (int w = 0; w < TW; w++) sX[row * TW + w] = x[w];
    if (wave < nb) {
        const int P = lw0 + wave;   // the panel whose pivots these rows would be
        const bool stored = lower && linv_store && rk[P] == 64 * P && rk[P + 1] == 64 * P + 64 &&
                            r0 + 64 * wave == 64 * P;
        sInv[row] = stored ? linv_store[(int64_t)P * 64 + lane] : tri_inverse64_row(dg, lane, lower != 0);
    }
    __syncthreads();
    // tables of each diagonal block's inverse, so that a row below block b can
    // fold its multipliers through Inv_bb: x_r += L[r][b] X_b(new)
    // = (L[r][b] Inv_bb) X_b(old), and one table of X_b(old) per step serves the
    // diagonal solve and the rows below alike
    for (int e = tid; e < nb * 256; e += TB_THREADS) {
        const int blk = e >> 8, g = (e >> 4) & 15, idx = e & 15;
        uint64_t v = 0;
#pragma unroll
        for (int u = 0; u < 4; u++)
            if ((idx >> u) & 1) v ^= sInv[64 * blk + 4 * g + u];
        sIT[e] = v;
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < TB_NB; st++) {
        if (st >= nb) break;
        const int b = lower ? st : nb - 1 - st;
        const int bn = min(64, nr - 64 * b);
        // the row's multipliers on X_b(old) (independent of X, ahead of the barrier)
        uint64_t cp = 0;
        const uint64_t lv = lw[st];
        if (lv) {
#pragma unroll
            for (int g = 0; g < 16; g++) cp ^= sIT[b * 256 + (g << 4) + (int)((lv >> (4 * g)) & 15)];
        }
        build_tables_k4<TW>(&sX[64 * b * TW], bn, 16, sT, tid, TB_THREADS);
        const uint64_t c = (rb == b && have) ? sInv[row] : cp;
        if (c) {
            uint64_t y[TW];
#pragma unroll
            for (int w = 0; w < TW; w++) y[w] = (rb == b) ? 0ull : sX[row * TW + w];
#pragma unroll
            for (int g = 0; g < 16; g++) {
                const uint64_t *t = &sT[((g << 4) + (int)((c >> (4 * g)) & 15)) * TW];
#pragma unroll
                for (int w = 0; w < TW; w++) y[w] ^= t[w];
            }
#pragma unroll
            for (int w = 0; w < TW; w++) sX[row * TW + w] = y[w];
        } else if (rb == b && have) {
#pragma unroll
            for (int w = 0; w < TW; w++) sX[row * TW + w] = 0ull;
        }
        __syncthreads();
    }
    if (have) {
        uint64_t *pa = A + (int64_t)(r0 + row) * stride + w0;
#pragma unroll
        for (int w = 0; w < TW; w++)
            if (w < tw_n) pa[w] = sX[row * TW + w];
    }
    if (Bt != nullptr && wave < nbmax) {
        // the solved rows as the next product's transposed operand: wave v holds
        // rows 64 v .. 64 v + 63 (zero past nr), one 64 x 64 block per word, which
        // becomes word kw0 + v of Bt rows 64 (w - w_lo) .. 64 (w - w_lo) + 63
#pragma unroll
        for (int w = 0; w < TW; w++)
            if (w < tw_n) {
                const uint64_t t = transpose64(sX[row * TW + w], lane);
                Bt[(int64_t)(64 * (w0 - w_lo + w) + lane) * sbt + kw0 + wave] = t;
            }
    }
}

int trsm_block_max_rows() { return TB_NB * 64; }

hipError_t launch_trsm_block(uint64_t *A, int64_t stride, const uint64_t *Lm, int64_t sl, int m,
                             RowRange rows, int lw0, int w_lo, int w_hi, const int32_t *rk,
                             int lower, int nbmax, const uint64_t *linv_store, uint64_t *Bt,
                             int64_t sbt, int kw0, hipStream_t st, const int32_t *nwd) {
    if (w_hi <= w_lo) return hipSuccess;
    if (nbmax > TB_NB) nbmax = TB_NB;
    const int words = w_hi - w_lo;
    if (words >= 512) {   // at least 256 blocks of word pairs
        hipLaunchKernelGGL((trsm_block_kernel<2>), dim3((words + 1) / 2), dim3(TB_THREADS), 0, st, A,
                           stride, Lm, sl, m, rows, lw0, w_lo, w_hi, rk, lower, nbmax, linv_store,
                           Bt, sbt, kw0, nwd);
    } else {
        hipLaunchKernelGGL((trsm_block_kernel<1>), dim3(words), dim3(TB_THREADS), 0, st, A, stride, Lm,
                           sl, m, rows, lw0, w_lo, w_hi, rk, lower, nbmax, linv_store, Bt, sbt, kw0, nwd);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ table update
// After a panel with r pivots (rows [R, R + r)), with B the pivot rows' words on
// the target columns as they were before any update (staged in Bbuf) and L the
// panel's r x r unit lower triangle:
//   pivot rows:      U = L^{-1} B                (the triangular solve)
//   rows below:      x <- x + l U = x + (l L^{-1}) B
// where l is the row's compressed panel word (its multipliers).  Both are
// combinations of B rows, so B is tabulated once per block (MakeTable, k rows
// per table) and every row adds one table row per table (AddRowsFromTable);
// l L^{-1} comes from tables of 8 rows of L^{-1}.  B is read only from the
// staging buffer, so blocks never race on the pivot rows they rewrite.
// A row is owned by 1, 2 or 4 threads, each with its share of the TW
// (<= TU_TWMAX) words of the block's tile (each forms l L^{-1} itself), so the
// rows spread over up to one block per CU; the grid is sized to be resident in
// one round.
constexpr int TU_THREADS = 1024;   // 16 waves hide the table build's latency
constexpr int TU_TWMAX = 8;
constexpr int TU_TABLE_LDS = 128 * 1024;   // budget for the B tables of one pass
constexpr int TU_LDS_MAX = 158 * 1024;
constexpr int CU_LDS = 160 * 1024;

int table_update_tile_words(int k, int tables) {
    int tw = TU_TABLE_LDS / (tables * (1 << k) * 8);
    if (tw > TU_TWMAX) tw = TU_TWMAX;
    if (tw < 1) tw = 1;
    return tw;
}

size_t table_update_lds_bytes(int k, int tables, int TW) {
    return (size_t)(8 * 256 + 64 + 2 * 64 * TW + tables * (1 << k) * TW) * 8;
}

// One block's share of the update: target words [w0, w0 + tw_n) (its tile, TW
// words wide in LDS), rows taken by block bx of the tile's nbx blocks.  Every
// thread of the block calls it.
__device__ inline void table_update_tile(uint64_t *A, int64_t stride, int m, int wc,
                                         const int32_t *rk, int b, int w_lo, int w0, int tw_n,
                                         int k, int tables, int TW, int lg_tpr, int bx, int nbx,
                                         const uint64_t *linv, const uint64_t *Bbuf,
                                         int64_t bstride, uint64_t *tu_lds) {
    uint64_t *sLT = tu_lds;                 // [8][256]   combinations of L^{-1} rows
    uint64_t *sInv = sLT + 8 * 256;         // [64]
    uint64_t *sB = sInv + 64;               // [64][TW]
    uint64_t *sU = sB + 64 * TW;            // [64][TW]   pivot rows' results
    uint64_t *sT = sU + 64 * TW;            // [tables][1 << k][TW]
    const int R = rk[b];
    const int R1 = rk[b + 1];
    const int r = R1 - R;
    if (r <= 0) return;
    const bool pivots_here = bx == 0;
    if (!pivots_here && R1 >= m) return;
    const int tid = threadIdx.x;
    if (tw_n <= 0) return;
    const int wq = tid % TW, pq = tid / TW, pstep = TU_THREADS / TW;
    if (tid < 64) sInv[tid] = linv[tid];
    if (pq < pstep)
        for (int t = pq; t < 64; t += pstep) {
            sB[t * TW + wq] =
                (t < r && wq < tw_n) ? Bbuf[(int64_t)t * bstride + (w0 - w_lo) + wq] : 0ull;
            sU[t * TW + wq] = 0ull;
        }
    // 2^lg_tpr threads share a row: part p owns its words [p wpt, p wpt + wpt)
    // of the tile (each forms the row's multipliers itself).  The first chunk's
    // row words are loaded after the staging loads above and stay in flight
    // while the tables are built: rows at or below R1 belong to their own
    // threads and the block shares nothing else but LDS, so every barrier up to
    // their use waits for LDS traffic only.
    const int rpb = TU_THREADS >> lg_tpr;                 // rows per block
    const int part = tid & ((1 << lg_tpr) - 1);
    const int wpt = (TW + (1 << lg_tpr) - 1) >> lg_tpr;   // words per thread (<= TU_TWMAX)
    const int wb = part * wpt;
    const int wn = max(0, min(wpt, tw_n - wb));           // this thread's words
    const int per = nbx * rpb;
    int i = R1 + bx * rpb + (tid >> lg_tpr);
    bool act = i < m;
    uint64_t l = 0;
    uint64_t x[TU_TWMAX];
    uint64_t *px = A + (int64_t)i * stride + w0 + wb;
    if (act) {
        l = A[(int64_t)i * stride + wc];
#pragma unroll
        for (int w = 0; w < TU_TWMAX; w++)
            if (w < wn) x[w] = px[w];
    }
    block_sync<true>();
    build_tables_8x8<TU_THREADS, true>(sInv, sLT, tid);
    const int ng = (r + k - 1) / k;
    const int npass = (ng + tables - 1) / tables;
    const int esz = 1 << k;
    const uint32_t kmask = (1u << k) - 1;
    const int nrows = m - R1;
    const int nchunks = nrows > 0 ? (nrows + per - 1) / per : 1;
    for (int chunk = 0; chunk < nchunks; chunk++) {
        // the next chunk's row (this thread's too) is requested before this
        // chunk's work, so its load is in flight while this one is updated
        const int in = i + per;
        const bool actn = chunk + 1 < nchunks && in < m;
        uint64_t *pxn = px + (int64_t)per * stride;
        uint64_t ln = 0;
        uint64_t xn[TU_TWMAX];
        if (actn) {
            ln = A[(int64_t)in * stride + wc];
#pragma unroll
            for (int w = 0; w < TU_TWMAX; w++)
                if (w < wn) xn[w] = pxn[w];
        }
        uint64_t c = 0;
        for (int pass = 0; pass < npass; pass++) {
            const int g0 = pass * tables, g1 = min(ng, g0 + tables);
            if (chunk == 0 || npass > 1) {
                if (chunk > 0 || pass > 0) block_sync<true>();
                build_group_tables<true>(sB + (size_t)g0 * k * TW, r - g0 * k, k, g1 - g0, sT, TW,
                                         tid, TU_THREADS);
                if (pivots_here && chunk == 0 && pq < pstep) {
                    for (int t = pq; t < r; t += pstep) {
                        const uint64_t ct = sInv[t];
                        uint64_t y = sU[t * TW + wq];
                        for (int g = g0; g < g1; g++)
                            y ^= sT[((g - g0) * esz + (int)((ct >> (k * g)) & kmask)) * TW + wq];
                        sU[t * TW + wq] = y;
                    }
                }
            }
            if (pass == 0 && act) {
                // the row's multipliers l L^{-1}, formed once its panel word has
                // landed (the empty asm keeps the compiler from hoisting the wait
                // for it above the table builds)
                uint64_t lv = l;
                asm volatile("" : "+v"(lv));
#pragma unroll
                for (int g8 = 0; g8 < 8; g8++) c ^= sLT[g8 * 256 + (int)((lv >> (8 * g8)) & 255)];
            }
            if (act) {
                for (int g = g0; g < g1; g++) {
                    const uint64_t *T =
                        sT + ((size_t)(g - g0) * esz + ((c >> (k * g)) & kmask)) * TW + wb;
#pragma unroll
                    for (int w = 0; w < TU_TWMAX; w++)
                        if (w < wn) x[w] ^= T[w];
                }
            }
        }
        if (act) {
#pragma unroll
            for (int w = 0; w < TU_TWMAX; w++)
                if (w < wn) px[w] = x[w];
        }
        i = in;
        act = actn;
        px = pxn;
        l = ln;
#pragma unroll
        for (int w = 0; w < TU_TWMAX; w++) x[w] = xn[w];
    }
    if (pivots_here && pq < pstep && wq < tw_n)
        for (int t = pq; t < r; t += pstep) A[(int64_t)(R + t) * stride + w0 + wq] = sU[t * TW + wq];
}

// The update after panel wc fused with the search of panel wc + 1.  Blocks
// [1, ...) update words [wc + 2, w_hi) in tiles of TW (table_update_tile); block 0 forms the pivot rows' word wc + 1 (U = L^{-1} B, also kept in
// info->unext) and searches panel wc + 1, giving each row that word's part of
// the update, l U, when it first loads the row (panel_search<..., true>); the
// rows it does not reach get it in the post pass.  The search reads and writes
// word wc + 1 of rows [rk[b + 1], m) and reads their word wc (final since the
// post pass of panel wc); the other blocks read word wc and write words
// >= wc + 2 and the pivot rows, which lie above the search's rows.
__global__ __launch_bounds__(TU_THREADS) void table_update_search_kernel(
    uint64_t *A, int64_t stride, int m, int n, int wc, int32_t *rk, int b, int w_lo, int w_hi,
    int k, int tables, int TW, int lg_tpr, int nxr, const uint64_t *linv, const uint64_t *Bbuf,
    int64_t bstride, int32_t *P, int32_t *Q, PanelInfo *info) {
    extern __shared__ uint64_t tu_lds[];
    const int bid = blockIdx.x;
    if (bid > 0) {
        const int j = bid - 1, ty = j / nxr;
        const int w0 = w_lo + 1 + ty * TW;
        table_update_tile(A, stride, m, wc, rk, b, w_lo, w0, min(TW, w_hi - w0), k, tables, TW,
                          lg_tpr, j - ty * nxr, nxr, linv, Bbuf, bstride, tu_lds);
        return;
    }
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int R = rk[b], R1 = rk[b + 1], r = R1 - R;
    uint64_t *sUn = tu_lds;             // [64]      U's rows
    uint64_t *sTU = sUn + 64;           // [8][256]  combinations of U's rows
    uint64_t *sBw = sTU + 8 * 256;      // [64]      B's rows (word wc + 1)
    uint64_t *sTB = sBw + 64;           // [8][256]  combinations of B's rows
    SearchLds &S = *reinterpret_cast<SearchLds *>(sTB + 8 * 256);
    if (tid >= LEAF_THREADS && tid < LEAF_THREADS + 2 * LEAF_W) {
        // bring the first window's words wc and wc + 1 into the caches while
        // U is formed (the value is only consumed, so the load must land)
        const int e = tid - LEAF_THREADS, o = R1 + (e >> 1);
        if (o < m) {
            const uint64_t pf = A[(int64_t)o * stride + wc + (e & 1)];
            asm volatile("" ::"v"(pf));
        }
    }
    // U = L^{-1} B on word wc + 1: row t is the combination of B's rows selected
    // by row t of L^{-1}, one lookup per 8 of them
    uint64_t lv = 0;
    if (tid < 64) {
        lv = tid < r ? linv[tid] : 0ull;
        sBw[tid] = tid < r ? Bbuf[(int64_t)tid * bstride] : 0ull;
    }
    __syncthreads();
    build_tables_8x8<TU_THREADS, true>(sBw, sTB, tid);
    if (tid < 64) {
        const uint64_t u = add_lu(0ull, lv, sTB);
        sUn[tid] = u;
        info->unext[tid] = u;
        if (tid < r) A[(int64_t)(R + tid) * stride + wc + 1] = u;
    }
    __syncthreads();
    build_tables_8x8<TU_THREADS, true>(sUn, sTU, tid);
    // the search runs on the first LEAF_THREADS threads; the other waves end here
    // (a barrier waits for the waves that have not ended)
    if (wave >= LEAF_THREADS / 64) return;
    const int r2 = panel_search<LEAF_THREADS, true>(A, stride, m, n, wc + 1, R1, P, Q, info, S,
                                                    nullptr, false, sTU);
    if (tid == 0) rk[b + 2] = R1 + r2;
}

hipError_t launch_table_update_search(uint64_t *A, int64_t stride, int m, int n, int wc, int32_t *rk,
                                      int b, int w_lo, int w_hi, int k, int tables,
                                      const uint64_t *linv, const uint64_t *Bbuf, int64_t bstride,
                                      int32_t *P, int32_t *Q, int32_t *infobuf, int target_blocks,
                                      hipStream_t st) {
    if (w_hi <= w_lo) return hipErrorInvalidValue;
    const int nrest = w_hi - w_lo - 1;
    int TW = table_update_tile_words(k, tables);
    if (TW > nrest) TW = std::max(nrest, 1);
    const int ny = nrest > 0 ? (nrest + TW - 1) / TW : 0;
    const size_t search_lds = 2 * (64 + 8 * 256) * 8 + sizeof(SearchLds);
    const size_t lds = std::max(ny > 0 ? table_update_lds_bytes(k, tables, TW) : 0, search_lds);
    const int occ = std::max(1, (int)(CU_LDS / lds));
    const int slots = std::max(2, target_blocks * occ);
    int nxr = 0, lg_tpr = 0;
    if (ny > 0) {
        lg_tpr = TW >= 4 ? 2 : (TW >= 2 ? 1 : 0);
        const int rpb = TU_THREADS >> lg_tpr;
        nxr = (m + rpb - 1) / rpb;
        const int fit = std::max(1, (slots - 1) / ny);
        if (nxr > fit) nxr = fit;
        if (nxr < 1) nxr = 1;
    }
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)table_update_search_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, TU_LDS_MAX);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    PanelInfo *info = reinterpret_cast<PanelInfo *>(infobuf);
    hipLaunchKernelGGL(table_update_search_kernel, dim3(1 + nxr * ny), dim3(TU_THREADS), lds, st, A,
                       stride, m, n, wc, rk, b, w_lo, w_hi, k, tables, TW, lg_tpr, std::max(nxr, 1),
                       linv, Bbuf, bstride, P, Q, info);
    return hipGetLastError();
}

// ---------------------------------------------------------- compress shift
// Node at column c0 with split n0: every row below the first block's pivots
// takes its part of the "compress L" move (shift_row).
__global__ void compress_shift_kernel(uint64_t *A, int64_t stride, int m, int c0, int n0,
                                      const int32_t *rk, int b0, int b1, int b2) {
    const int R = rk[b0], Rm = rk[b1], Re = rk[b2];
    const int r0 = Rm - R, r1 = Re - Rm;
    if (r0 >= n0 || r1 <= 0) return;
    for (int i = Rm + blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
        shift_row(A + (int64_t)i * stride, stride, c0, n0, r0, r1, i - Rm);
}

// The shifts of an MMPF block of nwd panels at word wb, innermost first: the
// block is a right-nested chain of 64-column splits.
__global__ void compress_chain_kernel(uint64_t *A, int64_t stride, int m, int wb, int nwd,
                                      const int32_t *rk, int64_t wlim) {
    const int Re = rk[wb + nwd];
    bool any = false;
    for (int p = 0; p + 1 < nwd; p++) {
        const int r0 = rk[wb + p + 1] - rk[wb + p];
        if (r0 < 64 && Re > rk[wb + p + 1]) any = true;
    }
    if (!any) return;
    for (int i = rk[wb + 1] + blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += gridDim.x * blockDim.x) {
        uint64_t *row = A + (int64_t)i * stride;
        for (int p = nwd - 2; p >= 0; p--) {
            const int Rp = rk[wb + p], Rm = rk[wb + p + 1];
            const int r0 = Rm - Rp, r1 = Re - Rm;
            if (r0 < 64 && r1 > 0 && i >= Rm) shift_row(row, wlim, 64 * (wb + p), 64, r0, r1, i - Rm);
        }
    }
}

hipError_t launch_compress_shift(uint64_t *A, int64_t stride, int m, int c0, int n0,
                                 const int32_t *rk, int b0, int b1, int b2, hipStream_t st) {
    int blocks = (m + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(compress_shift_kernel, dim3(blocks), dim3(256), 0, st, A, stride, m, c0, n0,
                       rk, b0, b1, b2);
    return hipGetLastError();
}

// The same chain on a base block held in a contiguous copy (Ab: rows of nwd
// words, word w of the block at Ab + row * nwd + (w - wb)), followed by the copy
// of the block's rows [rk[wb], m) back into A: one thread per row.
__global__ void compress_chain_out_kernel(uint64_t *A, int64_t stride, uint64_t *Ab, int m, int wb,
                                          int nwd, const int32_t *rk) {
    const int Re = rk[wb + nwd];
    bool any = false;
    for (int p = 0; p + 1 < nwd; p++) {
        const int r0 = rk[wb + p + 1] - rk[wb + p];
        if (r0 < 64 && Re > rk[wb + p + 1]) any = true;
    }
    for (int i = rk[wb] + blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += gridDim.x * blockDim.x) {
        uint64_t *row = Ab + (int64_t)i * nwd - wb;
        if (any)
            for (int p = nwd - 2; p >= 0; p--) {
                const int Rp = rk[wb + p], Rm = rk[wb + p + 1];
                const int r0 = Rm - Rp, r1 = Re - Rm;
                if (r0 < 64 && r1 > 0 && i >= Rm) shift_row(row, wb + nwd, 64 * (wb + p), 64, r0, r1, i - Rm);
            }
        uint64_t *dst = A + (int64_t)i * stride;
        for (int w = wb; w < wb + nwd; w++) dst[w] = row[w];
    }
}

hipError_t launch_compress_chain_out(uint64_t *A, int64_t stride, uint64_t *Ab, int m, int wb,
                                     int nwd, const int32_t *rk, hipStream_t st) {
    int blocks = (m + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(compress_chain_out_kernel, dim3(blocks), dim3(256), 0, st, A, stride, Ab, m,
                       wb, nwd, rk);
    return hipGetLastError();
}

hipError_t launch_compress_chain(uint64_t *A, int64_t stride, int m, int wb, int nwd,
                                 const int32_t *rk, int64_t wlim, hipStream_t st) {
    if (nwd < 2) return hipSuccess;
    int blocks = (m + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(compress_chain_kernel, dim3(blocks), dim3(256), 0, st, A, stride, m, wb,
                       nwd, rk, wlim);
    return hipGetLastError();
}

// ---------------------------------------------------------------- finalize
__global__ void finalize_kernel(int32_t *P, int32_t *Q, int32_t *rank, const int32_t *rk, int nb,
                                int m, int n) {
    const int r = rk[nb];
    const int mx = m > n ? m : n;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < mx; i += gridDim.x * blockDim.x) {
        if (i >= r && i < m) P[i] = i;
        if (i >= r && i < n) Q[i] = i;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *rank = r;
}

hipError_t launch_finalize(int32_t *P, int32_t *Q, int32_t *rank, const int32_t *rk, int nb,
                           int m, int n, hipStream_t st) {
    int mx = m > n ? m : n;
    int blocks = (mx + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(finalize_kernel, dim3(blocks), dim3(256), 0, st, P, Q, rank, rk, nb, m, n);
    return hipGetLastError();
}

}  // namespace gf2

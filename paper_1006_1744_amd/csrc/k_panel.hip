// Kernels of the single-matrix base case around the panel search: the search
// itself (one block), and the final pass plus the moves of the pivot rows'
// other words (panel_post).
#include "gf2_panel.h"

namespace gf2 {

__global__ __launch_bounds__(LEAF_THREADS) void leaf_search_kernel(
    uint64_t *A, int64_t stride, int m, int n, int wc, int32_t *rk, int b, int32_t *P,
    int32_t *Q, PanelInfo *info) {
    __shared__ SearchLds S;
    const int R = rk[b];
    // L^{-1} of the panel is left to the post kernel (its last block), off the
    // search's critical path: nothing reads it before the table update
    const int r = panel_search(A, stride, m, n, wc, R, P, Q, info, S, nullptr, false);
    if (threadIdx.x == 0) rk[b + 1] = R + r;
}

// Final pass over the panel (blocks [0, nfin)) and the other word columns of
// the moved rows (blocks [nfin, ...)), which touch disjoint words.
//  * final pass: rows >= F receive the previous panel's update of this word
//    when the search ran fused with it (lazy: l U, U = info->unext, l the row's
//    previous word), then the pending pivots [pa, r) through their tables, and
//    every row gets the panel's "compress L" column swaps; a thread's first
//    row is loaded before the tables are built.
//  * moves: the (destination, source) list goes to LDS once; a block copies
//    SWAP_W word columns of every moved row through LDS (all reads, one
//    barrier, all writes), and stages the pivot rows' words on [bw_lo, bw_hi)
//    for the table update that follows from the same copies.
//  * the last block computes the panel's L^{-1} (info->linv and the per-panel
//    store) from the pivot words and columns the search recorded.
constexpr int POST_THREADS = 256;
constexpr int SWAP_W = 8;

template <bool LAZY>
__global__ __launch_bounds__(POST_THREADS) void panel_post_kernel(
    uint64_t *A, int64_t stride, uint64_t *Ab, int64_t sb, int blk_lo, int blk_hi, int m, int wc,
    int nwords, const int32_t *rk, int b, PanelInfo *info, int nfin, uint64_t *Bbuf,
    int64_t bstride, int bw_lo, int bw_hi, uint64_t *linv_store) {
    __shared__ uint64_t sT[8][256];
    __shared__ uint64_t sTU[8 * 256];   // combinations of info->unext (lazy)
    __shared__ uint64_t sUn[64];
    __shared__ uint64_t sU[64];
    __shared__ int32_t sQ[64];
    __shared__ uint64_t stage[kMaxMoved * SWAP_W];
    __shared__ int32_t sDst[kMaxMoved], sSrc[kMaxMoved];
    __shared__ int32_t sPk[64];
    const int tid = threadIdx.x;
    const bool wave0 = __builtin_amdgcn_readfirstlane(tid >> 6) == 0;
    const int l64 = tid & 63;
    if (blockIdx.x == gridDim.x - 1) {
        // L^{-1} needs the panel record alone (r = 0 when no row was left: unit rows)
        if (wave0) {
            const int ru = info->r;
            const uint64_t lrow = panel_linv_row(l64 < ru ? info->u[l64] : 0ull, info->q[l64], ru, l64);
            info->linv[l64] = lrow;
            if (linv_store) linv_store[(int64_t)b * 64 + l64] = lrow;
        }
        return;
    }
    const bool rows_blk = (int)blockIdx.x < nfin;
    // Every load that does not depend on the rank goes out with it: the panel
    // record's words (rows blocks, first wave), its counts, the move list's length
    uint64_t iu = 0, iun = 0;
    int iq = 0;
    if (rows_blk && wave0) {
        iu = info->u[l64];
        iq = info->q[l64];
        if (LAZY) iun = info->unext[l64];
    }
    const int R = rk[b];
    const int r = info->r, F = info->F, pa = info->pa, cmp = info->compress;
    const int32_t *mv = info->moved;
    const int nk = mv[0];
    const int mrem = m - R;
    if (mrem <= 0) return;
    if (rows_blk) {
        uint64_t *col = Ab + (int64_t)R * sb + wc;   // the panel word lies in the block
        const int step = nfin * POST_THREADS;
        // the first row's words are requested as soon as the rank is known, before
        // the block decides whether it has work, and stay in flight across the
        // barriers below (they wait for LDS traffic only); addresses are clamped to
        // a valid row, so the loads are unconditional
        int o = blockIdx.x * POST_THREADS + tid;
        const int64_t oc = (int64_t)min(o, mrem - 1) * sb;
        uint64_t v = col[oc];
        uint64_t lp = LAZY ? col[oc - 1] : 0ull;   // word wc - 1 lies in the block when LAZY
        const bool pend = (F < mrem) && (r > pa);
        const bool lazy = LAZY && F < mrem;   // rows >= F lack the previous update
        if (!pend && !cmp && !lazy) return;
        if (wave0) {
            sU[l64] = iu;
            sQ[l64] = iq;
            sUn[l64] = iun;
        }
        block_sync<true>();
        if (pend) build_tables<POST_THREADS>(sU, sQ, pa, r, sT, tid);
        if (lazy) build_tables_8x8<POST_THREADS, true>(sUn, sTU, tid);
        block_sync<true>();
        for (; o < mrem; o += step) {
            if (o >= (int)(blockIdx.x + nfin) * POST_THREADS) {
                v = col[(int64_t)o * sb];
                lp = LAZY ? col[(int64_t)o * sb - 1] : 0ull;
            }
            uint64_t w = v;
            if (lazy && o >= F) w = add_lu(w, lp, sTU);
            if (pend && o >= F) w = apply_tables(w, sQ, pa, r, sT);
            if (cmp) {
                // compress L: swap panel columns s and q[s] in rows o >= s
                const int lim = min(o + 1, r);
                for (int s2 = 0; s2 < lim; s2++) {
                    const int qs = sQ[s2];
                    if (qs != s2) {
                        const uint64_t d = ((w >> s2) ^ (w >> qs)) & 1ull;
                        w ^= (d << s2) | (d << qs);
                    }
                }
            }
            if (w != v) col[(int64_t)o * sb] = w;
        }
        return;
    }
    const int w0 = ((int)blockIdx.x - nfin) * SWAP_W;
    if (tid < nk) {
        sDst[tid] = mv[1 + 2 * tid];
        sSrc[tid] = mv[2 + 2 * tid];
    }
    if (tid < 64) sPk[tid] = -1;
    __syncthreads();
    if (tid < nk && sDst[tid] < 64) sPk[sDst[tid]] = tid;
    // words of the block live in (Ab, sb), the others in (A, stride)
    auto wp = [&](int row, int w) -> uint64_t * {
        return (w >= blk_lo && w < blk_hi) ? Ab + (int64_t)row * sb + w : A + (int64_t)row * stride + w;
    };
    // every load of this thread first, then the stores (a fixed count per thread,
    // so that the loads are in flight together)
    constexpr int NPT = (kMaxMoved * SWAP_W + POST_THREADS - 1) / POST_THREADS;
    const int ne = nk * SWAP_W;
    uint64_t sv[NPT];
#pragma unroll
    for (int i = 0; i < NPT; i++) {
        const int e = tid + i * POST_THREADS;
        const int k = e / SWAP_W, w = w0 + e % SWAP_W;
        sv[i] = (e < ne && w < nwords && w != wc) ? *wp(R + sSrc[k], w) : 0ull;
    }
#pragma unroll
    for (int i = 0; i < NPT; i++) {
        const int e = tid + i * POST_THREADS;
        if (e < ne) stage[e] = sv[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NPT; i++) {
        const int e = tid + i * POST_THREADS;
        const int k = e / SWAP_W, w = w0 + e % SWAP_W;
        if (e < ne && w < nwords && w != wc) *wp(R + sDst[k], w) = sv[i];
    }
    // the pivot rows' words on [bw_lo, bw_hi) after the moves: a moved pivot row
    // takes the staged copy, any other is not written by this launch
    const int blo = max(bw_lo, w0), bhi = min(bw_hi, min(w0 + SWAP_W, nwords));
    if (Bbuf != nullptr && bhi > blo) {
        const int bw = bhi - blo;
        constexpr int NPB = (64 * SWAP_W + POST_THREADS - 1) / POST_THREADS;
        uint64_t bv[NPB];
#pragma unroll
        for (int i = 0; i < NPB; i++) {
            const int e = tid + i * POST_THREADS;
            const int t = e / bw, w = blo + e % bw;
            bv[i] = 0ull;
            if (e < r * bw) {
                const int k = sPk[t];
                bv[i] = k >= 0 ? stage[k * SWAP_W + (w - w0)] : *wp(R + t, w);
            }
        }
#pragma unroll
        for (int i = 0; i < NPB; i++) {
            const int e = tid + i * POST_THREADS;
            const int t = e / bw, w = blo + e % bw;
            if (e < r * bw) Bbuf[(int64_t)t * bstride + (w - bw_lo)] = bv[i];
        }
    }
}

hipError_t launch_leaf_search(uint64_t *Ab, int64_t sb, int m, int n, int wc, int32_t *rk, int b,
                              int32_t *P, int32_t *Q, int32_t *infobuf, hipStream_t st) {
    PanelInfo *info = reinterpret_cast<PanelInfo *>(infobuf);
    hipLaunchKernelGGL(leaf_search_kernel, dim3(1), dim3(LEAF_THREADS), 0, st, Ab, sb, m, n, wc, rk,
                       b, P, Q, info);
    return hipGetLastError();
}

hipError_t launch_panel_post(uint64_t *A, int64_t stride, uint64_t *Ab, int64_t sb, int blk_lo,
                             int blk_hi, int m, int n, int wc, int32_t *rk, int b, int32_t *infobuf,
                             uint64_t *Bbuf, int64_t bstride, int bw_lo, int bw_hi,
                             uint64_t *linv_store, bool lazy, hipStream_t st) {
    PanelInfo *info = reinterpret_cast<PanelInfo *>(infobuf);
    int nwords = (n + 63) / 64;
    int nfin = (m + POST_THREADS - 1) / POST_THREADS;
    if (nfin > 512) nfin = 512;
    if (nfin < 1) nfin = 1;
    int nswap = (nwords + SWAP_W - 1) / SWAP_W;
    if (lazy)
        hipLaunchKernelGGL(panel_post_kernel<true>, dim3(nfin + nswap + 1), dim3(POST_THREADS), 0, st,
                           A, stride, Ab, sb, blk_lo, blk_hi, m, wc, nwords, rk, b, info, nfin, Bbuf,
                           bstride, bw_lo, bw_hi, linv_store);
    else
        hipLaunchKernelGGL(panel_post_kernel<false>, dim3(nfin + nswap + 1), dim3(POST_THREADS), 0, st,
                           A, stride, Ab, sb, blk_lo, blk_hi, m, wc, nwords, rk, b, info, nfin, Bbuf,
                           bstride, bw_lo, bw_hi, linv_store);
    return hipGetLastError();
}

hipError_t launch_leaf(uint64_t *A, int64_t stride, uint64_t *Ab, int64_t sb, int blk_lo,
                       int blk_hi, int m, int n, int wc, int32_t *rk, int b, int32_t *P, int32_t *Q,
                       int32_t *infobuf, uint64_t *Bbuf, int64_t bstride, int bw_lo, int bw_hi,
                       uint64_t *linv_store, hipStream_t st) {
    hipError_t e = launch_leaf_search(Ab, sb, m, n, wc, rk, b, P, Q, infobuf, st);
    if (e != hipSuccess) return e;
    return launch_panel_post(A, stride, Ab, sb, blk_lo, blk_hi, m, n, wc, rk, b, infobuf, Bbuf,
                             bstride, bw_lo, bw_hi, linv_store, false, st);
}

size_t panel_info_bytes() { return sizeof(PanelInfo); }
size_t panel_info_linv_offset() { return offsetof(PanelInfo, linv); }

}  // namespace gf2

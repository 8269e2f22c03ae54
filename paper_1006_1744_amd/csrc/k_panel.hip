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
//  * final pass: rows >= F receive the pending pivots [pa, r) through their
//    tables, and every row gets the panel's "compress L" column swaps; each
//    thread holds POST_ROWS rows so that their loads are in flight together.
//  * moves: the (destination, source) list goes to LDS once; a block copies
//    SWAP_W word columns of every moved row through LDS (all reads, one
//    barrier, all writes), and stages the pivot rows' words on [bw_lo, bw_hi)
//    for the table update that follows from the same copies.
//  * the last block computes the panel's L^{-1} (info->linv and the per-panel
//    store) from the pivot words and columns the search recorded.
constexpr int POST_THREADS = 1024;
constexpr int POST_ROWS = 1;
constexpr int SWAP_W = 16;

__global__ __launch_bounds__(POST_THREADS) void panel_post_kernel(
    uint64_t *A, int64_t stride, uint64_t *Ab, int64_t sb, int blk_lo, int blk_hi, int m, int wc,
    int nwords, const int32_t *rk, int b, PanelInfo *info, int nfin, uint64_t *Bbuf,
    int64_t bstride, int bw_lo, int bw_hi, uint64_t *linv_store) {
    __shared__ uint64_t sT[8][256];
    __shared__ uint64_t sU[64];
    __shared__ int32_t sQ[64];
    __shared__ uint64_t stage[kMaxMoved * SWAP_W];
    __shared__ int32_t sDst[kMaxMoved], sSrc[kMaxMoved];
    __shared__ int32_t sPk[64];
    const int tid = threadIdx.x;
    const int R = rk[b];
    const int mrem = m - R;
    if (mrem <= 0) return;
    const int r = info->r, F = info->F, pa = info->pa, cmp = info->compress;
    if (blockIdx.x == gridDim.x - 1) {
        if (tid < 64) {
            const uint64_t urow = tid < r ? info->u[tid] : 0ull;
            const uint64_t lrow = panel_linv_row(urow, info->q[tid], __builtin_amdgcn_readfirstlane(r), tid);
            info->linv[tid] = lrow;
            if (linv_store) linv_store[(int64_t)b * 64 + tid] = lrow;
        }
        return;
    }
    if ((int)blockIdx.x < nfin) {
        const bool pend = (F < mrem) && (r > pa);
        if (!pend && !cmp) return;
        if (tid < 64) {
            sU[tid] = info->u[tid];
            sQ[tid] = info->q[tid];
        }
        __syncthreads();
        if (pend) build_tables<POST_THREADS>(sU, sQ, pa, r, sT, tid);
        __syncthreads();
        uint64_t *col = Ab + (int64_t)R * sb + wc;   // the panel word lies in the block
        const int step = nfin * POST_THREADS * POST_ROWS;
        for (int base = blockIdx.x * POST_THREADS * POST_ROWS; base < mrem; base += step) {
            uint64_t v[POST_ROWS];
#pragma unroll
            for (int u = 0; u < POST_ROWS; u++) {
                const int o = base + u * POST_THREADS + tid;
                v[u] = o < mrem ? col[(int64_t)o * sb] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < POST_ROWS; u++) {
                const int o = base + u * POST_THREADS + tid;
                if (o >= mrem) continue;
                uint64_t w = v[u];
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
                if (w != v[u]) col[(int64_t)o * sb] = w;
            }
        }
        return;
    }
    const int32_t *mv = info->moved;
    const int nk = mv[0];
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
    for (int e = tid; e < nk * SWAP_W; e += POST_THREADS) {
        const int k = e / SWAP_W, w = w0 + e % SWAP_W;
        if (w < nwords && w != wc) stage[e] = *wp(R + sSrc[k], w);
    }
    __syncthreads();
    for (int e = tid; e < nk * SWAP_W; e += POST_THREADS) {
        const int k = e / SWAP_W, w = w0 + e % SWAP_W;
        if (w < nwords && w != wc) *wp(R + sDst[k], w) = stage[e];
    }
    // the pivot rows' words on [bw_lo, bw_hi) after the moves: a moved pivot row
    // takes the staged copy, any other is not written by this launch
    const int blo = max(bw_lo, w0), bhi = min(bw_hi, min(w0 + SWAP_W, nwords));
    if (Bbuf != nullptr && bhi > blo) {
        const int bw = bhi - blo;
        for (int e = tid; e < r * bw; e += POST_THREADS) {
            const int t = e / bw, w = blo + e % bw;
            const int k = sPk[t];
            Bbuf[(int64_t)t * bstride + (w - bw_lo)] =
                k >= 0 ? stage[k * SWAP_W + (w - w0)] : *wp(R + t, w);
        }
    }
}

hipError_t launch_leaf(uint64_t *A, int64_t stride, uint64_t *Ab, int64_t sb, int blk_lo,
                       int blk_hi, int m, int n, int wc, int32_t *rk, int b, int32_t *P, int32_t *Q,
                       int32_t *infobuf, uint64_t *Bbuf, int64_t bstride, int bw_lo, int bw_hi,
                       uint64_t *linv_store, hipStream_t st) {
    PanelInfo *info = reinterpret_cast<PanelInfo *>(infobuf);
    hipLaunchKernelGGL(leaf_search_kernel, dim3(1), dim3(LEAF_THREADS), 0, st, Ab, sb, m, n, wc, rk,
                       b, P, Q, info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int nwords = (n + 63) / 64;
    int nfin = (m + POST_THREADS * POST_ROWS - 1) / (POST_THREADS * POST_ROWS);
    if (nfin > 256) nfin = 256;
    if (nfin < 1) nfin = 1;
    int nswap = (nwords + SWAP_W - 1) / SWAP_W;
    hipLaunchKernelGGL(panel_post_kernel, dim3(nfin + nswap + 1), dim3(POST_THREADS), 0, st, A,
                       stride, Ab, sb, blk_lo, blk_hi, m, wc, nwords, rk, b, info, nfin, Bbuf, bstride,
                       bw_lo, bw_hi, linv_store);
    return hipGetLastError();
}

size_t panel_info_bytes() { return sizeof(PanelInfo); }
size_t panel_info_linv_offset() { return offsetof(PanelInfo, linv); }

}  // namespace gf2

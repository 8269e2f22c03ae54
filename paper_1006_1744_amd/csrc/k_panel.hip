// Panel factorisation: PLS of one 64-column panel (one word column) of the rows
// [R, m), R = rk[b], with the pivot rule of Gaussian PLS (Appendix A): smallest
// column with a one among the remaining rows, first such row in the current
// order, transposition swap; additions keep the multiplier bit (L) in place.
//
// This is PlsSubmatrix (Appendix A) re-planned for one CU of gfx950:
//  * The search touches a window of LEAF_W rows held in registers of wave 0
//    (LEAF_H rows per lane); a column test is one 64-lane ballot per register
//    and the first set lane (ffs) is the first row in the current order.
//  * Window rows are reduced eagerly by each new pivot (one masked XOR).
//  * Rows past the window frontier F are reduced lazily, as PlsSubmatrix's
//    done[] bookkeeping does: the pivots [pa, t) found since they were last
//    touched ("pending") are kept as Gray-style tables (MakeTable1 with the
//    a-priori-id fix, Section 4.1) of 8 pivots each in LDS, and applied when a
//    row enters the window, is scanned by a far search, or in the final pass.
//  * If no window row has a one in the current column, a block-wide far search
//    scans the rows past the window in order and stops at the first hit.
// The final pass (panel_post) applies the pending tables to rows >= F and the
// "compress L" column swaps of the panel, and moves the pivot rows' other words.
#include <stddef.h>

#include "gf2_device.h"
#include "gf2_internal.h"

namespace gf2 {

constexpr int LEAF_THREADS = 256;
constexpr int LEAF_H = 2;
constexpr int LEAF_W = 64 * LEAF_H;

// Per-panel record written by the search kernel and read by panel_post.
struct PanelInfo {
    int32_t r;       // pivots found
    int32_t F;       // rows at offsets >= F still lack pivots [pa, r)
    int32_t pa;      // first pending pivot
    int32_t compress;// non-zero if some pivot column differs from its index
    int32_t q[64];   // pivot columns relative to the panel
    uint64_t u[64];  // pivot rows' panel words when chosen (reduced by earlier pivots)
    uint64_t linv[64];  // rows of L^{-1} for the panel's r x r unit lower triangle
    int32_t moved[kMovedInts];
};

__device__ inline int shfl32(int v, int src) { return __shfl(v, src); }

// Build tables for pivots [ta, tb) (consecutive columns q[ta], q[ta]+1, ...):
// group g holds pivots ta+8g .. ; entry [key] added to a row whose group bits
// read `key` clears them to the multipliers and reduces the bits above.
__device__ void build_tables(const uint64_t *U, const int32_t *q, int ta, int tb,
                             uint64_t (*T)[256], int tid, int nthr) {
    int np = tb - ta;
    int ng = (np + 7) >> 3;
    for (int e = tid; e < ng * 256; e += nthr) {
        int g = e >> 8, comb = e & 255;
        int gs = min(8, np - 8 * g);
        if (comb >= (1 << gs)) continue;
        uint64_t v = 0;
        for (int u = 0; u < gs; u++) {
            if ((comb >> u) & 1) {
                int s = ta + 8 * g + u;
                v ^= U[s] & (~0ull << q[s]);
            }
        }
        int off = q[ta] + 8 * g;
        int key = (int)((v >> off) & ((1u << gs) - 1));
        T[g][key] = v ^ ((uint64_t)comb << off);
    }
}

__device__ inline uint64_t apply_tables(uint64_t x, const int32_t *q, int ta, int tb,
                                        const uint64_t (*T)[256]) {
    int np = tb - ta;
    int base = np > 0 ? q[ta] : 0;
    for (int g = 0; 8 * g < np; g++) {
        int gs = min(8, np - 8 * g);
        int off = base + 8 * g;
        int key = (int)((x >> off) & ((1u << gs) - 1));
        x ^= T[g][key];
    }
    return x;
}

// Entry (h, l) of the window, h and l wave-uniform; every register is read
// with a static index so the window stays in VGPRs.
__device__ inline uint64_t window_get(const uint64_t (&x)[LEAF_H], int h, int l) {
    uint64_t v = 0;
#pragma unroll
    for (int k = 0; k < LEAF_H; k++) {
        uint64_t t = readlane64(x[k], l);
        v = (h == k) ? t : v;
    }
    return v;
}

// Wave-0 bookkeeping of a new pivot t (wave-uniform arguments): the pivot's
// multipliers in pivot order, Lc = (bit q_s of the pivot word for s < t), give
// row t of the panel's unit lower triangle L; lane j keeps column j of L^{-1}
// and extends it by one substitution step.
__device__ inline void note_pivot(int t, int col, uint64_t pw, int lane, int &lq,
                                  uint64_t &linvc) {
    const uint64_t Lc = __ballot(lane < t && ((pw >> lq) & 1ull));
    if (lane == t) lq = col;
    const uint64_t bit = (uint64_t)((__popcll(Lc & linvc) & 1) ^ (lane == t ? 1 : 0));
    linvc |= bit << t;
}

__global__ __launch_bounds__(LEAF_THREADS) void leaf_search_kernel(
    uint64_t *A, int64_t stride, int m, int n, int wc, int32_t *rk, int b, int32_t *P,
    int32_t *Q, PanelInfo *info) {
    __shared__ uint64_t sU[64];
    __shared__ int32_t sQ[64];
    __shared__ int32_t sPrel[64];
    __shared__ uint64_t sT[8][256];   // pending pivots [pa, t), for rows >= F
    __shared__ uint64_t sE[8][256];   // pivots of the last epoch, for rows in [window end, F)
    __shared__ int s_t, s_c, s_F, s_pa, s_brk, s_far, s_tab_lo, s_tab_hi, s_epochs;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int R = rk[b];
    const int mrem = m - R;
    const int nc = min(64, n - 64 * wc);
    uint64_t *col = A + (int64_t)R * stride + wc;
    const int NOHIT = 0x7fffffff;
    // wave 0 state kept across rounds
    int lq = 0;              // lane s: panel column of pivot s
    uint64_t linvc = 0;      // lane j: column j of L^{-1}
    int og[LEAF_H];          // original offset of the row in each window entry
    bool simple = true;      // one window, no far search: moves read off og[]

    if (tid == 0) {
        s_t = 0; s_c = 0; s_F = 0; s_pa = 0; s_tab_lo = -1; s_tab_hi = -1; s_brk = 0;
        s_far = NOHIT; s_epochs = 0;
    }
#pragma unroll
    for (int h = 0; h < LEAF_H; h++) og[h] = lane + 64 * h;
    __syncthreads();

    // Invariant at the top of each round: rows at offsets [t, F) are reduced by
    // every pivot found so far; rows >= F are reduced by pivots [0, pa) only.
    while (true) {
        const int t = s_t, c = s_c, F = s_F, pa = s_pa, tl = s_tab_lo, th = s_tab_hi;
        const int epochs = s_epochs;
        __syncthreads();
        if (mrem <= 0 || c >= nc || t >= mrem) break;
        if (epochs > 0) simple = false;
        const bool need_tab = F < mrem && t > pa && (tl != pa || th != t);
        if (need_tab) build_tables(sU, sQ, pa, t, sT, tid, LEAF_THREADS);
        __syncthreads();
        if (need_tab && tid == 0) { s_tab_lo = pa; s_tab_hi = t; }
        const int ts = t;
        if (wave == 0) {
            uint64_t x[LEAF_H];
            bool valid[LEAF_H];
#pragma unroll
            for (int h = 0; h < LEAF_H; h++) {
                const int o = ts + lane + 64 * h;
                valid[h] = o < mrem;
                uint64_t v = valid[h] ? col[(int64_t)o * stride] : 0;
                if (valid[h] && o >= F && t > pa) v = apply_tables(v, sQ, pa, t, sT);
                x[h] = v;
                og[h] = o;
            }
            int tt = t, cc = c, brk = 0;
            while (cc < nc && tt < mrem) {
                const int es = tt - ts;
                int fe = -1;
#pragma unroll
                for (int h = 0; h < LEAF_H; h++) {
                    const int e = lane + 64 * h;
                    const bool cand = valid[h] && e >= es && ((x[h] >> cc) & 1);
                    const uint64_t bal = __ballot(cand);
                    if (fe < 0 && bal) fe = 64 * h + __ffsll((unsigned long long)bal) - 1;
                }
                if (fe < 0) {
                    if (ts + LEAF_W >= mrem) { cc++; continue; }  // zero in every remaining row
                    brk = 1;
                    break;
                }
                const int he = fe >> 6, le = fe & 63;
                const uint64_t pw = window_get(x, he, le);
                if (fe != es) {
                    const int hs = es >> 6, ls = es & 63;
                    const uint64_t sw = window_get(x, hs, ls);
                    int og_e = 0, og_s = 0;
#pragma unroll
                    for (int h = 0; h < LEAF_H; h++) {
                        const int ve = __builtin_amdgcn_readlane(og[h], le);
                        const int vs = __builtin_amdgcn_readlane(og[h], ls);
                        og_e = (h == he) ? ve : og_e;
                        og_s = (h == hs) ? vs : og_s;
                    }
#pragma unroll
                    for (int h = 0; h < LEAF_H; h++) {
                        if (h == hs && lane == ls) { x[h] = pw; og[h] = og_e; }
                        if (h == he && lane == le) { x[h] = sw; og[h] = og_s; }
                    }
                }
                if (lane == 0) {
                    sU[tt] = pw;
                    sQ[tt] = cc;
                    sPrel[tt] = ts + fe;
                    P[R + tt] = R + ts + fe;
                    Q[R + tt] = 64 * wc + cc;
                }
                note_pivot(tt, cc, pw, lane, lq, linvc);
                const uint64_t above = cc == 63 ? 0ull : (~0ull << (cc + 1));
                const uint64_t add = pw & above;
#pragma unroll
                for (int h = 0; h < LEAF_H; h++) {
                    const int e = lane + 64 * h;
                    if (valid[h] && e > es && ((x[h] >> cc) & 1)) x[h] ^= add;
                }
                tt++;
                cc++;
            }
#pragma unroll
            for (int h = 0; h < LEAF_H; h++) {
                const int o = ts + lane + 64 * h;
                if (valid[h]) col[(int64_t)o * stride] = x[h];
            }
            if (lane == 0) {
                s_t = tt;
                s_c = cc;
                s_brk = brk;
                s_epochs = epochs + 1;
                const int nF = max(F, min(ts + LEAF_W, mrem));
                s_F = nF;
                if (nF >= mrem) s_pa = tt;   // no row is left past the frontier
            }
        }
        __syncthreads();
        const int t1 = s_t, c1 = s_c, brk = s_brk;
        __syncthreads();
        // Rows between the window and an older frontier miss this epoch's pivots.
        const int wend = min(ts + LEAF_W, mrem);
        if (t1 > ts && F > wend) {
            build_tables(sU, sQ, ts, t1, sE, tid, LEAF_THREADS);
            __syncthreads();
            for (int o = wend + tid; o < F; o += LEAF_THREADS)
                col[(int64_t)o * stride] = apply_tables(col[(int64_t)o * stride], sQ, ts, t1, sE);
            __syncthreads();
        }
        if (!brk || t1 > ts) continue;
        // Far search: no window row has a one in column c1.  Scan the rows past
        // the window in order, bringing rows >= F up to date, and stop after the
        // first block-sized chunk holding a hit.
        simple = false;
        const int F2 = s_F, pa2 = s_pa, tl2 = s_tab_lo, th2 = s_tab_hi;
        __syncthreads();
        const bool need2 = F2 < mrem && t1 > pa2 && (tl2 != pa2 || th2 != t1);
        if (need2) build_tables(sU, sQ, pa2, t1, sT, tid, LEAF_THREADS);
        if (tid == 0) s_far = NOHIT;
        __syncthreads();
        if (need2 && tid == 0) { s_tab_lo = pa2; s_tab_hi = t1; }
        int scan_end = wend;
        for (int base = wend; base < mrem; base += LEAF_THREADS) {
            const int o = base + tid;
            if (o < mrem) {
                uint64_t v = col[(int64_t)o * stride];
                if (o >= F2 && t1 > pa2) {
                    v = apply_tables(v, sQ, pa2, t1, sT);
                    col[(int64_t)o * stride] = v;
                }
                if ((v >> c1) & 1) atomicMin(&s_far, o);
            }
            scan_end = min(base + LEAF_THREADS, mrem);
            __syncthreads();
            const bool hit = s_far != NOHIT;
            __syncthreads();
            if (hit) break;
        }
        const int f = s_far;
        const int F3 = max(F2, scan_end);
        if (f == NOHIT) {
            // column c1 is zero in every remaining row; every row is reduced now
            if (tid == 0) { s_c = c1 + 1; s_F = F3; s_pa = t1; }
            __syncthreads();
            continue;
        }
        if (tid == 0) {
            uint64_t pw = col[(int64_t)f * stride];
            uint64_t tw = col[(int64_t)t1 * stride];
            col[(int64_t)t1 * stride] = pw;
            col[(int64_t)f * stride] = tw;
            sU[t1] = pw;
            sQ[t1] = c1;
            sPrel[t1] = f;
            P[R + t1] = R + f;
            Q[R + t1] = 64 * wc + c1;
        }
        __syncthreads();
        if (wave == 0) note_pivot(t1, c1, sU[t1], lane, lq, linvc);
        {
            // rows after f up to the new frontier may hold a one in column c1
            const uint64_t pw = sU[t1];
            const uint64_t above = c1 == 63 ? 0ull : (~0ull << (c1 + 1));
            for (int o = f + 1 + tid; o < F3; o += LEAF_THREADS) {
                uint64_t v = col[(int64_t)o * stride];
                if ((v >> c1) & 1) col[(int64_t)o * stride] = v ^ (pw & above);
            }
        }
        __syncthreads();
        if (tid == 0) {
            s_t = t1 + 1;
            s_c = c1 + 1;
            s_F = F3;
            s_pa = F3 >= mrem ? t1 + 1 : pa2;
            s_epochs = 2;   // moved rows no longer follow from one window
        }
        __syncthreads();
    }
    __syncthreads();

    const int r = max(0, min(s_t, mrem));
    if (wave == 0) {
        int32_t *mv = info->moved;
        if (simple) {
            // one window starting at offset 0: entry e holds the row from og[e]
            int base_cnt = 0;
#pragma unroll
            for (int h = 0; h < LEAF_H; h++) {
                const int e = lane + 64 * h;
                const bool mvd = og[h] != e && e < mrem;
                const uint64_t bal = __ballot(mvd);
                const int idx = base_cnt + __popcll(bal & ((1ull << lane) - 1));
                if (mvd) { mv[1 + 2 * idx] = e; mv[2 + 2 * idx] = og[h]; }
                base_cnt += __popcll(bal);
            }
            if (lane == 0) mv[0] = base_cnt;
        } else {
            // compose the transpositions (s, sPrel[s]) into (position, source) pairs;
            // lane holds list entries lane and lane + 64
            int pos0 = -1, src0 = 0, pos1 = -1, src1 = 0;
            int nk = 0;
            for (int s2 = 0; s2 < r; s2++) {
                const int a = s2, qq = sPrel[s2];
                if (a == qq) continue;
                const uint64_t ba = __ballot(pos0 == a), ba1 = __ballot(pos1 == a);
                const uint64_t bq = __ballot(pos0 == qq), bq1 = __ballot(pos1 == qq);
                const int ia = ba ? __ffsll((unsigned long long)ba) - 1
                                  : (ba1 ? 64 + __ffsll((unsigned long long)ba1) - 1 : -1);
                const int iq = bq ? __ffsll((unsigned long long)bq) - 1
                                  : (bq1 ? 64 + __ffsll((unsigned long long)bq1) - 1 : -1);
                int sa = a, sq = qq;
                if (ia >= 0)
                    sa = ia < 64 ? __builtin_amdgcn_readlane(src0, ia)
                                 : __builtin_amdgcn_readlane(src1, ia - 64);
                if (iq >= 0)
                    sq = iq < 64 ? __builtin_amdgcn_readlane(src0, iq)
                                 : __builtin_amdgcn_readlane(src1, iq - 64);
                // position a now holds the row that was at qq, and qq the one at a
                const int slot_a = ia >= 0 ? ia : nk;
                if (ia < 0) nk++;
                const int slot_q = iq >= 0 ? iq : nk;
                if (iq < 0) nk++;
                if (slot_a < 64) { if (lane == slot_a) { pos0 = a; src0 = sq; } }
                else if (lane == slot_a - 64) { pos1 = a; src1 = sq; }
                if (slot_q < 64) { if (lane == slot_q) { pos0 = qq; src0 = sa; } }
                else if (lane == slot_q - 64) { pos1 = qq; src1 = sa; }
            }
            if (lane == 0) mv[0] = nk;
            if (lane < nk) { mv[1 + 2 * lane] = pos0; mv[2 + 2 * lane] = src0; }
            if (lane + 64 < nk) { mv[1 + 2 * (lane + 64)] = pos1; mv[2 + 2 * (lane + 64)] = src1; }
        }
        // L^{-1}: identity past r, then columns -> rows
        if (lane >= r) linvc = 1ull << lane;
        info->linv[lane] = transpose64(linvc, lane);
        info->q[lane] = lane < r ? sQ[lane] : lane;
        info->u[lane] = lane < r ? sU[lane] : 0ull;
    }
    if (tid == 0) {
        int cmp = 0;
        for (int s2 = 0; s2 < r; s2++) cmp |= (sQ[s2] != s2);
        info->r = r;
        info->F = max(0, min(s_F, mrem));
        info->pa = min(s_pa, r);
        info->compress = cmp;
        rk[b + 1] = R + r;
    }
}

// Final pass over the panel (blocks [0, nfin)) and the other word columns of
// the moved rows (blocks [nfin, ...)), which touch disjoint words.
constexpr int POST_THREADS = 256;
constexpr int SWAP_COLS = 64;

__global__ __launch_bounds__(POST_THREADS) void panel_post_kernel(
    uint64_t *A, int64_t stride, int m, int wc, int nwords, const int32_t *rk, int b,
    const PanelInfo *info, int nfin, uint64_t *Bbuf, int64_t bstride, int bw_lo, int bw_hi) {
    __shared__ uint64_t sT[8][256];
    __shared__ uint64_t sU[64];
    __shared__ int32_t sQ[64];
    __shared__ uint64_t stage[kMaxMoved][SWAP_COLS];
    const int tid = threadIdx.x;
    const int R = rk[b];
    const int mrem = m - R;
    if (mrem <= 0) return;
    const int r = info->r, F = info->F, pa = info->pa, cmp = info->compress;
    if ((int)blockIdx.x < nfin) {
        if (tid < 64) {
            sU[tid] = info->u[tid];
            sQ[tid] = info->q[tid];
        }
        __syncthreads();
        const bool pend = (F < mrem) && (r > pa);
        if (pend) build_tables(sU, sQ, pa, r, sT, tid, POST_THREADS);
        __syncthreads();
        if (!pend && !cmp) return;
        uint64_t *col = A + (int64_t)R * stride + wc;
        for (int o = blockIdx.x * POST_THREADS + tid; o < mrem; o += nfin * POST_THREADS) {
            uint64_t v = col[(int64_t)o * stride];
            uint64_t w = v;
            if (pend && o >= F) w = apply_tables(w, sQ, pa, r, sT);
            if (cmp) {
                // compress L: swap panel columns s and q[s] in rows o >= s
                int lim = min(o + 1, r);
                for (int s = 0; s < lim; s++) {
                    int qs = sQ[s];
                    if (qs != s) {
                        uint64_t d = ((w >> s) ^ (w >> qs)) & 1ull;
                        w ^= (d << s) | (d << qs);
                    }
                }
            }
            if (w != v) col[(int64_t)o * stride] = w;
        }
        return;
    }
    // moved rows, other word columns: stage every source, then write
    const int32_t *mv = info->moved;
    const int nk = mv[0];
    const int w = (blockIdx.x - nfin) * SWAP_COLS + (tid & (SWAP_COLS - 1));
    const int part = tid / SWAP_COLS;          // POST_THREADS / SWAP_COLS parts
    const bool act = w < nwords && w != wc;
    if (nk > 0) {
        for (int k = part; k < nk; k += POST_THREADS / SWAP_COLS)
            stage[k][tid & (SWAP_COLS - 1)] =
                act ? A[(int64_t)(R + mv[2 + 2 * k]) * stride + w] : 0;
        __syncthreads();
        if (act)
            for (int k = part; k < nk; k += POST_THREADS / SWAP_COLS)
                A[(int64_t)(R + mv[1 + 2 * k]) * stride + w] = stage[k][tid & (SWAP_COLS - 1)];
    }
    // the pivot rows' words on [bw_lo, bw_hi), for the update that follows
    if (Bbuf != nullptr && bw_hi > bw_lo) {
        __syncthreads();
        if (w >= bw_lo && w < bw_hi)
            for (int t = part; t < r; t += POST_THREADS / SWAP_COLS)
                Bbuf[(int64_t)t * bstride + (w - bw_lo)] = A[(int64_t)(R + t) * stride + w];
    }
}

hipError_t launch_leaf(uint64_t *A, int64_t stride, int m, int n, int wc, int32_t *rk, int b,
                       int32_t *P, int32_t *Q, int32_t *infobuf, uint64_t *Bbuf,
                       int64_t bstride, int bw_lo, int bw_hi, hipStream_t st) {
    PanelInfo *info = reinterpret_cast<PanelInfo *>(infobuf);
    hipLaunchKernelGGL(leaf_search_kernel, dim3(1), dim3(LEAF_THREADS), 0, st, A, stride, m, n,
                       wc, rk, b, P, Q, info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int nwords = (n + 63) / 64;
    int nfin = (m + POST_THREADS - 1) / POST_THREADS;
    if (nfin > 512) nfin = 512;
    if (nfin < 1) nfin = 1;
    int nswap = (nwords + SWAP_COLS - 1) / SWAP_COLS;
    hipLaunchKernelGGL(panel_post_kernel, dim3(nfin + nswap), dim3(POST_THREADS), 0, st, A,
                       stride, m, wc, nwords, rk, b, info, nfin, Bbuf, bstride, bw_lo, bw_hi);
    return hipGetLastError();
}

size_t panel_info_bytes() { return sizeof(PanelInfo); }
size_t panel_info_linv_offset() { return offsetof(PanelInfo, linv); }

}  // namespace gf2

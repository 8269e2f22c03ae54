// The panel search of the MMPF base case (PlsSubmatrix, Appendix A), as a
// device function shared by the single-matrix panel kernel and the batched
// kernel: PLS of one 64-column panel (one word column) of the rows [R, m),
// with the pivot rule of Gaussian PLS (Appendix A): smallest column with a one
// among the remaining rows, first such row in the current order, transposition
// swap; additions keep the multiplier bit (L) in place.
//
// PlsSubmatrix re-planned for one CU of gfx950:
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
// The final pass (pending tables for rows >= F, the panel's "compress L"
// column swaps) and the moves of the pivot rows' other words follow the search.
#pragma once

#include <stddef.h>

#include "gf2_device.h"
#include "gf2_internal.h"

namespace gf2 {


constexpr int LEAF_THREADS = 256;
constexpr int LEAF_H = 2;
constexpr int LEAF_W = 64 * LEAF_H;

// Per-panel record written by the search and read by the passes after it.
struct PanelInfo {
    int32_t r;       // pivots found
    int32_t F;       // rows at offsets >= F still lack pivots [pa, r)
    int32_t pa;      // first pending pivot
    int32_t compress;// non-zero if some pivot column differs from its index
    int32_t q[64];   // pivot columns relative to the panel
    uint64_t u[64];  // pivot rows' panel words when chosen (reduced by earlier pivots)
    uint64_t linv[64];  // rows of L^{-1} for the panel's r x r unit lower triangle
    int32_t moved[kMovedInts];
    // When the search ran fused with the update after the previous panel: that
    // panel's pivot rows' words on this panel's column (U = L^{-1} B there), zero
    // past its rank.  Rows the search did not reach (offsets >= F) still lack
    // their part of that update, x += l U with l their previous-panel word.
    uint64_t unext[64];
};

// x + l U on one word: 8 lookups in the 8 tables of 256 combinations of U's rows
// (T[g * 256 + e], build_tables_8x8), l the row's multipliers.
__device__ inline uint64_t add_lu(uint64_t x, uint64_t l, const uint64_t *T) {
#pragma unroll
    for (int g = 0; g < 8; g++) x ^= T[g * 256 + (int)((l >> (8 * g)) & 255)];
    return x;
}

// Build tables for pivots [ta, tb) (consecutive columns q[ta], q[ta]+1, ...):
// group g holds pivots ta+8g .. ; entry [key] added to a row whose group bits
// read `key` clears them to the multipliers and reduces the bits above.  The
// NTHR threads are split into 8 sets of NTHR / 8 (a power of two), set g
// building group g: a thread reads its group's 8 (masked) pivot rows from LDS
// once; its combinations share their low log2(NTHR / 8) bits, whose part of
// the sum it forms once, and it walks the high bits in Gray-code order, one
// XOR per entry.  No barrier inside.
template <int NTHR>
__device__ inline void build_tables(const uint64_t *U, const int32_t *q, int ta, int tb,
                                    uint64_t (*T)[256], int tid) {
    constexpr int TPG = NTHR / 8;
    static_assert(TPG > 0 && (TPG & (TPG - 1)) == 0 && TPG <= 256, "threads per group");
    constexpr int LB = __builtin_ctz(TPG);   // low bits fixed per thread
    const int np = tb - ta;
    const int ng = (np + 7) >> 3;
    const int g = tid / TPG;
    if (g >= ng) return;
    const int gs = min(8, np - 8 * g);
    uint64_t uu[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const int s = min(ta + 8 * g + u, tb - 1);   // in range for every u
        const uint64_t keep = u < gs ? ~0ull : 0ull;
        uu[u] = U[s] & (~0ull << (q[s] & 63)) & keep;
    }
    const int off = q[ta] + 8 * g;
    const int base = tid - g * TPG;
    uint64_t vlow = 0;
#pragma unroll
    for (int u = 0; u < LB; u++) vlow ^= ((base >> u) & 1) ? uu[u] : 0ull;
    uint64_t vh = 0;
#pragma unroll
    for (int i = 0; i < (256 >> LB); i++) {
        if (i > 0) vh ^= uu[LB + __builtin_ctz(i)];   // Gray codes i - 1 and i differ there
        const int comb = base + ((i ^ (i >> 1)) << LB);
        if (comb < (1 << gs)) {
            const uint64_t v = vlow ^ vh;
            const int key = (int)((v >> off) & ((1u << gs) - 1));
            T[g][key] = v ^ ((uint64_t)comb << off);
        }
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

// All-ones if bit 0 of x is set, else zero (one v_bfe_i32; left to itself the
// compiler turns the field extract into a compare and a select).
__device__ inline uint32_t sext_bit0(uint32_t x) {
    uint32_t r;
    asm("v_bfe_i32 %0, %1, 0, 1" : "=v"(r) : "v"(x));
    return r;
}

// v with bit b cleared (wave-uniform, one scalar instruction).
__device__ inline uint64_t sbitclear64(uint64_t v, int b) {
    asm("s_bitset0_b64 %0, %1" : "+s"(v) : "s"(b));
    return v;
}

// Value v (wave-uniform) written into lane l of a per-lane register.
__device__ inline uint64_t writelane64(uint64_t old, uint64_t v, int l) {
    return (int)__lane_id() == l ? v : old;
}

__device__ inline int writelane32(int v, int l, int old) {
    return (int)__lane_id() == l ? v : old;
}


// LDS of one search (every thread of the block takes part).
struct SearchLds {
    uint64_t sU[64];
    int32_t sQ[64];
    int32_t sPrel[64];
    uint64_t sT[8][256];   // pending pivots [pa, t), for rows >= F
    uint64_t sE[8][256];   // pivots of the last epoch, for rows in [window end, F)
    int s_t, s_c, s_F, s_pa, s_brk, s_far, s_tab_lo, s_tab_hi, s_epochs;
    int sOg[LEAF_W];       // first window: original offset of each entry's row
    // OR of the rows past the window, taken by a far search that found no row
    // with a one; it stays exact for every column while no pivot found since has
    // a one there in it (s_or_ok)
    unsigned long long s_orv;
    int s_or_ok;
    int s_touch;           // the last epoch's pivots may have ones in those rows
    unsigned long long s_dry;   // columns with no candidate in any row of the last window
};

// Row `lane` of L^{-1} for a panel with ru pivots, lane t holding pivot word
// urow = u[t] and pivot column qv = q[t] (identity past ru); one wave.
// L (ru x ru, pivot order): L[t][s] is bit q[s] of u[t].  Forward substitution
// by rows: X[t] = e_t + sum of X[s] over s < t with L[t][s] = 1, so at step s
// row s is final and is added to every later row whose strictly lower part has
// bit s.  Lane t keeps that part with its bits already in pivot order (gathered
// through two transposes when some pivot column is not its own index); X[s] has
// no bits above s, so before step 32 only the low halves change.  Rows past ru
// stay unit vectors.  Plain code (no inline assembly): the row read back by
// readlane feeds vector instructions, and the compiler places the wait states
// that such a read needs.
__device__ inline uint64_t panel_linv_row(uint64_t urow, int qv, int ru, int lane) {
    uint64_t uq = urow;   // bit s: bit q[s] of this row
    if (__ballot(lane < ru && qv != lane)) {
        const uint64_t ct = transpose64(urow, lane);   // lane c: column c over the rows
        const uint64_t cq = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(ct >> 32), qv) << 32) |
                            (uint32_t)__shfl((int)(uint32_t)ct, qv);   // lane s: column q[s]
        uq = transpose64(cq, lane);
    }
    const uint64_t l = lane < ru && lane > 0 ? uq & (~0ull >> (64 - lane)) : 0ull;
    const int llo = (int)(uint32_t)l, lhi = (int)(uint32_t)(l >> 32);
    uint32_t xlo = lane < 32 ? 1u << lane : 0u;
    uint32_t xhi = lane >= 32 ? 1u << (lane - 32) : 0u;
#pragma unroll
    for (int s2 = 0; s2 < 63; s2++) {
        const uint32_t f = (uint32_t)__builtin_amdgcn_sbfe(s2 < 32 ? llo : lhi, s2 & 31, 1);
        xlo ^= (uint32_t)__builtin_amdgcn_readlane((int)xlo, s2) & f;
        if (s2 >= 32) xhi ^= (uint32_t)__builtin_amdgcn_readlane((int)xhi, s2) & f;
    }
    return ((uint64_t)xhi << 32) | xlo;
}

// Search of the panel at word column wc over rows [R, m).  Writes P and Q at
// the pivot slots R + t, the window rows' and scanned rows' panel words, and
// *info (r, F, pa, compress, q, u, moved), and, when want_linv, L^{-1} to
// info->linv and to linv_out (64 words) when given.  Returns r (in every thread).
// Every one of the block's NT threads calls it.
// LAZY: the previous panel's update has not reached this panel's word yet; a row
// receives it (add_lu with tables TU and the row's word wc - 1) when the search
// first loads it, i.e. at offsets >= F, so rows the search never reaches keep
// lacking it (info->unext, the post pass).
template <int NT = LEAF_THREADS, bool LAZY = false>
__device__ inline int panel_search(uint64_t *A, int64_t stride, int m, int n, int wc, int R,
                                   int32_t *P, int32_t *Q, PanelInfo *info, SearchLds &S,
                                   uint64_t *linv_out = nullptr, bool want_linv = true,
                                   const uint64_t *TU = nullptr) {
    uint64_t *sU = S.sU;
    int32_t *sQ = S.sQ;
    int32_t *sPrel = S.sPrel;
    uint64_t (*sT)[256] = S.sT;
    uint64_t (*sE)[256] = S.sE;
    int &s_t = S.s_t, &s_c = S.s_c, &s_F = S.s_F, &s_pa = S.s_pa, &s_brk = S.s_brk;
    int &s_far = S.s_far, &s_tab_lo = S.s_tab_lo, &s_tab_hi = S.s_tab_hi, &s_epochs = S.s_epochs;
    int &s_or_ok = S.s_or_ok;
    int *sOg = S.sOg;

    // wave index made visibly uniform, so that the one-wave sections below are
    // uniform branches and their loop state stays in scalar registers
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int mrem = m - R;
    const int nc = min(64, n - 64 * wc);
    uint64_t *col = A + (int64_t)R * stride + wc;
    const int NOHIT = 0x7fffffff;
    bool simple = true;      // one window, no far search: moves read off sOg[]

    if (tid == 0) {
        s_t = 0; s_c = 0; s_F = 0; s_pa = 0; s_tab_lo = -1; s_tab_hi = -1; s_brk = 0;
        s_far = NOHIT; s_epochs = 0; s_or_ok = 0;
    }
    __syncthreads();

    // Invariant at the top of each round: rows at offsets [t, F) are reduced by
    // every pivot found so far; rows >= F are reduced by pivots [0, pa) only.
    while (true) {
        const int t = s_t, c = s_c, F = s_F, pa = s_pa, tl = s_tab_lo, th = s_tab_hi;
        const int epochs = s_epochs;
        // (block-uniform values, kept in scalar registers)
        const int or_ok = __builtin_amdgcn_readfirstlane(s_or_ok);
        const uint64_t orv0 = S.s_orv;
        const uint64_t orv = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(orv0 >> 32)) << 32) |
                             (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)orv0);
        __syncthreads();
        if (mrem <= 0 || c >= nc || t >= mrem) break;
        if (epochs > 0) simple = false;
        const bool need_tab = F < mrem && t > pa && (tl != pa || th != t);
        if (need_tab) build_tables<NT>(sU, sQ, pa, t, sT, tid);
        __syncthreads();
        if (need_tab && tid == 0) { s_tab_lo = pa; s_tab_hi = t; }
        const int ts = t;
        if (wave == 0) {
            // Window: entries e = lane and 64 + lane hold the rows at offsets ts + e,
            // all reduced by every pivot found so far.  The search works on the
            // transpose: lane j holds column j of the window as two 64-bit words
            // (bit e = entry e), so a column's candidates are one readlane and a
            // row operation is one masked XOR per lane.
            const int o0 = ts + lane, o1 = ts + 64 + lane;
            uint64_t x0 = o0 < mrem ? col[(int64_t)o0 * stride] : 0ull;
            uint64_t x1 = o1 < mrem ? col[(int64_t)o1 * stride] : 0ull;
            if constexpr (LAZY) {
                const bool n0 = o0 < mrem && o0 >= F, n1 = o1 < mrem && o1 >= F;
                const uint64_t l0 = n0 ? col[(int64_t)o0 * stride - 1] : 0ull;
                const uint64_t l1 = n1 ? col[(int64_t)o1 * stride - 1] : 0ull;
                if (n0) x0 = add_lu(x0, l0, TU);
                if (n1) x1 = add_lu(x1, l1, TU);
            }
            if (t > pa) {
                if (o0 < mrem && o0 >= F) x0 = apply_tables(x0, sQ, pa, t, sT);
                if (o1 < mrem && o1 >= F) x1 = apply_tables(x1, sQ, pa, t, sT);
            }
            int og0 = o0, og1 = o1;
            uint64_t m0 = __ballot(o0 < mrem), m1 = __ballot(o1 < mrem);   // candidates
            uint64_t c0 = transpose64(x0, lane), c1 = transpose64(x1, lane);
            int fer = -1;   // lane j: window entry of the pivot of column j (this epoch)
            // loop state kept in scalar registers: column, pivot count, candidates
            int cc = __builtin_amdgcn_readfirstlane(c);
            int tt = __builtin_amdgcn_readfirstlane(t);
            const int tsu = __builtin_amdgcn_readfirstlane(ts);
            int brk = 0;
            while (true) {
                // Common case, kept in a loop of its own with one path: the pivot
                // of column cc lies in the first half, at entry fl >= es.  Rows
                // with a one in column cc other than the pivot add the pivot row
                // on the columns right of cc (column j > cc flips them where the
                // pivot has a one); then entries es and fl trade places (no change
                // when fl == es).
                // cc and tt advance together here, so one bound covers both limits
                const int lim = min(nc, cc + (mrem - tt));
                // all-ones in lanes j > cc (the columns right of the current one)
                uint32_t gt = lane > cc ? ~0u : 0u;
                // candidates of column cc, none once cc reaches lim (a lane index
                // of 64 reads lane 0, whose value is then dropped)
                uint64_t b0 = readlane64(c0, cc & 63) & m0 & (cc < lim ? ~0ull : 0ull);
                while (b0) {
                    const uint64_t b1 = readlane64(c1, cc) & m1;
                    const int es = tt - tsu;   // < 64: pivots fill the window from its start
                    const int fl = __ffsll((unsigned long long)b0) - 1;
                    const uint64_t E0 = sbitclear64(b0, fl);
                    // all-ones in lanes j > cc whose pivot bit is set (bit fl brought
                    // down, then sign-extended)
                    const uint32_t f32 = sext_bit0((uint32_t)(c0 >> fl)) & gt;
                    c0 = ((uint64_t)xor_and_s((uint32_t)(c0 >> 32), (uint32_t)(E0 >> 32), f32) << 32) |
                         xor_and_s((uint32_t)c0, (uint32_t)E0, f32);
                    c1 = ((uint64_t)xor_and_s((uint32_t)(c1 >> 32), (uint32_t)(b1 >> 32), f32) << 32) |
                         xor_and_s((uint32_t)c1, (uint32_t)b1, f32);
                    if (fl != es) {
                        // entries es and fl trade places, in the window and in the
                        // original-row record
                        const uint64_t d = ((c0 >> es) ^ (c0 >> fl)) & 1ull;
                        const uint64_t de = d << es, df = d << fl;
                        c0 = ((uint64_t)xor_or((uint32_t)(c0 >> 32), (uint32_t)(de >> 32), (uint32_t)(df >> 32)) << 32) |
                             xor_or((uint32_t)c0, (uint32_t)de, (uint32_t)df);
                        const int ogs = __builtin_amdgcn_readlane(og0, es);
                        const int oge = __builtin_amdgcn_readlane(og0, fl);
                        og0 = gf2_amdgcn_writelane(oge, es, og0);
                        og0 = gf2_amdgcn_writelane(ogs, fl, og0);
                    }
                    fer = gf2_amdgcn_writelane(fl, cc, fer);
                    m0 = sbitclear64(m0, es);
                    tt++;
                    cc++;
                    // lane cc drops out (cc & 63: at cc = 64 the loop ends, and
                    // lane 0 is already clear)
                    gt = (uint32_t)gf2_amdgcn_writelane(0, cc & 63, (int)gt);
                    b0 = readlane64(c0, cc & 63) & m0 & (cc < lim ? ~0ull : 0ull);
                }
                if (!(cc < nc && tt < mrem)) break;
                // no first-half entry has a one in column cc
                const uint64_t b1 = readlane64(c1, cc) & m1;
                const int es = tt - tsu;
                if (b1) {
                    // pivot in the second half, at entry 64 + fl
                    const int fl = __ffsll((unsigned long long)b1) - 1;
                    const uint64_t E1 = b1 & ~(1ull << fl);
                    const uint64_t f1 = (lane > cc && ((c1 >> fl) & 1ull)) ? ~0ull : 0ull;
                    c1 ^= E1 & f1;
                    const uint64_t d = ((c0 >> es) ^ (c1 >> fl)) & 1ull;
                    c0 ^= d << es;
                    c1 ^= d << fl;
                    const int ogs = __builtin_amdgcn_readlane(og0, es);
                    const int oge = __builtin_amdgcn_readlane(og1, fl);
                    og0 = lane == es ? oge : og0;
                    og1 = lane == fl ? ogs : og1;
                    fer = lane == cc ? 64 + fl : fer;
                    m0 &= ~(1ull << es);
                    tt++;
                    cc++;
                    continue;
                }
                if (tsu + LEAF_W >= mrem) {   // zero in every remaining row
                    cc++;
                    continue;
                }
                if (or_ok) {
                    // zero in every row past the window too, if no pivot since the
                    // last full far search has touched those rows.  The tables
                    // take an epoch's pivot columns as consecutive, so the column
                    // is skipped in place only before the epoch's first pivot;
                    // otherwise the epoch ends here (no far search) and the next
                    // one starts with it
                    const uint64_t piv = __ballot(fer >= 0);
                    if (!((piv | (1ull << cc)) & orv)) {
                        if (tt != tsu) break;
                        cc++;
                        continue;
                    }
                }
                brk = 1;
                break;
            }
            // columns (lanes) in which no row of the window is a candidate (read
            // only when a far search follows)
            const uint64_t dry = brk ? __ballot(((c0 & m0) | (c1 & m1)) == 0ull) : 0ull;
            x0 = transpose64(c0, lane);
            x1 = transpose64(c1, lane);
            if (o0 < mrem) col[(int64_t)o0 * stride] = x0;
            if (o1 < mrem) col[(int64_t)o1 * stride] = x1;
            // bookkeeping of the pivots [t, tt), one lane per column
            const uint64_t isp = __ballot(fer >= 0);
            // do this epoch's pivots touch the rows past the window?
            const bool touch = !or_ok || (isp & orv) != 0;
            if (or_ok && touch && lane == 0) s_or_ok = 0;
            if (fer >= 0) {
                const int pidx = t + __popcll(isp & ((1ull << lane) - 1));
                P[R + pidx] = R + ts + fer;
                Q[R + pidx] = 64 * wc + lane;
                sQ[pidx] = lane;
                sPrel[pidx] = ts + fer;
            }
            if (lane < tt - t) sU[t + lane] = x0;   // pivot rows stay where they were put
            if (epochs == 0) {
                sOg[lane] = og0;
                sOg[64 + lane] = og1;
            }
            if (lane == 0) {
                s_t = tt;
                s_c = cc;
                s_brk = brk;
                s_epochs = epochs + 1;
                S.s_touch = touch;
                S.s_dry = dry;
                const int nF = max(F, min(ts + LEAF_W, mrem));
                s_F = nF;
                if (nF >= mrem) s_pa = tt;   // no row is left past the frontier
            }
        }
        __syncthreads();
        const int t1 = s_t, c1 = s_c, brk = s_brk, touch = S.s_touch;
        __syncthreads();
        // Rows between the window and an older frontier miss this epoch's pivots.
        const int wend = min(ts + LEAF_W, mrem);
        if (t1 > ts && F > wend && touch) {
            build_tables<NT>(sU, sQ, ts, t1, sE, tid);
            __syncthreads();
            for (int o = wend + tid; o < F; o += NT)
                col[(int64_t)o * stride] = apply_tables(col[(int64_t)o * stride], sQ, ts, t1, sE);
            __syncthreads();
        }
        if (!brk || t1 >= wend) continue;
        // Far search: no row left in the window (offsets [t1, wend), reduced by
        // every pivot and written back) has a one in column c1.  Scan the rows
        // past the window in order, bringing rows >= F up to date, and stop after
        // the first block-sized chunk holding a hit.  After a hit, the next column
        // goes straight to another far search while it too has no candidate in
        // those window rows (dry): they then have zeros in every far pivot's
        // column, so no pivot found meanwhile changes them, and reloading them
        // would find nothing.
        simple = false;
        const uint64_t dry = S.s_dry;
        int tf = t1, cf = c1;
        while (true) {
            const int F2 = s_F, pa2 = s_pa, tl2 = s_tab_lo, th2 = s_tab_hi;
            __syncthreads();
            const bool need2 = F2 < mrem && tf > pa2 && (tl2 != pa2 || th2 != tf);
            // the row a pivot found here will displace (a window row), requested
            // before the tables are built
            const uint64_t tw = tid == 0 ? col[(int64_t)tf * stride] : 0ull;
            if (need2) build_tables<NT>(sU, sQ, pa2, tf, sT, tid);
            if (tid == 0) { s_far = NOHIT; S.s_orv = 0; }
            __syncthreads();
            if (need2 && tid == 0) { s_tab_lo = pa2; s_tab_hi = tf; }
            int scan_end = wend;
            uint64_t acc = 0;   // OR of this thread's scanned rows
            int o = -1;         // this thread's row of the last chunk scanned, and its value
            uint64_t v = 0;
            for (int base = wend; base < mrem; base += NT) {
                o = base + tid;
                if (o < mrem) {
                    v = col[(int64_t)o * stride];
                    if (o >= F2 && (LAZY || tf > pa2)) {
                        if constexpr (LAZY) v = add_lu(v, col[(int64_t)o * stride - 1], TU);
                        if (tf > pa2) v = apply_tables(v, sQ, pa2, tf, sT);
                        col[(int64_t)o * stride] = v;
                    }
                    acc |= v;
                    if ((v >> cf) & 1) atomicMin(&s_far, o);
                }
                scan_end = min(base + NT, mrem);
                __syncthreads();
                const bool hit = s_far != NOHIT;
                __syncthreads();
                if (hit) break;
            }
            const int f = s_far;
            const int F3 = max(F2, scan_end);
            if (f == NOHIT) {
                // column cf is zero in every remaining row; every row is reduced
                // now, and the scan covered every row past the window
                if (acc) atomicOr(&S.s_orv, (unsigned long long)acc);
                if (tid == 0) { s_c = cf + 1; s_F = F3; s_pa = tf; s_or_ok = 1; }
                __syncthreads();
                break;
            }
            // the pivot row comes from the thread that scanned it; rows after it
            // in the last chunk are still in their threads' registers
            if (o == f) sU[tf] = v;
            __syncthreads();
            {
                // rows after f up to the new frontier may hold a one in column cf
                const uint64_t pw = sU[tf];
                const uint64_t above = cf == 63 ? 0ull : (~0ull << (cf + 1));
                if (o > f && o < mrem && ((v >> cf) & 1)) col[(int64_t)o * stride] = v ^ (pw & above);
                for (int o2 = max(f + 1, scan_end) + tid; o2 < F3; o2 += NT) {
                    const uint64_t v2 = col[(int64_t)o2 * stride];
                    if ((v2 >> cf) & 1) col[(int64_t)o2 * stride] = v2 ^ (pw & above);
                }
                if (tid == 0) {
                    col[(int64_t)tf * stride] = pw;
                    col[(int64_t)f * stride] = tw;
                    sQ[tf] = cf;
                    sPrel[tf] = f;
                    P[R + tf] = R + f;
                    Q[R + tf] = 64 * wc + cf;
                }
            }
            __syncthreads();
            if (tid == 0) {
                s_t = tf + 1;
                s_c = cf + 1;
                s_F = F3;
                s_pa = F3 >= mrem ? tf + 1 : pa2;
                s_epochs = 2;   // moved rows no longer follow from one window
                s_or_ok = 0;    // the scan stopped at the hit
            }
            __syncthreads();
            tf++;
            cf++;
            // the rows [tf, wend) are window rows: the chain needs one of them left
            if (!(cf < nc && tf < mrem && tf < wend && ((dry >> cf) & 1ull))) break;
        }
    }
    __syncthreads();

    const int r = max(0, min(s_t, mrem));
    if (wave == 0) {
        int32_t *mv = info->moved;
        if (simple) {
            // one window starting at offset 0: entry e holds the row from sOg[e]
            int base_cnt = 0;
#pragma unroll
            for (int h = 0; h < LEAF_H; h++) {
                const int e = lane + 64 * h;
                const int og = sOg[e];
                const bool mvd = og != e && e < mrem;
                const uint64_t bal = __ballot(mvd);
                const int idx = base_cnt + __popcll(bal & ((1ull << lane) - 1));
                if (mvd) { mv[1 + 2 * idx] = e; mv[2 + 2 * idx] = og; }
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
        const int ru = __builtin_amdgcn_readfirstlane(r);
        const uint64_t urow = lane < ru ? sU[lane] : 0ull;
        const int qv = lane < ru ? sQ[lane] : lane;
        if (want_linv) {
            const uint64_t lrow = panel_linv_row(urow, qv, ru, lane);
            info->linv[lane] = lrow;
            if (linv_out) linv_out[lane] = lrow;
        }
        info->q[lane] = qv;
        info->u[lane] = urow;
        const uint64_t moved_cols = __ballot(lane < ru && qv != lane);
        if (lane == 0) {
            info->r = r;
            info->F = max(0, min(s_F, mrem));
            info->pa = min(s_pa, r);
            info->compress = moved_cols != 0;
        }
    }
    __syncthreads();
    return r;
}


}  // namespace gf2

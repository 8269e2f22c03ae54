// Device helpers shared by the gfx950 kernels: wave-level bit matrix
// operations on 64 x 64 blocks (one 64-bit row per lane) and the LDS tables of
// row combinations used by every table-driven update.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gf2 {

// v_writelane_b32 (the LLVM intrinsic, so that the compiler places the wait
// states and the lane-select register it needs): the wave-uniform value v
// replaces lane `lane` of old.
extern "C" __device__ int gf2_amdgcn_writelane(int v, int lane, int old)
    __asm("llvm.amdgcn.writelane.i32");

// Three-input bit operations of gfx950 (v_bitop3_b32; the truth table is
// indexed by (a << 2) | (b << 1) | c), for the forms the compiler leaves as
// two instructions.  b is wave-uniform (a scalar register), and must come from a
// scalar instruction: a vector instruction that reads a scalar register written by
// another vector instruction (a ballot, a readlane) needs wait states between the
// two, which the compiler inserts for its own code but not before inline assembly.
__device__ inline uint32_t xor_and_s(uint32_t a, uint32_t b, uint32_t c) {   // a ^ (b & c)
    uint32_t d;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x78" : "=v"(d) : "v"(a), "s"(b), "v"(c));
    return d;
}
__device__ inline uint32_t xor_or(uint32_t a, uint32_t b, uint32_t c) {      // a ^ (b | c)
    uint32_t d;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x1e" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

__device__ inline uint64_t readlane64(uint64_t v, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t shfl_xor64(uint64_t v, int mask) {
    int lo = __shfl_xor((int)(uint32_t)v, mask);
    int hi = __shfl_xor((int)(uint32_t)(v >> 32), mask);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// x of lane (lane ^ S), without LDS: v_permlane32_swap / v_permlane16_swap for
// S = 32, 16 (each swaps the halves of a register pair; called with the same
// register twice, its two results hold the other half's values), DPP row
// rotations for S = 8, 4 (row_ror:n gives lane i the value of lane i - n
// within its row of 16; S = 4 rotates by 12 in 4-lane banks 0 and 2 and by 4 in
// banks 1 and 3), DPP quad permutations for S = 2, 1.
template <int S>
__device__ inline uint32_t lane_xor32(uint32_t x, int lane) {
    if constexpr (S == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        return (lane & 32) ? r[0] : r[1];
    } else if constexpr (S == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        return (lane & 16) ? r[0] : r[1];
    } else if constexpr (S == 8) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false);
    } else if constexpr (S == 4) {
        const int p = __builtin_amdgcn_update_dpp(0, (int)x, 0x12C, 0xF, 0x5, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(p, (int)x, 0x124, 0xF, 0xA, false);
    } else if constexpr (S == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);
    } else {
        static_assert(S == 1, "lane distance");
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);
    }
}

// One butterfly stage of the transpose: lanes i and i ^ S trade the S-bit
// blocks that belong to each other (mh: the upper block of every 2S bits).  Each
// lane sends its value already shifted toward the partner's position and keeps
// its own half with one bit-field select.
template <int S>
__device__ inline uint64_t transpose_stage(uint64_t v, uint64_t mh, int lane) {
    const bool up = (lane & S) != 0;
    const uint64_t o = up ? (v << S) : (v >> S);
    const uint64_t q = ((uint64_t)lane_xor32<S>((uint32_t)(o >> 32), lane) << 32) |
                       lane_xor32<S>((uint32_t)o, lane);
    const uint64_t keep = up ? mh : ~mh;
    return (v & keep) | (q & ~keep);
}

// 64 x 64 bit transpose across a wave: lane i holds row i on entry and column i
// on exit.  Six butterfly stages, each exchanging the s-bit of the row and
// column indices between lanes i and i ^ s.  Every lane of the wave must be
// active (the exchanges read the partner lanes' registers).
__device__ inline uint64_t transpose64(uint64_t v, int lane) {
    v = transpose_stage<32>(v, 0xFFFFFFFF00000000ull, lane);
    v = transpose_stage<16>(v, 0xFFFF0000FFFF0000ull, lane);
    v = transpose_stage<8>(v, 0xFF00FF00FF00FF00ull, lane);
    v = transpose_stage<4>(v, 0xF0F0F0F0F0F0F0F0ull, lane);
    v = transpose_stage<2>(v, 0xCCCCCCCCCCCCCCCCull, lane);
    v = transpose_stage<1>(v, 0xAAAAAAAAAAAAAAAAull, lane);
    return v;
}

// Inverse of a 64 x 64 unit triangular matrix T given by the rows in LDS `rows`
// (only the strictly lower part, bits < i of row i, is read when lower != 0;
// only the strictly upper part otherwise).  Lane j holds row j, and solves
// T x = e_j column by column: for each column s (upward for lower, downward for
// upper), if x has bit s set it adds column s of T (one ballot over the rows).
// x is then column j of T^{-1}; the result is returned as rows (lane i = row i
// of T^{-1}) by one transpose.
__device__ inline uint64_t tri_inverse64_row(uint64_t row, int lane, bool lower) {
    uint64_t x = 1ull << lane;
    if (lower) {
        for (int s = 0; s < 63; s++) {
            const uint64_t col = __ballot(lane > s && ((row >> s) & 1ull));
            if ((x >> s) & 1ull) x ^= col;
        }
    } else {
        for (int s = 63; s > 0; s--) {
            const uint64_t col = __ballot(lane < s && ((row >> s) & 1ull));
            if ((x >> s) & 1ull) x ^= col;
        }
    }
    return transpose64(x, lane);
}

__device__ inline uint64_t tri_inverse64(const uint64_t *rows, int lane, bool lower) {
    return tri_inverse64_row(rows[lane], lane, lower);
}

// Workgroup barrier.  LDS_ONLY: waits for this wave's LDS operations only, so
// global loads the wave has in flight stay in flight across it (a
// __syncthreads also drains them); for sections that share nothing but LDS.
template <bool LDS_ONLY>
__device__ inline void block_sync() {
    if constexpr (LDS_ONLY)
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else
        __syncthreads();
}

// Tables of all 256 combinations of each 8 consecutive rows of 64 one-word rows
// (8 groups): T[g * 256 + e] = XOR of rows 8g + u with bit u of e set.  The
// NTHR threads are split into 8 sets of NTHR / 8 (a power of two), set g
// building group g from its 8 rows held in registers; a thread's entries share
// their low log2(NTHR / 8) bits, whose part of the XOR it forms once, and it
// walks the high bits in Gray-code order, one XOR per entry.  One barrier.
template <int NTHR, bool LDS_ONLY = false>
__device__ inline void build_tables_8x8(const uint64_t *rows, uint64_t *T, int tid) {
    constexpr int TPG = NTHR / 8;
    static_assert(TPG > 0 && (TPG & (TPG - 1)) == 0 && TPG <= 256, "threads per group");
    constexpr int LB = __builtin_ctz(TPG);
    const int g = tid / TPG;
    const int base = tid - g * TPG;
    uint64_t rr[8];
#pragma unroll
    for (int u = 0; u < 8; u++) rr[u] = rows[8 * g + u];
    uint64_t vlow = 0;
#pragma unroll
    for (int u = 0; u < LB; u++) vlow ^= ((base >> u) & 1) ? rr[u] : 0ull;
    uint64_t vh = 0;
#pragma unroll
    for (int i = 0; i < (256 >> LB); i++) {
        if (i > 0) vh ^= rr[LB + __builtin_ctz(i)];   // Gray codes i - 1 and i differ there
        T[g * 256 + base + ((i ^ (i >> 1)) << LB)] = vlow ^ vh;
    }
    block_sync<LDS_ONLY>();
}

// Tables of all 16 combinations of each 4 consecutive rows, built directly
// (each entry the XOR of at most 4 rows, one barrier at the end): for group g,
// T[(g * 16 + e) * TW + w] = XOR of rows 4g + u with bit u of e set (rows past
// nrows read as zero).  rows: LDS [>= 4*ng][TW].  All threads must call it.
template <int TW>
__device__ inline void build_tables_k4(const uint64_t *rows, int nrows, int ng, uint64_t *T,
                                       int tid, int nthr) {
    for (int e = tid; e < ng * 16 * TW; e += nthr) {
        const int w = e % TW, idx = (e / TW) & 15, g = e / (16 * TW);
        uint64_t v = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int row = 4 * g + u;
            if (((idx >> u) & 1) && row < nrows) v ^= rows[row * TW + w];
        }
        T[e] = v;
    }
    __syncthreads();
}

// Tables of all combinations of groups of k consecutive rows: for group g,
// T[(g * 2^k + e) * TW + w] = XOR of rows g*k + u with bit u of e set (rows
// past nrows read as zero), word w of a TW-word tile.  k <= 4: every entry
// directly (at most 4 loads), one barrier.  k > 4: by doubling three rows at a
// time, one level per barrier: with entries [0, 2^l) complete, entry
// idx + j 2^l (j < 2^d, d = min(3, k - l)) is entry idx plus the combination j of
// rows g*k + l .. g*k + l + d - 1.  Thread tid works on word tid % TW of items
// tid / TW, tid / TW + nthr / TW, ...  rows: LDS [>= ng*k][TW]; T: LDS
// [ng][2^k][TW].  All threads must call it.
template <bool LDS_ONLY = false>
__device__ inline void build_group_tables(const uint64_t *rows, int nrows, int k, int ng,
                                          uint64_t *T, int TW, int tid, int nthr) {
    const int esz = 1 << k;
    const int wq = tid % TW, pq = tid / TW, pstep = nthr / TW;
    const bool on = pq < pstep;
    if (k <= 4) {
        if (on)
            for (int p = pq; p < ng * esz; p += pstep) {
                const int g = p >> k, comb = p & (esz - 1);
                uint64_t v = 0;
                for (int u = 0; u < k; u++) {
                    const int row = g * k + u;
                    if (((comb >> u) & 1) && row < nrows) v ^= rows[row * TW + wq];
                }
                T[(size_t)p * TW + wq] = v;
            }
        block_sync<LDS_ONLY>();
        return;
    }
    for (int l = 0; l < k; l += 3) {
        const int d = min(3, k - l);
        const int nd = 1 << d;
        if (on)
            for (int p = pq; p < (ng << l); p += pstep) {
                const int g = p >> l, idx = p & ((1 << l) - 1);
                uint64_t *tg = T + ((size_t)g * esz + idx) * TW + wq;
                const uint64_t base = l == 0 ? 0ull : tg[0];
                uint64_t r[3];
#pragma unroll
                for (int u = 0; u < 3; u++) {
                    const int row = g * k + l + u;
                    r[u] = (u < d && row < nrows) ? rows[row * TW + wq] : 0ull;
                }
                uint64_t c[8];
                c[0] = base;
                c[1] = base ^ r[0];
                c[2] = base ^ r[1];
                c[3] = c[1] ^ r[1];
                c[4] = base ^ r[2];
                c[5] = c[1] ^ r[2];
                c[6] = c[2] ^ r[2];
                c[7] = c[3] ^ r[2];
#pragma unroll
                for (int j = 0; j < 8; j++)
                    if (j < nd && (j > 0 || l == 0)) tg[(size_t)(j << l) * TW] = c[j];
            }
        block_sync<LDS_ONLY>();
    }
}

// One row's part of the "compress L" column move of a node at column c0 split
// at n0 (both multiples of 64): the second block's L columns [c0+n0, c0+n0+r1)
// move to [c0+r0, c0+r0+r1) as the column swaps "i <-> n0 + (i - r0), from row
// i" of Section 5 leave them: a row at offset v below the first block's pivots
// moves min(v + 1, r1) columns and zeroes the vacated ones.  Words at index
// >= wlim are not read (the row's extent).
__device__ inline void shift_row(uint64_t *row, int64_t wlim, int c0, int n0, int r0, int r1,
                                 int v) {
    const int d = n0 - r0;
    const int len = min(v + 1, r1);
    const int D = c0 + r0;             // first destination bit
    const int S = c0 + n0;             // first source bit
    const int end = S + len;           // bits [D, end) change
    for (int w = D >> 6; w <= (end - 1) >> 6; w++) {
        const int p0 = w * 64;
        const int sb = p0 + d;         // source of position p0
        const int sw = sb >> 6, so = sb & 63;
        const uint64_t lo = sw < wlim ? row[sw] : 0ull;
        const uint64_t hi = (so && sw + 1 < wlim) ? row[sw + 1] : 0ull;
        const uint64_t src = so ? ((lo >> so) | (hi << (64 - so))) : lo;
        const uint64_t old = row[w];
        uint64_t mv = 0, clr = 0;
        int a = max(D, p0), e = min(D + len, p0 + 64);
        if (e > a) mv = ((e - a) == 64 ? ~0ull : ((1ull << (e - a)) - 1)) << (a - p0);
        a = max(D + len, p0);
        e = min(end, p0 + 64);
        if (e > a) clr = ((e - a) == 64 ? ~0ull : ((1ull << (e - a)) - 1)) << (a - p0);
        row[w] = (old & ~(mv | clr)) | (src & mv);
    }
}

}  // namespace gf2

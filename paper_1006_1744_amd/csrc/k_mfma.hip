// Variant M of the GF(2) product C <- C + A * Bt^T (both operands packed along
// K) on the matrix cores, result reduced mod 2, with one of two operand types:
//  * fp4 (e2m1), v_mfma_scale_f32_32x32x64_f8f6f4 with unit block scales, fp32
//    accumulation: 64 K-bits per instruction, twice the int8 rate (the default);
//  * int8, v_mfma_i32_32x32x32_i8, int32 accumulation: 32 K-bits per instruction.
//
// Exactness.  Only the parity of each sum is kept.  Every operand element is 0
// or 1 (the bit itself), so every product is 0 or 1 and each sum is the exact
// count of matching bit pairs: integers in int32, and in fp32 integers below
// 2^24 (K <= 65536 per call) with exact rounding-free sums.  A lane's 32
// K-bits w become operand elements by shifts and masks, with the same (lane
// group, register, element) -> K mapping on both operands, so the hardware
// sums each of the 64 K-bits of a word exactly once:
//  * int8: two 16-byte operands per 32 bits, register v of step s being
//    (w >> (4 s + v)) & 0x01010101, whose byte t is bit 8 t + 4 s + v of w;
//  * fp4: one 16-byte operand per 32 bits, register v holding bit 4 n + v of w
//    in nibble n, as e2m1 values whose A x B products are exactly 1 (four
//    masks and, per pair of 32-bit parts, one or two 64-bit shifts).
//
// 0/1 elements are also what keeps the clock up: the matrix cores' power grows
// with the number of toggling operand bits, and with 0/1 bytes the chip holds a
// markedly higher clock under the int8 product than with random bytes (measured
// on 32768^3: about 2.26 GHz against 1.76 GHz, 3.7 against 3.1 POP/s).

#include <type_traits>

#include "gf2_device.h"
#include "gf2_internal.h"

namespace gf2 {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

// fp4 (e2m1) operands of v_mfma_scale_f32_32x32x64_f8f6f4 from a lane's 32
// K-bits d: register v holds bit 4 n + v of d in nibble n (n = 0..7), on a
// nibble bit below the sign bit.  A set bit reads on the A side as 0.5, 1, 2, 1
// (registers 0-3: e2m1 codes 0001, 0010, 0100, 0010) and on the B side as 2, 1,
// 0.5, 1, so every product of two set bits is exactly 1 and a clear bit reads
// as 0.  The block scales are 127 (2^0) on both sides.  The shifted copies come
// from one 64-bit shift of two consecutive K steps' words (lo, hi): the bits a
// shift carries across the halves land on nibble bits the masks clear.
__device__ inline v8i g2_fp4_a(uint32_t d, uint32_t s2) {   // s2: d >> 2
    v8i f;
    f[0] = (int)(d & 0x11111111u);
    f[1] = (int)(d & 0x22222222u);
    f[2] = (int)(d & 0x44444444u);
    f[3] = (int)(s2 & 0x22222222u);
    f[4] = f[5] = f[6] = f[7] = 0;   // unused by fp4 operands
    return f;
}
__device__ inline v8i g2_fp4_b(uint32_t d, uint32_t s2, uint32_t l2) {   // l2: d << 2
    v8i f;
    f[0] = (int)(l2 & 0x44444444u);
    f[1] = (int)(d & 0x22222222u);
    f[2] = (int)(s2 & 0x11111111u);
    f[3] = (int)(s2 & 0x22222222u);
    f[4] = f[5] = f[6] = f[7] = 0;
    return f;
}
__device__ inline uint64_t g2_pair(uint32_t lo, uint32_t hi) {
    return ((uint64_t)hi << 32) | lo;
}
// one v_lshrrev_b64 / v_lshlrev_b64 (left to itself the compiler splits a 64-bit
// shift into two 32-bit instructions)
__device__ inline uint64_t g2_shr2(uint64_t x) {
    uint64_t y;
    asm("v_lshrrev_b64 %0, 2, %1" : "=v"(y) : "v"(x));
    return y;
}
__device__ inline uint64_t g2_shl2(uint64_t x) {
    uint64_t y;
    asm("v_lshlrev_b64 %0, 2, %1" : "=v"(y) : "v"(x));
    return y;
}

// Block tiles of 256 x 256 (4 x 4 MFMA tiles of 32 x 32 per wave, 256
// accumulators) or 128 x 128 (2 x 2 per wave), 2 x 2 waves, fed by direct
// global -> LDS loads (global_load_lds_dwordx4): the operand tiles never pass
// through registers, so three stages of 8 K words (512 bits) are in flight at
// once.  One load instruction fills a 1 KiB chunk of 16 tile rows x 4 word
// pairs, lane j writing slot j; slot 4 r + (p ^ h(r)) holds word pair p of chunk
// row r, with h(r) = ((r >> 1) ^ (r >> 3)) & 3, so the 16-byte LDS reads of the
// MFMA fragments (32 rows, one pair) hit distinct bank groups.  Each lane reads
// a whole word pair: lane group lg takes pair 2 q + lg in round q, and its four
// 32-bit parts feed four MFMA K steps of two register sets each.  Full stages
// only: a K tail of fewer than 8 words is staged with ordinary guarded loads
// after the pipeline has drained.  Tiles are walked in groups of 8 row tiles per
// column tile, and consecutive tiles are kept on one XCD (blocks are dealt
// round-robin over the 8 XCDs), so the operands a group shares stay in that
// XCD's L2.
constexpr int G2_KC = 8;
constexpr int G2_GROUP = 8;                // row tiles walked per column tile

__device__ inline int g2_slot(int r, int p) {
    return 4 * r + (p ^ (((r >> 1) ^ (r >> 3)) & 3));
}

// Issued as inline assembly so that the compiler neither tracks the LDS write
// nor inserts its own wait for it before every LDS read: the kernel waits for
// the load counter itself.  M0 holds the chunk's LDS byte address (one wait
// state before the load that reads it) and gets its old value back afterwards.
__device__ inline void g2_dma16(const uint64_t *src, uint32_t lds) {
    uint32_t keep;
    asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\ts_nop 0\n\t"
                 "global_load_lds_dwordx4 %1, off\n\ts_mov_b32 m0, %0"
                 : "=&s"(keep) : "v"(src), "s"(lds) : "memory");
}

// lane l of o <- the wave-uniform value v (v_writelane_b32)
__device__ inline uint32_t g2_writelane(uint32_t o, uint32_t v, int l) {
    return (uint32_t)gf2_amdgcn_writelane((int)v, l, (int)o);
}

__device__ inline uint32_t g2_lds_addr(const uint64_t *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint64_t *)p;
}

// WA x WB MFMA tiles of 32 x 32 per wave, 2 x NWN waves: (WA, WB, NWN) = (4, 2, 4)
// gives 256 x 256 block tiles with two waves on each SIMD (128 matrix registers
// each, so one wave's operand unpacking overlaps the other's matrix work),
// (2, 2, 2) gives 128 x 128 tiles with one wave per SIMD and three blocks per CU.
// The block walks its tiles' K stages as one sequence (tile i, stage s), so the
// loads of the next tile's first stages are in flight while the current tile
// finishes and writes back.
template <int WA, int WB, int NWN, int NB, bool F4>
__global__ __launch_bounds__(128 * NWN) void gemm_dma_kernel(uint64_t *C, int64_t sc,
                                                       const uint64_t *A, int64_t sa, int m,
                                                       RowRange rows, int aw, int w_lo, int nw,
                                                       const uint64_t *Bt, int64_t sbt, int nkw,
                                                       RowRange krows, int kmrows,
                                                       const int32_t *rk, int32_t *prof,
                                                       const int32_t *nwd) {
    constexpr int NW = 2 * NWN;             // waves
    constexpr int NT = 64 * NW;             // threads
    constexpr int TM = 64 * WA;             // block tile rows
    constexpr int TN = 32 * WB * NWN;       // block tile columns
    constexpr int CPWA = TM / 16 / NW;      // 1 KiB chunks per wave and stage, A
    constexpr int CPWB = TN / 16 / NW;      // the same for B
    static_assert(CPWA * 16 * NW == TM && CPWB * 16 * NW == TN, "chunks per wave");
    __shared__ __attribute__((aligned(16))) uint64_t sA[NB][TM * G2_KC];
    __shared__ __attribute__((aligned(16))) uint64_t sB[NB][TN * G2_KC];
    if (nwd) nw = min(nw, *nwd);
    int r0, r1;
    eval_range(rk, m, rows, r0, r1);
    const int M = r1 - r0;
    int k0, k1;
    eval_range(rk, kmrows, krows, k0, k1);
    if (prof && blockIdx.x == 0 && threadIdx.x == 0) {
        prof[0] = M;
        prof[1] = k1 - k0;
        prof[2] = 64 * max(nw, 0);
    }
    if (M <= 0 || nw <= 0) return;
    nkw = min(nkw, (k1 - k0 + 63) / 64);
    if (nkw <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave & 1, wn = wave >> 1;
    const int li = lane & 31, lg = lane >> 5;
    const int tiles_m = (M + TM - 1) / TM;
    const int ncol = nw * 64;
    const int tiles_n = (ncol + TN - 1) / TN;
    const int ntiles = tiles_m * tiles_n;
    const int nfull = nkw / G2_KC;
    const bool ktail = nkw % G2_KC != 0;
    const int nstage = nfull + (ktail ? 1 : 0);
    const int per = gridDim.x / 8;
    const int vid = (gridDim.x % 8 == 0) ? (blockIdx.x % 8) * per + blockIdx.x / 8 : blockIdx.x;
    const int ntb = vid < ntiles ? (ntiles - 1 - vid) / (int)gridDim.x + 1 : 0;
    const int nsteps = ntb * nstage;
    // loader role: chunks CPW wave + c of each operand; lane -> (chunk row, pair)
    const int lr = lane >> 2;
    const int lp = (lane & 3) ^ (((lr >> 1) ^ (lr >> 3)) & 3);
    // reader role: word offset of the slot of pair 2 q + lg of this lane's row
    // in row group t (the swizzle is an XOR, so each round has its own offset)
    int offa[2][WA], offb[2][WB];
#pragma unroll
    for (int q = 0; q < 2; q++) {
#pragma unroll
        for (int t = 0; t < WA; t++) {
            const int ra = wm * (32 * WA) + t * 32 + li;
            offa[q][t] = (ra >> 4) * 128 + 2 * g2_slot(ra & 15, 2 * q + lg);
        }
#pragma unroll
        for (int t = 0; t < WB; t++) {
            const int rb = wn * (32 * WB) + t * 32 + li;
            offb[q][t] = (rb >> 4) * 128 + 2 * g2_slot(rb & 15, 2 * q + lg);
        }
    }
    // tile i of this block -> first row and first column word (groups of 8 row
    // tiles per column tile)
    auto tile_at = [&](int i, int &row0, int &cw0) {
        const int tile = vid + i * (int)gridDim.x;
        const int grp = tile / (G2_GROUP * tiles_n);
        const int gsz = min(G2_GROUP, tiles_m - grp * G2_GROUP);
        const int in = tile % (G2_GROUP * tiles_n);
        row0 = r0 + (grp * G2_GROUP + in % gsz) * TM;
        cw0 = (in / gsz) * (TN / 64);
    };
    // DMA cursor: the next step to load is stage n_st of tile n_i, into buffer
    // n_buf; pa / pb hold the tile's per-lane row pointers (rows past the matrix
    // edge load a clamped, valid row, whose outputs are never stored).  Advanced
    // step by step, so no division runs in the stage loop.
    int n_i = 0, n_st = 0, n_buf = 0;
    const uint64_t *pa[CPWA], *pb[CPWB];
    auto cursor_tile = [&]() {
        int row0, cw0;
        tile_at(n_i, row0, cw0);
#pragma unroll
        for (int c = 0; c < CPWA; c++) {
            const int tr = 16 * (CPWA * wave + c) + lr;
            pa[c] = A + (int64_t)min(row0 + tr, r1 - 1) * sa + aw + 2 * lp;
        }
#pragma unroll
        for (int c = 0; c < CPWB; c++) {
            const int tr = 16 * (CPWB * wave + c) + lr;
            pb[c] = Bt + (int64_t)min(cw0 * 64 + tr, ncol - 1) * sbt + 2 * lp;
        }
    };
    if (ntb > 0) cursor_tile();
    // issue the cursor's step (a full stage; a tail stage is staged later by
    // ordinary loads) and advance the cursor
    auto issue_next = [&]() {
        if (!(ktail && n_st == nstage - 1)) {
            const uint32_t la = g2_lds_addr(&sA[n_buf][wave * CPWA * 128]);
            const uint32_t lb = g2_lds_addr(&sB[n_buf][wave * CPWB * 128]);
#pragma unroll
            for (int c = 0; c < CPWA; c++) g2_dma16(pa[c] + n_st * G2_KC, la + 1024 * c);
#pragma unroll
            for (int c = 0; c < CPWB; c++) g2_dma16(pb[c] + n_st * G2_KC, lb + 1024 * c);
        }
        n_buf = n_buf == NB - 1 ? 0 : n_buf + 1;
        if (++n_st == nstage) {
            n_st = 0;
            if (++n_i < ntb) cursor_tile();
        }
    };
    typedef typename std::conditional<F4, v16f, v16i>::type acc_t;
    acc_t acc[WA][WB];
    // one round: the MFMAs of the word pairs (xa, xb) a lane read for round q
    auto compute_round = [&](const v4i *xa, const v4i *xb) {
        if constexpr (F4) {
            // one fp4 MFMA (64 K-bits over both lane groups) per 32-bit part; the
            // shifts run on pairs of parts
#pragma unroll
            for (int h = 0; h < 2; h++) {
                uint64_t sa2[WA], sb2[WB], lb2[WB];
#pragma unroll
                for (int t = 0; t < WA; t++)
                    sa2[t] = g2_shr2(g2_pair((uint32_t)xa[t][2 * h], (uint32_t)xa[t][2 * h + 1]));
#pragma unroll
                for (int t = 0; t < WB; t++) {
                    const uint64_t pb = g2_pair((uint32_t)xb[t][2 * h], (uint32_t)xb[t][2 * h + 1]);
                    sb2[t] = g2_shr2(pb);
                    lb2[t] = g2_shl2(pb);
                }
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    const int u = 2 * h + j;
                    v8i fa[WA], fb[WB];
#pragma unroll
                    for (int t = 0; t < WA; t++)
                        fa[t] = g2_fp4_a((uint32_t)xa[t][u], (uint32_t)(sa2[t] >> (32 * j)));
#pragma unroll
                    for (int t = 0; t < WB; t++)
                        fb[t] = g2_fp4_b((uint32_t)xb[t][u], (uint32_t)(sb2[t] >> (32 * j)),
                                         (uint32_t)(lb2[t] >> (32 * j)));
#pragma unroll
                    for (int a = 0; a < WA; a++)
#pragma unroll
                        for (int b = 0; b < WB; b++)
                            acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                                fa[a], fb[b], acc[a][b], 4, 4, 0, 127, 0, 127);
                }
            }
        } else {
            // two int8 MFMAs (32 K-bits each) per 32-bit part
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int s = 0; s < 2; s++) {
                    v4i fa[WA], fb[WB];
#pragma unroll
                    for (int v = 0; v < 4; v++) {
#pragma unroll
                        for (int t = 0; t < WA; t++)
                            fa[t][v] = (int)(((uint32_t)xa[t][u] >> (4 * s + v)) & 0x01010101u);
#pragma unroll
                        for (int t = 0; t < WB; t++)
                            fb[t][v] = (int)(((uint32_t)xb[t][u] >> (4 * s + v)) & 0x01010101u);
                    }
#pragma unroll
                    for (int a = 0; a < WA; a++)
#pragma unroll
                        for (int b = 0; b < WB; b++)
                            acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b],
                                                                             acc[a][b], 0, 0, 0);
                }
        }
    };
    auto read_round = [&](int b, int q, v4i *xa, v4i *xb) {
#pragma unroll
        for (int t = 0; t < WA; t++) xa[t] = *reinterpret_cast<const v4i *>(&sA[b][offa[q][t]]);
#pragma unroll
        for (int t = 0; t < WB; t++) xb[t] = *reinterpret_cast<const v4i *>(&sB[b][offb[q][t]]);
    };
    // Make step gn's operands visible to every wave (step gn is stage sn of tile
    // tn).  Before the call each wave has issued all its LDS reads of step gn - 1
    // and DMA up to step gn + 1.
    //  * full stage: this wave's DMA of step gn has landed once at most step
    //    gn + 1's is in flight; after the barrier every wave's has, and every wave
    //    has read step gn - 1 (the lgkmcnt wait), so step gn + 2 may reuse its
    //    buffer.
    //  * tail stage: drain, then stage the tail words (zero past the end) with
    //    ordinary loads into the same slot layout; buffer gn % 3 was last read at
    //    step gn - 3 and no DMA targets it.
    auto arrive = [&](int gn, int sn, int tn) {
        const int b = gn % NB;
        if (ktail && sn == nstage - 1) {
            asm volatile("s_waitcnt vmcnt(0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
            int row0, cw0;
            tile_at(tn, row0, cw0);
            const int kb = nfull * G2_KC;
            for (int e = tid; e < TM * 4; e += NT) {
                const int tr = e >> 2, p = e & 3;
                const int slot = (tr >> 4) * 128 + 2 * g2_slot(tr & 15, p);
                const int arow = row0 + tr;
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const int kw = kb + 2 * p + h;
                    sA[b][slot + h] = (arow < r1 && kw < nkw) ? A[(int64_t)arow * sa + aw + kw] : 0ull;
                }
            }
            for (int e = tid; e < TN * 4; e += NT) {
                const int tr = e >> 2, p = e & 3;
                const int slot = (tr >> 4) * 128 + 2 * g2_slot(tr & 15, p);
                const int brow = cw0 * 64 + tr;
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const int kw = kb + 2 * p + h;
                    sB[b][slot + h] = (brow < ncol && kw < nkw) ? Bt[(int64_t)brow * sbt + kw] : 0ull;
                }
            }
            __syncthreads();
            return;
        }
        // is step gn + 1 a DMA stage (issued, possibly still in flight)?
        const bool next_full = gn + 1 < nsteps &&
                               !(ktail && (sn + 1 < nstage ? sn + 2 == nstage : nstage == 1));
        if (next_full) {
            static_assert(CPWA + CPWB == 8 || CPWA + CPWB == 4, "DMA loads per wave and step");
            if constexpr (CPWA + CPWB == 8)
                asm volatile("s_waitcnt vmcnt(8)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
            else
                asm volatile("s_waitcnt vmcnt(4)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        } else {
            asm volatile("s_waitcnt vmcnt(0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        }
    };
    // Software pipeline over the flat step sequence: step g's round-1 reads are
    // issued before its round-0 MFMAs, and step g + 1 is made visible (and its
    // round-0 reads issued) between step g's two rounds, so the LDS latency and
    // the barrier overlap matrix-core work instead of opening each round.
    static_assert(NB == 3, "three stages in flight");
    v4i xa0[WA], xb0[WB], xa1[WA], xb1[WB];
#pragma unroll
    for (int gi = 0; gi < NB - 1; gi++)
        if (gi < nsteps) issue_next();
    if (nsteps > 0) {
        arrive(0, 0, 0);
        if (NB - 1 < nsteps) issue_next();
        read_round(0, 0, xa0, xb0);
    }
    int g = 0;
    for (int i = 0; i < ntb; i++) {
#pragma unroll
        for (int a = 0; a < WA; a++)
#pragma unroll
            for (int b = 0; b < WB; b++)
#pragma unroll
                for (int v = 0; v < 16; v++) {
                    // one matrix-register write per element (a float zero vector
                    // would otherwise be kept in spare matrix registers and copied)
                    asm volatile("v_accvgpr_write_b32 %0, 0" : "=a"(acc[a][b][v]));
                }
        for (int st = 0; st < nstage; st++, g++) {
            read_round(g % NB, 1, xa1, xb1);
            compute_round(xa0, xb0);
            // keep round 0's matrix work ahead of the next stage's barrier, so the
            // next stage's first LDS reads overlap round 1 (left alone, the
            // compiler sinks round 0 below the barrier)
#pragma unroll
            for (int a = 0; a < WA; a++)
#pragma unroll
                for (int b = 0; b < WB; b++) asm volatile("" : "+a"(acc[a][b]));
            if (g + 1 < nsteps) {
                const bool same = st + 1 < nstage;
                arrive(g + 1, same ? st + 1 : 0, same ? i : i + 1);
                if (g + NB < nsteps) issue_next();
                read_round((g + 1) % NB, 0, xa0, xb0);
            }
            compute_round(xa1, xb1);
        }
        {
            // bit 0 of each sum -> packed words.  A ballot over one accumulator
            // register gives 32 columns of two rows (lanes 0-31: row rlo, lanes
            // 32-63: row rlo + 4); each half is written straight into the lane that
            // stores that row.  Lane L ends up with rows 64 h + L of the wave's rows,
            // words q of its columns, every 32-bit half written once.
            uint32_t ow[WA / 2][WB / 2][2] = {};
            // the reads below are assembly, so the wait states a matrix-register
            // read needs after the MFMA that wrote it are placed here by hand
            asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
#pragma unroll
            for (int a = 0; a < WA; a++)
#pragma unroll
                for (int b = 0; b < WB; b++)
#pragma unroll
                    for (int v = 0; v < 16; v++) {
                        // read one matrix register at a time (left to itself the
                        // compiler copies all 256 out at once, which spills)
                        int x;
                        asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(x) : "a"(acc[a][b][v]));
                        if constexpr (F4) x = (int)__builtin_bit_cast(float, x);   // exact count
                        const uint64_t bal = __ballot(x & 1);
                        const int rlo = 32 * (a & 1) + 8 * (v >> 2) + (v & 3);
                        uint32_t &o = ow[a >> 1][b >> 1][b & 1];
                        o = g2_writelane(o, (uint32_t)bal, rlo);
                        o = g2_writelane(o, (uint32_t)(bal >> 32), rlo + 4);
                    }
            int row0, cw0;
            tile_at(i, row0, cw0);
#pragma unroll
            for (int h = 0; h < WA / 2; h++) {
                const int grow = row0 + wm * (32 * WA) + h * 64 + lane;
#pragma unroll
                for (int q = 0; q < WB / 2; q++) {
                    const uint64_t out = (uint64_t)ow[h][q][0] | ((uint64_t)ow[h][q][1] << 32);
                    const int cw = cw0 + wn * (WB / 2) + q;
                    if (grow < r1 && cw < nw && out) {
                        uint64_t *pc = C + (int64_t)grow * sc + w_lo + cw;
                        *pc ^= out;
                    }
                }
            }
        }
    }
}

hipError_t launch_gemm_mfma(uint64_t *C, int64_t sc, const uint64_t *A, int64_t sa, int m,
                            RowRange rows, int aw, int w_lo, int nw, const uint64_t *Bt,
                            int64_t sbt, int kmax, RowRange krows, int kmrows, const int32_t *rk,
                            int32_t *prof, bool fp4, hipStream_t st, const int32_t *nwd) {
    int nkw = (kmax + 63) / 64;
    if (nw <= 0 || nkw <= 0) return hipSuccess;
    // 256 x 256 tiles pay off once the inner dimension is long enough to
    // amortize their larger prologue and epilogue (from K = 2048 on the 65536^2
    // recursion); shorter products use 128 x 128 tiles
    if (nw >= 4 && kmax > 1024) {
        // persistent: one block of eight waves per CU (two per SIMD, 128 matrix
        // registers each), each block walking its tiles' stages as one pipeline
        int64_t tiles = (int64_t)((m + 255) / 256) * ((nw * 64 + 255) / 256);
        int64_t blocks = tiles < 256 ? tiles : 256;
        if (blocks >= 8) blocks = blocks / 8 * 8;
        if (blocks < 1) blocks = 1;
        if (fp4)
            hipLaunchKernelGGL((gemm_dma_kernel<4, 2, 4, 3, true>), dim3((unsigned)blocks), dim3(512), 0, st, C,
                               sc, A, sa, m, rows, aw, w_lo, nw, Bt, sbt, nkw, krows, kmrows, rk, prof, nwd);
        else
            hipLaunchKernelGGL((gemm_dma_kernel<4, 2, 4, 3, false>), dim3((unsigned)blocks), dim3(512), 0, st, C,
                               sc, A, sa, m, rows, aw, w_lo, nw, Bt, sbt, nkw, krows, kmrows, rk, prof, nwd);
        return hipGetLastError();
    }
    // three blocks per CU (48 KiB of LDS each)
    int64_t tiles = (int64_t)((m + 127) / 128) * ((nw * 64 + 127) / 128);
    int64_t blocks = tiles < 768 ? tiles : 768;
    if (blocks >= 8) blocks = blocks / 8 * 8;
    if (blocks < 1) blocks = 1;
    if (fp4)
        hipLaunchKernelGGL((gemm_dma_kernel<2, 2, 2, 3, true>), dim3((unsigned)blocks), dim3(256), 0, st, C, sc,
                           A, sa, m, rows, aw, w_lo, nw, Bt, sbt, nkw, krows, kmrows, rk, prof, nwd);
    else
        hipLaunchKernelGGL((gemm_dma_kernel<2, 2, 2, 3, false>), dim3((unsigned)blocks), dim3(256), 0, st, C, sc,
                           A, sa, m, rows, aw, w_lo, nw, Bt, sbt, nkw, krows, kmrows, rk, prof, nwd);
    return hipGetLastError();
}

}  // namespace gf2

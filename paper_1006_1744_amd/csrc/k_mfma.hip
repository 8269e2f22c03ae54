// Variant M of the GF(2) product C <- C + A * Bt^T (both operands packed along
// K): int8 matrix cores (v_mfma_i32_32x32x32_i8), int32 accumulation, result
// reduced mod 2.
//
// Exactness.  Only the parity of the int32 sum is kept.  For integers a, b the
// product's parity is (a mod 2)(b mod 2), so every operand byte only has to
// carry the wanted bit in its least significant position.  A lane's 32 K-bits w
// therefore become two 16-byte MFMA operands: register v of step s is
// (w >> (4 s + v)) & 0x01010101, whose byte t is bit 8 t + 4 s + v of w.  Both
// operands use the same (lane group, byte) -> K mapping, so the hardware sums
// each of the 64 K-bits of a word exactly once.  Sums stay below K <= 65536 per
// call, far from int32 overflow.
//
// The mask is not needed for the parity (bits above a byte's LSB never reach
// the LSB of a product) but for the clock: the matrix cores' power grows with
// the number of toggling operand bits, and with 0/1 bytes the chip holds a
// markedly higher clock under this load than with random bytes (measured on
// 32768^3: about 2.26 GHz against 1.76 GHz, 3.7 against 3.1 POP/s).

#include "gf2_internal.h"

namespace gf2 {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int GM_TM = 128;      // rows per block tile
constexpr int GM_TN = 128;      // columns per block tile (2 words)
constexpr int GM_KC = 8;        // K words staged per step
constexpr int GM_LD = GM_KC + 1;

__global__ __launch_bounds__(256) void gemm_mfma_kernel(uint64_t *C, int64_t sc,
                                                        const uint64_t *A, int64_t sa, int m,
                                                        RowRange rows, int aw, int w_lo, int nw,
                                                        const uint64_t *Bt, int64_t sbt, int nkw,
                                                        RowRange krows, int kmrows,
                                                        const int32_t *rk, int32_t *prof) {
    __shared__ uint64_t sA[GM_TM][GM_LD];
    __shared__ uint64_t sB[GM_TN][GM_LD];
    int r0, r1;
    eval_range(rk, m, rows, r0, r1);
    const int M = r1 - r0;
    int k0, k1;
    eval_range(rk, kmrows, krows, k0, k1);
    if (prof && blockIdx.x == 0 && threadIdx.x == 0) {
        prof[0] = M;
        prof[1] = k1 - k0;
    }
    if (M <= 0) return;
    nkw = min(nkw, (k1 - k0 + 63) / 64);
    if (nkw <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;          // 2 x 2 waves, 64 x 64 each
    const int li = lane & 31, lg = lane >> 5;         // row in block, K half
    const int tiles_m = (M + GM_TM - 1) / GM_TM;
    const int tiles_n = (nw * 64 + GM_TN - 1) / GM_TN;
    const int ntiles = tiles_m * tiles_n;
    const uint32_t *sA32 = reinterpret_cast<const uint32_t *>(&sA[0][0]);
    const uint32_t *sB32 = reinterpret_cast<const uint32_t *>(&sB[0][0]);
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int tm = tile % tiles_m, tn = tile / tiles_m;
        const int row0 = r0 + tm * GM_TM;
        const int cw0 = tn * (GM_TN / 64);
        v16i acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int v = 0; v < 16; v++) acc[a][b][v] = 0;
        for (int kc = 0; kc < nkw; kc += GM_KC) {
            __syncthreads();
            for (int e = tid; e < GM_TM * GM_KC; e += 256) {
                int rr = e / GM_KC, w = e % GM_KC;
                int grow = row0 + rr;
                sA[rr][w] = (grow < r1 && kc + w < nkw) ? A[(int64_t)grow * sa + aw + kc + w] : 0ull;
            }
            for (int e = tid; e < GM_TN * GM_KC; e += 256) {
                int rr = e / GM_KC, w = e % GM_KC;
                int brow = cw0 * 64 + rr;
                sB[rr][w] = (brow < nw * 64 && kc + w < nkw) ? Bt[(int64_t)brow * sbt + kc + w] : 0ull;
            }
            __syncthreads();
            const int kend = min(GM_KC, nkw - kc);
            for (int w = 0; w < kend; w++) {
                uint32_t wa[2], wb[2];
#pragma unroll
                for (int t = 0; t < 2; t++) {
                    wa[t] = sA32[((wm * 64 + t * 32 + li) * GM_LD + w) * 2 + lg];
                    wb[t] = sB32[((wn * 64 + t * 32 + li) * GM_LD + w) * 2 + lg];
                }
#pragma unroll
                for (int s = 0; s < 2; s++) {
                    v4i fa[2], fb[2];
#pragma unroll
                    for (int t = 0; t < 2; t++) {
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            fa[t][v] = (int)((wa[t] >> (4 * s + v)) & 0x01010101u);
                            fb[t][v] = (int)((wb[t] >> (4 * s + v)) & 0x01010101u);
                        }
                    }
#pragma unroll
                    for (int a = 0; a < 2; a++)
#pragma unroll
                        for (int b = 0; b < 2; b++)
                            acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b],
                                                                             acc[a][b], 0, 0, 0);
                }
            }
        }
        // bit 0 of each sum; lane L collects the C word of row L of the wave tile.
        // Output layout of the 32x32 MFMA: lane l holds column l % 32 and, in
        // register v, row 8 (v / 4) + 4 (l / 32) + v % 4.
        uint64_t word = 0;
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int v = 0; v < 16; v++) {
                    uint64_t bal = __ballot(acc[a][b][v] & 1);
                    const int rlo = a * 32 + 8 * (v >> 2) + (v & 3);
                    const uint64_t flo = (bal & 0xFFFFFFFFull) << (32 * b);
                    const uint64_t fhi = (bal >> 32) << (32 * b);
                    if (lane == rlo) word |= flo;
                    if (lane == rlo + 4) word |= fhi;
                }
        const int grow = row0 + wm * 64 + lane;
        const int cw = cw0 + wn;
        if (grow < r1 && cw < nw && word) {
            uint64_t *pc = C + (int64_t)grow * sc + w_lo + cw;
            *pc ^= word;
        }
    }
}

// Large-tile variant: 256 x 256 outputs per block, 128 x 128 per wave (4 x 4
// MFMA tiles, 256 accumulators), fed by direct global -> LDS loads
// (global_load_lds_dwordx4): the operand tiles never pass through registers, so
// three stages of 8 K words (512 bits) are in flight at once.  One load
// instruction fills a 1 KiB chunk of 16 tile rows x 4 word pairs, lane j writing
// slot j; slot 4 r + (p ^ h(r)) holds word pair p of chunk row r, with
// h(r) = ((r >> 1) ^ (r >> 3)) & 3, so the 16-byte LDS reads of the MFMA
// fragments (32 rows, one pair) hit distinct bank groups.  Each lane reads a
// whole word pair: lane group lg takes pair 2 q + lg in round q, and its four
// 32-bit parts feed four MFMA K steps of two register sets each.  Full stages
// only: a K tail of fewer than 8 words is staged with ordinary guarded loads
// after the pipeline has drained.  Tiles are walked in groups of 8 row tiles
// per column tile, and consecutive tiles are kept on one XCD (blocks are dealt
// round-robin over the 8 XCDs), so the operands a group shares stay in that
// XCD's L2.
constexpr int G2_TM = 256;
constexpr int G2_TN = 256;
constexpr int G2_KC = 8;
constexpr int G2_NBUF = 3;
constexpr int G2_GROUP = 8;                // row tiles walked per column tile
constexpr int G2_STAGE = G2_TM * G2_KC;   // words per operand per stage (16 KiB)

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

// v_writelane_b32 (the LLVM intrinsic, so that the compiler places the wait
// states a lane write needs after the compare that produced its value): the
// wave-uniform value v replaces lane l of o.
extern "C" __device__ int gf2_amdgcn_writelane(int v, int lane, int old)
    __asm("llvm.amdgcn.writelane.i32");

__device__ inline uint32_t g2_writelane(uint32_t o, uint32_t v, int l) {
    return (uint32_t)gf2_amdgcn_writelane((int)v, l, (int)o);
}

__device__ inline uint32_t g2_lds_addr(const uint64_t *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint64_t *)p;
}

__global__ __launch_bounds__(256) void gemm_mfma2_kernel(uint64_t *C, int64_t sc,
                                                         const uint64_t *A, int64_t sa, int m,
                                                         RowRange rows, int aw, int w_lo, int nw,
                                                         const uint64_t *Bt, int64_t sbt, int nkw,
                                                         RowRange krows, int kmrows,
                                                         const int32_t *rk, int32_t *prof) {
    __shared__ __attribute__((aligned(16))) uint64_t sA[G2_NBUF][G2_STAGE];
    __shared__ __attribute__((aligned(16))) uint64_t sB[G2_NBUF][G2_STAGE];
    int r0, r1;
    eval_range(rk, m, rows, r0, r1);
    const int M = r1 - r0;
    int k0, k1;
    eval_range(rk, kmrows, krows, k0, k1);
    if (prof && blockIdx.x == 0 && threadIdx.x == 0) {
        prof[0] = M;
        prof[1] = k1 - k0;
    }
    if (M <= 0) return;
    nkw = min(nkw, (k1 - k0 + 63) / 64);
    if (nkw <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int li = lane & 31, lg = lane >> 5;
    const int tiles_m = (M + G2_TM - 1) / G2_TM;
    const int ncol = nw * 64;
    const int tiles_n = (ncol + G2_TN - 1) / G2_TN;
    const int ntiles = tiles_m * tiles_n;
    const int nfull = nkw / G2_KC;
    const int ktail = nkw - nfull * G2_KC;
    // loader role: chunks 4 wave + i (i < 4) of each operand; lane -> (row, pair)
    const int lr = lane >> 2;
    const int lp = (lane & 3) ^ (((lr >> 1) ^ (lr >> 3)) & 3);
    // reader role: word offset of the slot of pair 2 q + lg of this lane's row
    // in row group t (the swizzle is an XOR, so each round has its own offset)
    int offa[2][4], offb[2][4];
#pragma unroll
    for (int q = 0; q < 2; q++)
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int ra = wm * 128 + t * 32 + li, rb = wn * 128 + t * 32 + li;
            offa[q][t] = (ra >> 4) * 128 + 2 * g2_slot(ra & 15, 2 * q + lg);
            offb[q][t] = (rb >> 4) * 128 + 2 * g2_slot(rb & 15, 2 * q + lg);
        }
    const int per = gridDim.x / 8;
    const int vid = (gridDim.x % 8 == 0) ? (blockIdx.x % 8) * per + blockIdx.x / 8 : blockIdx.x;
    for (int tile = vid; tile < ntiles; tile += gridDim.x) {
        const int grp = tile / (G2_GROUP * tiles_n);
        const int gsz = min(G2_GROUP, tiles_m - grp * G2_GROUP);
        const int in = tile % (G2_GROUP * tiles_n);
        const int tm = grp * G2_GROUP + in % gsz;
        const int tn = in / gsz;
        const int row0 = r0 + tm * G2_TM;
        const int cw0 = tn * (G2_TN / 64);
        // rows past the matrix edge load a clamped (valid) row; their outputs are
        // never stored
        const uint64_t *pa[4], *pb[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int tr = 16 * (4 * wave + i) + lr;
            const int arow = min(row0 + tr, r1 - 1);
            const int brow = min(cw0 * 64 + tr, ncol - 1);
            pa[i] = A + (int64_t)arow * sa + aw + 2 * lp;
            pb[i] = Bt + (int64_t)brow * sbt + 2 * lp;
        }
        auto dma = [&](int st) {
            const int buf = st % G2_NBUF;
            const uint32_t la = __builtin_amdgcn_readfirstlane(g2_lds_addr(&sA[buf][wave * 512]));
            const uint32_t lb = __builtin_amdgcn_readfirstlane(g2_lds_addr(&sB[buf][wave * 512]));
#pragma unroll
            for (int i = 0; i < 4; i++) {
                g2_dma16(pa[i] + st * G2_KC, la + 1024 * i);
                g2_dma16(pb[i] + st * G2_KC, lb + 1024 * i);
            }
        };
        v16i acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++)
#pragma unroll
                for (int v = 0; v < 16; v++) acc[a][b][v] = 0;
        auto compute = [&](int buf) {
#pragma unroll
            for (int q = 0; q < 2; q++) {
                v4i xa[4], xb[4];
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    xa[t] = *reinterpret_cast<const v4i *>(&sA[buf][offa[q][t]]);
                    xb[t] = *reinterpret_cast<const v4i *>(&sB[buf][offb[q][t]]);
                }
#pragma unroll
                for (int u = 0; u < 4; u++)
#pragma unroll
                    for (int s = 0; s < 2; s++) {
                        v4i fa[4], fb[4];
#pragma unroll
                        for (int t = 0; t < 4; t++)
#pragma unroll
                            for (int v = 0; v < 4; v++) {
                                fa[t][v] = (int)(((uint32_t)xa[t][u] >> (4 * s + v)) & 0x01010101u);
                                fb[t][v] = (int)(((uint32_t)xb[t][u] >> (4 * s + v)) & 0x01010101u);
                            }
#pragma unroll
                        for (int a = 0; a < 4; a++)
#pragma unroll
                            for (int b = 0; b < 4; b++)
                                acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b],
                                                                                 acc[a][b], 0, 0, 0);
                    }
            }
        };
        __syncthreads();   // the previous tile's last reads are done
#pragma unroll
        for (int s = 0; s < G2_NBUF - 1; s++)
            if (s < nfull) dma(s);
        for (int st = 0; st < nfull; st++) {
            // this wave's loads of stage st have landed (those of stage st + 1, 8
            // instructions, may still be in flight); after the barrier every
            // wave's have, and buffer (st + 2) % 3 is no longer read
            if (st + 1 < nfull)
                asm volatile("s_waitcnt vmcnt(8)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
            else
                asm volatile("s_waitcnt vmcnt(0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
            if (st + G2_NBUF - 1 < nfull) dma(st + G2_NBUF - 1);
            compute(st % G2_NBUF);
        }
        if (ktail) {
            // the pipeline is drained (the last full stage waited for vmcnt 0);
            // wait for every wave to leave the buffer, then stage the tail words
            // (zero past the end) with ordinary loads into the same slot layout
            const int buf = nfull % G2_NBUF;
            __syncthreads();
            const int kb = nfull * G2_KC;
            for (int e = tid; e < G2_TM * 4; e += 256) {
                const int tr = e >> 2, p = e & 3;
                const int slot = (tr >> 4) * 128 + 2 * g2_slot(tr & 15, p);
                const int arow = row0 + tr, brow = cw0 * 64 + tr;
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const int kw = kb + 2 * p + h;
                    sA[buf][slot + h] = (arow < r1 && kw < nkw) ? A[(int64_t)arow * sa + aw + kw] : 0ull;
                    sB[buf][slot + h] = (brow < ncol && kw < nkw) ? Bt[(int64_t)brow * sbt + kw] : 0ull;
                }
            }
            __syncthreads();
            compute(buf);
        }
        // bit 0 of each sum -> packed words.  A ballot over one accumulator
        // register gives 32 columns of two rows (lanes 0-31: row rlo, lanes 32-63:
        // row rlo + 4); each half is written straight into the lane that stores
        // that row.  Lane L ends up with rows L and 64 + L of the wave's 128 rows,
        // words 0 and 1 of its 128 columns, every 32-bit half written once.
        uint32_t ow[2][2][2] = {};
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++)
#pragma unroll
                for (int v = 0; v < 16; v++) {
                    const uint64_t bal = __ballot(acc[a][b][v] & 1);
                    const int rlo = 32 * (a & 1) + 8 * (v >> 2) + (v & 3);
                    uint32_t &o = ow[a >> 1][b >> 1][b & 1];
                    o = g2_writelane(o, (uint32_t)bal, rlo);
                    o = g2_writelane(o, (uint32_t)(bal >> 32), rlo + 4);
                }
        uint64_t out[2][2];
#pragma unroll
        for (int h = 0; h < 2; h++)
#pragma unroll
            for (int q = 0; q < 2; q++)
                out[h][q] = (uint64_t)ow[h][q][0] | ((uint64_t)ow[h][q][1] << 32);
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int grow = row0 + wm * 128 + h * 64 + lane;
#pragma unroll
            for (int q = 0; q < 2; q++) {
                const int cw = cw0 + wn * 2 + q;
                if (grow < r1 && cw < nw && out[h][q]) {
                    uint64_t *pc = C + (int64_t)grow * sc + w_lo + cw;
                    *pc ^= out[h][q];
                }
            }
        }
    }
}

hipError_t launch_gemm_mfma(uint64_t *C, int64_t sc, const uint64_t *A, int64_t sa, int m,
                            RowRange rows, int aw, int w_lo, int nw, const uint64_t *Bt,
                            int64_t sbt, int kmax, RowRange krows, int kmrows, const int32_t *rk,
                            int32_t *prof, hipStream_t st) {
    int nkw = (kmax + 63) / 64;
    if (nw <= 0 || nkw <= 0) return hipSuccess;
    // 256 x 256 tiles pay off once the inner dimension is long enough to hide
    // their larger prologue and epilogue (measured on the 65536^2 recursion:
    // K = 4096 runs 8% faster on them, K = 2048 26% slower); shorter products
    // use the 128 x 128 kernel
    if (nw >= 4 && kmax > 2048) {
        int64_t tiles = (int64_t)((m + G2_TM - 1) / G2_TM) * ((nw * 64 + G2_TN - 1) / G2_TN);
        int64_t blocks = tiles < 1024 ? tiles : 1024;
        if (blocks >= 8) blocks = blocks / 8 * 8;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(gemm_mfma2_kernel, dim3((unsigned)blocks), dim3(256), 0, st, C, sc, A, sa,
                           m, rows, aw, w_lo, nw, Bt, sbt, nkw, krows, kmrows, rk, prof);
        return hipGetLastError();
    }
    int64_t tiles = (int64_t)((m + GM_TM - 1) / GM_TM) * ((nw * 64 + GM_TN - 1) / GM_TN);
    int64_t blocks = tiles < 2048 ? tiles : 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(gemm_mfma_kernel, dim3((unsigned)blocks), dim3(256), 0, st, C, sc, A, sa, m,
                       rows, aw, w_lo, nw, Bt, sbt, nkw, krows, kmrows, rk, prof);
    return hipGetLastError();
}

}  // namespace gf2

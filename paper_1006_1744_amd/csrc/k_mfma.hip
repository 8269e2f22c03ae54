// Variant M of the GF(2) product C <- C + A * Bt^T (both operands packed along
// K): int8 matrix cores (v_mfma_i32_32x32x32_i8), int32 accumulation, result
// reduced mod 2.
//
// Exactness.  Only the parity of the int32 sum is kept.  For integers a, b the
// product's parity is (a mod 2)(b mod 2), so every operand byte only has to
// carry the wanted bit in its least significant position; the other seven bits
// may hold anything.  A lane's 32 K-bits w therefore become two 16-byte MFMA
// operands with seven shifts: register v of step s is w >> (4 s + v), whose byte
// t carries bit 8 t + 4 s + v of w in its LSB.  Both operands use the same
// (lane group, byte) -> K mapping, so the hardware sums each of the 64 K-bits of
// a word exactly once.  |a b| <= 128 * 128 and K <= 65536 per call keep the
// int32 sum far from overflow, and two's complement parity is the LSB anyway.

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
                            fa[t][v] = (int)(wa[t] >> (4 * s + v));
                            fb[t][v] = (int)(wb[t] >> (4 * s + v));
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
// MFMA tiles, 256 accumulators), K staged 8 words (512 bits) at a time through
// double-buffered LDS with the next stage's global loads in flight during the
// current stage's MFMAs.  Tiles are walked in groups of 8 row-tiles per column
// tile, and consecutive tiles are kept on one XCD (blocks are dealt round-robin
// over the 8 XCDs), so the operands a group shares stay in that XCD's L2.
constexpr int G2_TM = 256;
constexpr int G2_TN = 256;
constexpr int G2_KC = 8;                    // K words per stage
constexpr int G2_LD = 2 * G2_KC + 2;        // u32 per LDS row (padded, 8-byte aligned)
constexpr int G2_GROUP = 8;

__global__ __launch_bounds__(256) void gemm_mfma2_kernel(uint64_t *C, int64_t sc,
                                                         const uint64_t *A, int64_t sa, int m,
                                                         RowRange rows, int aw, int w_lo, int nw,
                                                         const uint64_t *Bt, int64_t sbt, int nkw,
                                                         RowRange krows, int kmrows,
                                                         const int32_t *rk, int32_t *prof) {
    __shared__ uint32_t sA[2][G2_TM * G2_LD];
    __shared__ uint32_t sB[2][G2_TN * G2_LD];
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
    const int tiles_n = (nw * 64 + G2_TN - 1) / G2_TN;
    const int ntiles = tiles_m * tiles_n;
    const int nstage = (nkw + G2_KC - 1) / G2_KC;
    // XCD-contiguous virtual block id
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
        // cooperative loads: element e = tid + 256 i is word e % KC of tile row e / KC,
        // so KC consecutive lanes read one row's KC words (one 64-byte segment)
        uint64_t ra[G2_KC], rb[G2_KC];
        auto gload = [&](int st) {
#pragma unroll
            for (int i = 0; i < G2_KC; i++) {
                const int e = tid + 256 * i;
                const int rr = e / G2_KC, w = e % G2_KC;
                const int kw = st * G2_KC + w;
                const int arow = row0 + rr;
                const int brow = cw0 * 64 + rr;
                ra[i] = (arow < r1 && kw < nkw) ? A[(int64_t)arow * sa + aw + kw] : 0ull;
                rb[i] = (brow < nw * 64 && kw < nkw) ? Bt[(int64_t)brow * sbt + kw] : 0ull;
            }
        };
        auto lstore = [&](int buf) {
#pragma unroll
            for (int i = 0; i < G2_KC; i++) {
                const int e = tid + 256 * i;
                const int rr = e / G2_KC, w = e % G2_KC;
                *reinterpret_cast<uint64_t *>(&sA[buf][rr * G2_LD + 2 * w]) = ra[i];
                *reinterpret_cast<uint64_t *>(&sB[buf][rr * G2_LD + 2 * w]) = rb[i];
            }
        };
        v16i acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++)
#pragma unroll
                for (int v = 0; v < 16; v++) acc[a][b][v] = 0;
        __syncthreads();
        gload(0);
        lstore(0);
        __syncthreads();
        for (int st = 0; st < nstage; st++) {
            const int buf = st & 1;
            if (st + 1 < nstage) gload(st + 1);
            const int kend = min(G2_KC, nkw - st * G2_KC);
            for (int w = 0; w < kend; w++) {
                uint32_t wa[4], wb[4];
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    wa[t] = sA[buf][(wm * 128 + t * 32 + li) * G2_LD + 2 * w + lg];
                    wb[t] = sB[buf][(wn * 128 + t * 32 + li) * G2_LD + 2 * w + lg];
                }
#pragma unroll
                for (int s = 0; s < 2; s++) {
                    v4i fa[4], fb[4];
#pragma unroll
                    for (int t = 0; t < 4; t++)
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            fa[t][v] = (int)(wa[t] >> (4 * s + v));
                            fb[t][v] = (int)(wb[t] >> (4 * s + v));
                        }
#pragma unroll
                    for (int a = 0; a < 4; a++)
#pragma unroll
                        for (int b = 0; b < 4; b++)
                            acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b],
                                                                             acc[a][b], 0, 0, 0);
                }
            }
            if (st + 1 < nstage) lstore(buf ^ 1);
            __syncthreads();
        }
        // bit 0 of each sum -> packed words; lane L collects rows L and 64 + L of
        // the wave's 128 rows, words 0 and 1 of its 128 columns.
        uint64_t out[2][2] = {{0ull, 0ull}, {0ull, 0ull}};
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++)
#pragma unroll
                for (int v = 0; v < 16; v++) {
                    const uint64_t bal = __ballot(acc[a][b][v] & 1);
                    const int rlo = 32 * (a & 1) + 8 * (v >> 2) + (v & 3);
                    const int sh = 32 * (b & 1);
                    const uint64_t flo = (bal & 0xFFFFFFFFull) << sh;
                    const uint64_t fhi = (bal >> 32) << sh;
                    if (lane == rlo) out[a >> 1][b >> 1] |= flo;
                    if (lane == rlo + 4) out[a >> 1][b >> 1] |= fhi;
                }
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
    // their larger prologue and epilogue (measured: K >= 8192 on 65536^2 PLS);
    // shorter products use the 128 x 128 kernel
    if (nw >= 4 && kmax > 4096) {
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

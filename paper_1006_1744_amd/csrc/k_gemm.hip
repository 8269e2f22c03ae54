// GF(2) matrix product C <- C + A * B, the Schur-complement update of the
// recursive PLS (Section 5: A_SE <- A_SE + A_SW * A_NE) and of the recursive
// triangular solve.  A is packed along K (its rows), B along N; B is first
// transposed bitwise so both operands are packed along K, and then
//   C[i][j] ^= parity( popcount( A_i[0:K] AND Bt_j[0:K] ) ).
// Variant X (this file) evaluates it on the vector ALUs: every 32-bit word
// step is one AND-XOR (v_bitop3_b32 on gfx950) per output element, parity at
// the end.  Variant M (k_mfma.hip) uses the matrix cores (fp4 or int8).
#include "gf2_device.h"
#include "gf2_internal.h"

namespace gf2 {

// Bt[64 jw + c][kw] <- bits c of words jw of B rows 64 kw .. 64 kw + 63 (rows at
// or past K read as zero).
// Small transposes: one wave per 64 x 64 block, each lane loading its row's word
// and storing its column's word directly (the most blocks in flight).
__global__ __launch_bounds__(256) void transpose_direct_kernel(const uint64_t *B, int64_t sb, int m,
                                                               RowRange brows, int w_lo, int nw,
                                                               int kmax, uint64_t *Bt, int64_t sbt,
                                                               const int32_t *rk, const int32_t *nwd) {
    if (nwd) nw = min(nw, *nwd);
    int b0, b1;
    eval_range(rk, m, brows, b0, b1);
    const int K = b1 - b0;
    const int nkw = (kmax + 63) / 64;
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (blockDim.x / 64);
    const int total = nkw * nw;
    for (int blk = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); blk < total;
         blk += waves) {
        const int kw = blk % nkw, jw = blk / nkw;
        const int row = 64 * kw + lane;
        uint64_t v = row < K ? B[(int64_t)(b0 + row) * sb + w_lo + jw] : 0ull;
        v = transpose64(v, lane);
        Bt[(int64_t)(64 * jw + lane) * sbt + kw] = v;
    }
}

// Large transposes: a block stages a tile of 64 rows x 16 words through
// LDS (each row's 16 words are one 128-byte read), then each wave transposes
// 64 x 64 blocks of it in registers.  Tiles are dealt so that the blocks of one
// XCD walk consecutive kw of one word group: the output words a line of Bt
// gathers from several tiles are then written through one L2.
constexpr int TP_JW = 16;

__global__ __launch_bounds__(256) void transpose_kernel(const uint64_t *B, int64_t sb, int m,
                                                        RowRange brows, int w_lo, int nw, int kmax,
                                                        uint64_t *Bt, int64_t sbt,
                                                        const int32_t *rk, const int32_t *nwd) {
    __shared__ uint64_t sT[64][TP_JW + 1];
    if (nwd) nw = min(nw, *nwd);
    int b0, b1;
    eval_range(rk, m, brows, b0, b1);
    const int K = b1 - b0;
    const int nkw = (kmax + 63) / 64;
    const int njb = (nw + TP_JW - 1) / TP_JW;
    const int total = nkw * njb;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int per = gridDim.x / 8;
    const int vid = (gridDim.x % 8 == 0) ? (blockIdx.x % 8) * per + blockIdx.x / 8 : blockIdx.x;
    for (int t = vid; t < total; t += gridDim.x) {
        const int kw = t % nkw, jb = t / nkw;
        for (int e = threadIdx.x; e < 64 * TP_JW; e += 256) {
            const int r = e / TP_JW, w = e % TP_JW;
            const int row = 64 * kw + r, jw = jb * TP_JW + w;
            sT[r][w] = (row < K && jw < nw) ? B[(int64_t)(b0 + row) * sb + w_lo + jw] : 0ull;
        }
        __syncthreads();
        for (int j = wave; j < TP_JW; j += 4) {
            const int jw = jb * TP_JW + j;
            if (jw < nw) {
                const uint64_t v = transpose64(sT[lane][j], lane);
                Bt[(int64_t)(64 * jw + lane) * sbt + kw] = v;
            }
        }
        __syncthreads();
    }
}

hipError_t launch_transpose(const uint64_t *B, int64_t sb, int m, RowRange brows, int w_lo,
                            int nw, int kmax, uint64_t *Bt, int64_t sbt, const int32_t *rk,
                            hipStream_t st, const int32_t *nwd) {
    const int nkw = (kmax + 63) / 64;
    if ((int64_t)nkw * nw <= 0) return hipSuccess;
    if ((int64_t)nkw * nw < 16384) {
        const int64_t blocks = ((int64_t)nkw * nw + 3) / 4;
        hipLaunchKernelGGL(transpose_direct_kernel, dim3((unsigned)blocks), dim3(256), 0, st, B, sb,
                           m, brows, w_lo, nw, kmax, Bt, sbt, rk, nwd);
        return hipGetLastError();
    }
    const int64_t total = (int64_t)nkw * ((nw + TP_JW - 1) / TP_JW);
    int64_t blocks = total < 2048 ? total : 2048;
    if (blocks >= 8) blocks = blocks / 8 * 8;
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)blocks), dim3(256), 0, st, B, sb, m, brows,
                       w_lo, nw, kmax, Bt, sbt, rk, nwd);
    return hipGetLastError();
}

// ------------------------------------------------------------- variant X
constexpr int GX_TM = 128;     // rows per tile
constexpr int GX_TNW = 2;      // C words per tile (128 columns)
constexpr int GX_KC = 8;       // K words staged per step
constexpr int GX_LD = GX_KC + 1;

__global__ __launch_bounds__(256) void gemm_xor_kernel(uint64_t *C, int64_t sc, const uint64_t *A,
                                                       int64_t sa, int m, RowRange rows, int aw,
                                                       int w_lo, int nw, const uint64_t *Bt,
                                                       int64_t sbt, int nkw, RowRange krows,
                                                       int kmrows, const int32_t *rk,
                                                       int32_t *prof, const int32_t *nwd) {
    __shared__ uint64_t sA[GX_TM][GX_LD];
    __shared__ uint64_t sB[GX_TNW * 64][GX_LD];
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
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const int lane = tid & 63;
    const int tiles_m = (M + GX_TM - 1) / GX_TM;
    const int tiles_n = (nw + GX_TNW - 1) / GX_TNW;
    const int ntiles = tiles_m * tiles_n;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int tm = tile % tiles_m, tn = tile / tiles_m;
        const int row0 = r0 + tm * GX_TM;
        const int cw0 = tn * GX_TNW;   // relative C word
        uint32_t acc[8][8];
#pragma unroll
        for (int i = 0; i < 8; i++)
#pragma unroll
            for (int j = 0; j < 8; j++) acc[i][j] = 0;
        for (int kc = 0; kc < nkw; kc += GX_KC) {
            __syncthreads();
            for (int e = tid; e < GX_TM * GX_KC; e += 256) {
                int rr = e / GX_KC, w = e % GX_KC;
                int grow = row0 + rr;
                sA[rr][w] = (grow < r1 && kc + w < nkw) ? A[(int64_t)grow * sa + aw + kc + w] : 0ull;
            }
            for (int e = tid; e < GX_TNW * 64 * GX_KC; e += 256) {
                int rr = e / GX_KC, w = e % GX_KC;
                int brow = cw0 * 64 + rr;
                sB[rr][w] = (brow < nw * 64 && kc + w < nkw) ? Bt[(int64_t)brow * sbt + kc + w] : 0ull;
            }
            __syncthreads();
#pragma unroll 2
            for (int w = 0; w < GX_KC; w++) {
                uint64_t a[8], b[8];
#pragma unroll
                for (int i = 0; i < 8; i++) a[i] = sA[ty + 16 * i][w];
#pragma unroll
                for (int j = 0; j < 8; j++) b[j] = sB[tx + 16 * j][w];
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    const uint32_t alo = (uint32_t)a[i], ahi = (uint32_t)(a[i] >> 32);
#pragma unroll
                    for (int j = 0; j < 8; j++) {
                        uint32_t t = acc[i][j] ^ (alo & (uint32_t)b[j]);
                        acc[i][j] = t ^ (ahi & (uint32_t)(b[j] >> 32));
                    }
                }
            }
        }
        // parity -> bits; column tx + 16 j is bit (tx + 16 (j % 4)) of word j / 4
        uint64_t part[8][GX_TNW];
#pragma unroll
        for (int i = 0; i < 8; i++) {
            part[i][0] = 0;
            part[i][1] = 0;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                uint64_t bit = (uint64_t)(__popc(acc[i][j]) & 1);
                part[i][j >> 2] |= bit << (tx + 16 * (j & 3));
            }
        }
#pragma unroll
        for (int i = 0; i < 8; i++)
#pragma unroll
            for (int q = 0; q < GX_TNW; q++) {
                uint64_t v = part[i][q];
                v |= shfl_xor64(v, 1);
                v |= shfl_xor64(v, 2);
                v |= shfl_xor64(v, 4);
                v |= shfl_xor64(v, 8);
                part[i][q] = v;
            }
        // lane tx writes (i, q) = (tx >> 1, tx & 1)
        {
            const int i = tx >> 1, q = tx & 1;
            uint64_t v = 0;
#pragma unroll
            for (int ii = 0; ii < 8; ii++)
#pragma unroll
                for (int qq = 0; qq < GX_TNW; qq++)
                    if (ii == i && qq == q) v = part[ii][qq];
            const int grow = row0 + ty + 16 * i;
            const int cw = cw0 + q;
            if (grow < r1 && cw < nw && v) {
                uint64_t *pc = C + (int64_t)grow * sc + w_lo + cw;
                *pc ^= v;
            }
        }
        (void)lane;
    }
}

hipError_t launch_gemm_xor(uint64_t *C, int64_t sc, const uint64_t *A, int64_t sa, int m,
                           RowRange rows, int aw, int w_lo, int nw, const uint64_t *Bt,
                           int64_t sbt, int kmax, RowRange krows, int kmrows, const int32_t *rk,
                           int32_t *prof, hipStream_t st, const int32_t *nwd) {
    int nkw = (kmax + 63) / 64;
    if (nw <= 0 || nkw <= 0) return hipSuccess;
    int64_t tiles = (int64_t)((m + GX_TM - 1) / GX_TM) * ((nw + GX_TNW - 1) / GX_TNW);
    int64_t blocks = tiles < 2048 ? tiles : 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(gemm_xor_kernel, dim3((unsigned)blocks), dim3(256), 0, st, C, sc, A, sa, m,
                       rows, aw, w_lo, nw, Bt, sbt, nkw, krows, kmrows, rk, prof, nwd);
    return hipGetLastError();
}

}  // namespace gf2

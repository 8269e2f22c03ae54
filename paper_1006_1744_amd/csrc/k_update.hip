// Table-driven updates of the MMPF base case and the small pieces of the
// recursive driver.
//
// trsm_base_kernel   X <- L^{-1} X for a block of at most 64 rows (unit lower
//                    triangular L = the block's own bits below the diagonal in
//                    one word column), or X <- U^{-1} X with the bits above it.
//                    Rows are processed in groups of k: within a group by plain
//                    substitution, then the group's 2^k combinations are
//                    tabulated in LDS (MakeTable, Section 3.1) and every later
//                    row of the block adds one table row per group
//                    (AddRowsFromTable, Appendix A).
// table_update_kernel Schur update after one panel: every row below the
//                    panel's pivot rows adds L[i] * U on the target columns, with
//                    L[i] the row's (final, compressed) panel word and U the
//                    pivot rows; one table per k multipliers, `tables` tables per
//                    pass over the rows.
// compress_shift_kernel  final "compress L" of Section 5.
// finalize_kernel    P, Q tails and the rank.
#include "gf2_internal.h"

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

// ------------------------------------------------------------------ TRSM
constexpr int TRSM_THREADS = 256;
constexpr int TRSM_TW = 16;   // tile words
constexpr int TRSM_K = 8;

__global__ __launch_bounds__(TRSM_THREADS) void trsm_base_kernel(
    uint64_t *A, int64_t stride, const uint64_t *Lm, int64_t sl, int m, RowRange rows, int lw,
    int w_lo, int w_hi, const int32_t *rk, int lower) {
    __shared__ uint64_t sX[64][TRSM_TW];
    __shared__ uint64_t sT[256][TRSM_TW];
    __shared__ uint64_t sL[64];
    int r0, r1;
    eval_range(rk, m, rows, r0, r1);
    const int nr = min(r1 - r0, 64);
    if (nr <= 1) return;
    const int tid = threadIdx.x;
    const int w0 = w_lo + blockIdx.x * TRSM_TW;
    const int tw_n = min(TRSM_TW, w_hi - w0);
    if (tw_n <= 0) return;
    for (int e = tid; e < 64 * TRSM_TW; e += TRSM_THREADS) {
        int s = e / TRSM_TW, w = e % TRSM_TW;
        sX[s][w] = (s < nr && w < tw_n) ? A[(int64_t)(r0 + s) * stride + w0 + w] : 0ull;
    }
    if (tid < 64) {
        uint64_t lv = tid < nr ? Lm[(int64_t)(r0 + tid) * sl + lw] : 0ull;
        uint64_t below = tid == 0 ? 0ull : (~0ull >> (64 - tid));
        sL[tid] = lower ? (lv & below) : (lv & ~below & ~(1ull << tid));
    }
    __syncthreads();
    const int ng = (nr + TRSM_K - 1) / TRSM_K;
    for (int gi = 0; gi < ng; gi++) {
        const int g = lower ? gi : ng - 1 - gi;
        const int gb = g * TRSM_K, gs = min(TRSM_K, nr - gb);
        // substitution inside the group
        if (tid < TRSM_TW) {
            const int w = tid;
            if (lower) {
                for (int u = 1; u < gs; u++) {
                    uint64_t lv = sL[gb + u];
                    uint64_t acc = sX[gb + u][w];
                    for (int v = 0; v < u; v++)
                        if ((lv >> (gb + v)) & 1) acc ^= sX[gb + v][w];
                    sX[gb + u][w] = acc;
                }
            } else {
                for (int u = gs - 2; u >= 0; u--) {
                    uint64_t lv = sL[gb + u];
                    uint64_t acc = sX[gb + u][w];
                    for (int v = u + 1; v < gs; v++)
                        if ((lv >> (gb + v)) & 1) acc ^= sX[gb + v][w];
                    sX[gb + u][w] = acc;
                }
            }
        }
        __syncthreads();
        const bool more = lower ? (gb + gs < nr) : (gb > 0);
        if (!more) break;
        // tabulate the group's combinations
        for (int e = tid; e < (1 << gs) * TRSM_TW; e += TRSM_THREADS) {
            int comb = e / TRSM_TW, w = e % TRSM_TW;
            uint64_t v = 0;
            for (int u = 0; u < gs; u++)
                if ((comb >> u) & 1) v ^= sX[gb + u][w];
            sT[comb][w] = v;
        }
        __syncthreads();
        // one table row per remaining row of the block
        const int lo = lower ? gb + gs : 0, hi = lower ? nr : gb;
        for (int e = tid; e < (hi - lo) * TRSM_TW; e += TRSM_THREADS) {
            int s = lo + e / TRSM_TW, w = e % TRSM_TW;
            int id = (int)((sL[s] >> gb) & ((1u << gs) - 1));
            sX[s][w] ^= sT[id][w];
        }
        __syncthreads();
    }
    for (int e = tid; e < nr * TRSM_TW; e += TRSM_THREADS) {
        int s = e / TRSM_TW, w = e % TRSM_TW;
        if (w < tw_n) A[(int64_t)(r0 + s) * stride + w0 + w] = sX[s][w];
    }
}

hipError_t launch_trsm_base(uint64_t *A, int64_t stride, const uint64_t *Lm, int64_t sl, int m,
                            RowRange rows, int lw, int w_lo, int w_hi, const int32_t *rk,
                            int lower, hipStream_t st) {
    if (w_hi <= w_lo) return hipSuccess;
    int nb = (w_hi - w_lo + TRSM_TW - 1) / TRSM_TW;
    hipLaunchKernelGGL(trsm_base_kernel, dim3(nb), dim3(TRSM_THREADS), 0, st, A, stride, Lm, sl, m,
                       rows, lw, w_lo, w_hi, rk, lower);
    return hipGetLastError();
}

// ------------------------------------------------------------ table update
constexpr int TU_THREADS = 256;
constexpr int TU_LDS = 64 * 1024;   // table budget per block

int table_update_tile_words(int k, int tables) {
    int tw = TU_LDS / (tables * (1 << k) * 8);
    if (tw > 64) tw = 64;
    if (tw < 1) tw = 1;
    return tw;
}

__global__ __launch_bounds__(TU_THREADS) void table_update_kernel(
    uint64_t *A, int64_t stride, int m, int wc, const int32_t *rk, int b, int w_lo, int w_hi,
    int k, int tables, int TW) {
    extern __shared__ uint64_t tu_lds[];   // U rows [64][TW], then tables [tables][1<<k][TW]
    const int R = rk[b];
    const int R1 = rk[b + 1];
    const int r = R1 - R;
    if (r <= 0 || R1 >= m) return;
    const int tid = threadIdx.x;
    const int w0 = w_lo + blockIdx.y * TW;
    const int tw_n = min(TW, w_hi - w0);
    if (tw_n <= 0) return;
    uint64_t *sU = tu_lds;
    uint64_t *sT = tu_lds + 64 * TW;
    for (int e = tid; e < r * TW; e += TU_THREADS) {
        int s = e / TW, w = e % TW;
        sU[e] = w < tw_n ? A[(int64_t)(R + s) * stride + w0 + w] : 0ull;
    }
    const int ng = (r + k - 1) / k;
    const int npass = (ng + tables - 1) / tables;
    const int esz = 1 << k;
    const int rows_per_it = TU_THREADS / TW;
    const int my_w = tid % TW, my_row = tid / TW;
    for (int pass = 0; pass < npass; pass++) {
        const int g0 = pass * tables, g1 = min(ng, g0 + tables);
        __syncthreads();
        // MakeTable: all combinations of each group's U rows (tile words only)
        for (int e = tid; e < (g1 - g0) * esz * TW; e += TU_THREADS) {
            int w = e % TW, comb = (e / TW) % esz, slot = e / (TW * esz);
            int gb = (g0 + slot) * k, gs = min(k, r - gb);
            uint64_t v = 0;
            if (comb < (1 << gs))
                for (int u = 0; u < gs; u++)
                    if ((comb >> u) & 1) v ^= sU[(gb + u) * TW + w];
            sT[e] = v;
        }
        __syncthreads();
        // AddRowsFromTable: rows below the pivot rows, one table row per group
        if (my_row < rows_per_it && my_w < tw_n) {
            for (int i = R1 + blockIdx.x * rows_per_it + my_row; i < m;
                 i += gridDim.x * rows_per_it) {
                const uint64_t lv = A[(int64_t)i * stride + wc];
                uint64_t *px = A + (int64_t)i * stride + w0 + my_w;
                uint64_t x = *px;
                for (int g = g0; g < g1; g++) {
                    int gb = g * k, gs = min(k, r - gb);
                    int id = (int)((lv >> gb) & ((1u << gs) - 1));
                    x ^= sT[((g - g0) * esz + id) * TW + my_w];
                }
                *px = x;
            }
        }
    }
}

hipError_t launch_table_update(uint64_t *A, int64_t stride, int m, int wc, const int32_t *rk,
                               int b, int w_lo, int w_hi, int k, int tables, hipStream_t st) {
    if (w_hi <= w_lo) return hipSuccess;
    int TW = table_update_tile_words(k, tables);
    if (TW > w_hi - w_lo) TW = w_hi - w_lo;
    int ny = (w_hi - w_lo + TW - 1) / TW;
    int rows_per_it = TU_THREADS / TW;
    int nx = (m + rows_per_it - 1) / rows_per_it;
    int want = (2048 + ny - 1) / ny;   // enough blocks to fill the device
    if (nx > want) nx = want;
    if (nx < 1) nx = 1;
    size_t lds = ((size_t)64 + (size_t)tables * (1 << k)) * TW * 8;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)table_update_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(table_update_kernel, dim3(nx, ny), dim3(TU_THREADS), lds, st, A, stride, m,
                       wc, rk, b, w_lo, w_hi, k, tables, TW);
    return hipGetLastError();
}

// ---------------------------------------------------------- compress shift
// Node at column c0 with split n0 (both multiples of 64): the second block's L
// columns [c0+n0, c0+n0+r1) move to [c0+r0, c0+r0+r1), row by row as the column
// swaps "i <-> n0 + (i - r0), from row i" leave them: a row at offset v below
// the first block's pivots moves min(v + 1, r1) columns and zeroes the vacated ones.
__global__ void compress_shift_kernel(uint64_t *A, int64_t stride, int m, int c0, int n0,
                                      const int32_t *rk, int b0, int b1, int b2) {
    const int R = rk[b0], Rm = rk[b1], Re = rk[b2];
    const int r0 = Rm - R, r1 = Re - Rm;
    if (r0 >= n0 || r1 <= 0) return;
    const int d = n0 - r0;
    for (int i = Rm + blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const int v = i - Rm;
        const int len = min(v + 1, r1);
        uint64_t *row = A + (int64_t)i * stride;
        const int D = c0 + r0;             // first destination bit
        const int S = c0 + n0;             // first source bit
        const int end = S + len;           // bits [D, end) change
        for (int w = D >> 6; w <= (end - 1) >> 6; w++) {
            const int p0 = w * 64;
            // source bits for positions p0 .. p0+63 are p0 + d ..
            const int sb = p0 + d;
            const int sw = sb >> 6, so = sb & 63;
            uint64_t lo = sw < stride ? row[sw] : 0ull;
            uint64_t hi = (so && sw + 1 < stride) ? row[sw + 1] : 0ull;
            uint64_t src = so ? ((lo >> so) | (hi << (64 - so))) : lo;
            uint64_t old = row[w];
            // masks over positions p0+j
            uint64_t mv = 0, clr = 0;
            int a = max(D, p0), e = min(D + len, p0 + 64);
            if (e > a) mv = ((e - a) == 64 ? ~0ull : ((1ull << (e - a)) - 1)) << (a - p0);
            a = max(D + len, p0);
            e = min(end, p0 + 64);
            if (e > a) clr = ((e - a) == 64 ? ~0ull : ((1ull << (e - a)) - 1)) << (a - p0);
            row[w] = (old & ~(mv | clr)) | (src & mv);
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

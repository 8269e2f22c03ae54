// M4RI: the reduced row echelon form directly (Section 3.1, algorithm "M4RI",
// with GaussSubmatrix, MakeTable and AddRowsFromTable of Appendix A), and the
// pieces of the "M+P" hybrid of Section 6 that start with it.
//
// Strips are 64-column panels here, as in the MMPF base case.  Per panel, the
// panel search and its final pass (shared with the PLS) find the pivots of the
// rows [R, m) in the pivot order of Gaussian elimination and move the pivot
// rows to [R, R + r), leaving in every row below its multipliers l (the panel's
// L word) and the pivot rows' words right of the panel staged as B.  M4RI then
// reduces every other row, above and below:
//  * U = L^{-1} B are the echelon pivot rows; their panel part Us is upper
//    triangular on the pivot columns q (V = Us[:, q], unit upper triangular).
//    GaussSubmatrix's identity block is reached with W = V^{-1}: the reduced
//    pivot rows are U' = W U, i.e. E = W Us on the panel and N B right of it,
//    N = W L^{-1}.
//  * a row above (i < R) with panel word xs adds its pivot-column bits times
//    U': on the panel xs ^ xs H, right of it x ^ (xs G) B, where G and H hold N
//    and E at the pivot positions q (zero rows elsewhere), so the bit selection
//    and the change of basis are one table lookup per byte of xs;
//  * a row below adds (l L^{-1}) B right of the panel (the unique combination
//    of the pivot rows that clears its pivot columns) and its panel word
//    becomes zero (its non-pivot panel columns were already zero: a column
//    with no pivot is zero in every remaining row).
// The tables of B (k rows each, `tables` per pass) are MakeTable's; one table
// row per table and row is AddRowsFromTable.
// Every row's multiplier (xs G or l L^{-1}) and new panel word are formed by
// one kernel before the update, which reads the multipliers from a buffer: the
// update's column tiles of one row run in different blocks, and none of them
// may see the panel word after another has rewritten it.
#include <algorithm>

#include "gf2_device.h"
#include "gf2_panel.h"

namespace gf2 {

struct M4riRec {
    uint64_t G[64];   // row q[t] = N_t, zero at non-pivot positions
    uint64_t H[64];   // row q[t] = E_t, zero at non-pivot positions
    uint64_t N[64];   // N_t = (W L^{-1})_t for the pivot rows' results
    uint64_t E[64];   // E_t: the pivot rows' panel words after the reduction
};

size_t m4ri_rec_bytes() { return sizeof(M4riRec); }

__device__ inline uint64_t shfl64(uint64_t v, int src) {
    const int lo = __shfl((int)(uint32_t)v, src);
    const int hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// One wave: W = V^{-1}, N = W L^{-1}, E = W Us, and G, H by pivot position.
__global__ __launch_bounds__(64) void m4ri_prep_kernel(const PanelInfo *info, const int32_t *rk,
                                                       int b, M4riRec *rec) {
    const int lane = threadIdx.x;
    const int r = __builtin_amdgcn_readfirstlane(rk[b + 1] - rk[b]);
    if (r <= 0) return;
    const int qv = lane < r ? info->q[lane] : 0;
    const uint64_t us = lane < r ? (info->u[lane] & (~0ull << qv)) : 0ull;
    const uint64_t li = info->linv[lane];   // rows past r are unit vectors
    uint64_t pm = 0, v = 0;
    for (int s = 0; s < r; s++) {
        const int qs = __builtin_amdgcn_readlane(qv, s);
        pm |= 1ull << qs;
        v |= ((us >> qs) & 1ull) << s;
    }
    if (lane >= r) v = 1ull << lane;
    const uint64_t w = tri_inverse64_row(v, lane, false);
    uint64_t nrow = 0, erow = 0;
    for (int s = 0; s < r; s++) {
        const uint64_t ls = readlane64(li, s), es = readlane64(us, s);
        if ((w >> s) & 1ull) {
            nrow ^= ls;
            erow ^= es;
        }
    }
    const bool isp = (pm >> lane) & 1ull;
    const int tj = __popcll(pm & ((1ull << lane) - 1));
    const uint64_t nj = shfl64(nrow, tj & 63), ej = shfl64(erow, tj & 63);
    rec->G[lane] = isp ? nj : 0ull;
    rec->H[lane] = isp ? ej : 0ull;
    rec->N[lane] = lane < r ? nrow : 0ull;
    rec->E[lane] = lane < r ? erow : 0ull;
}

constexpr int M4_THREADS = 1024;
constexpr int M4_TWMAX = 8;
constexpr int M4_TABLE_LDS = 120 * 1024;   // the B tables of one pass
constexpr int M4_LDS_MAX = 150 * 1024;

int m4ri_tile_words(int k, int tables) {
    int tw = M4_TABLE_LDS / (tables * (1 << k) * 8);
    return std::max(1, std::min(tw, M4_TWMAX));
}

size_t m4ri_lds_bytes(int k, int tables, int TW) {
    return (size_t)(64 + 2 * 64 * TW + tables * (1 << k) * TW) * 8;
}

// Per row: the multiplier on the staged pivot rows B (rows above: xs G, rows
// below: l L^{-1}) into cbuf, and the row's new panel word (above: xs ^ xs H,
// below: zero, pivot row t: E_t).
__global__ __launch_bounds__(M4_THREADS) void m4ri_mult_kernel(uint64_t *A, int64_t stride, int m,
                                                               int wc, const int32_t *rk, int b,
                                                               const uint64_t *linv,
                                                               const M4riRec *rec, uint64_t *cbuf) {
    __shared__ uint64_t sLT[8 * 256], sGT[8 * 256], sHT[8 * 256];
    __shared__ uint64_t sRows[64];
    const int R = rk[b];
    const int r = rk[b + 1] - R;
    if (r <= 0) return;
    const int tid = threadIdx.x;
    const uint64_t *srcs[3] = {linv, rec->G, rec->H};
    uint64_t *dsts[3] = {sLT, sGT, sHT};
    for (int u = 0; u < 3; u++) {
        if (tid < 64) sRows[tid] = srcs[u][tid];
        __syncthreads();
        build_tables_8x8<M4_THREADS>(sRows, dsts[u], tid);
    }
    for (int i = blockIdx.x * M4_THREADS + tid; i < m; i += gridDim.x * M4_THREADS) {
        uint64_t *px = A + (int64_t)i * stride + wc;
        if (i >= R && i < R + r) {
            *px = rec->E[i - R];
            continue;
        }
        const uint64_t xs = *px;
        const bool above = i < R;
        const uint64_t *tt = above ? sGT : sLT;
        uint64_t c = 0, h = 0;
#pragma unroll
        for (int g8 = 0; g8 < 8; g8++) {
            const int byte = (int)((xs >> (8 * g8)) & 255);
            c ^= tt[g8 * 256 + byte];
            if (above) h ^= sHT[g8 * 256 + byte];
        }
        cbuf[i] = c;
        const uint64_t ns = above ? (xs ^ h) : 0ull;
        if (ns != xs) *px = ns;
    }
}

// Every row but the pivot rows on the word tile [w0, w0 + TW) of [w_lo, w_hi):
// x += c B with c = cbuf[row]; block (0, y) writes the pivot rows' results
// N B.  2^lg_tpr threads share a row (each its words).
__global__ __launch_bounds__(M4_THREADS) void m4ri_update_kernel(
    uint64_t *A, int64_t stride, int m, const int32_t *rk, int b, int w_lo, int w_hi, int k,
    int tables, int TW, int lg_tpr, const M4riRec *rec, const uint64_t *cbuf, const uint64_t *Bbuf,
    int64_t bstride) {
    extern __shared__ uint64_t m4_lds[];
    uint64_t *sN = m4_lds;               // [64]
    uint64_t *sB = sN + 64;              // [64][TW]
    uint64_t *sU = sB + 64 * TW;         // [64][TW] pivot rows' results
    uint64_t *sT = sU + 64 * TW;         // [tables][1 << k][TW]
    const int R = rk[b];
    const int r = rk[b + 1] - R;
    if (r <= 0) return;
    const int tid = threadIdx.x;
    const int w0 = w_lo + blockIdx.y * TW;
    const int tw_n = min(TW, w_hi - w0);
    if (tw_n <= 0) return;
    const bool pivots_here = blockIdx.x == 0;
    const int wq = tid % TW, pq = tid / TW, pstep = M4_THREADS / TW;
    if (tid < 64) sN[tid] = rec->N[tid];
    if (pq < pstep)
        for (int t = pq; t < 64; t += pstep) {
            sB[t * TW + wq] =
                (t < r && wq < tw_n) ? Bbuf[(int64_t)t * bstride + (w0 - w_lo) + wq] : 0ull;
            sU[t * TW + wq] = 0ull;
        }
    const int ng = (r + k - 1) / k;
    const int npass = (ng + tables - 1) / tables;
    const int esz = 1 << k;
    const uint32_t kmask = (1u << k) - 1;
    const int rpb = M4_THREADS >> lg_tpr;
    const int part = tid & ((1 << lg_tpr) - 1);
    const int wpt = (TW + (1 << lg_tpr) - 1) >> lg_tpr;
    const int wb = part * wpt;
    const int wn = max(0, min(wpt, tw_n - wb));
    const int nrows = m - r;   // rows [0, R) and [R + r, m)
    const int per = gridDim.x * rpb;
    const int nchunks = nrows > 0 ? (nrows + per - 1) / per : 1;
    int j = blockIdx.x * rpb + (tid >> lg_tpr);
    for (int chunk = 0; chunk < nchunks; chunk++, j += per) {
        const bool act = j < nrows;
        const int i = j < R ? j : j + r;
        uint64_t x[M4_TWMAX];
        uint64_t c = 0;
        uint64_t *px = A + (int64_t)i * stride + w0 + wb;
        if (act) {
            c = cbuf[i];
#pragma unroll
            for (int w = 0; w < M4_TWMAX; w++)
                if (w < wn) x[w] = px[w];
        }
        for (int pass = 0; pass < npass; pass++) {
            const int g0 = pass * tables, g1 = min(ng, g0 + tables);
            if (chunk == 0 || npass > 1) {
                __syncthreads();
                build_group_tables(sB + (size_t)g0 * k * TW, r - g0 * k, k, g1 - g0, sT, TW, tid,
                                   M4_THREADS);
                if (pivots_here && chunk == 0 && pq < pstep) {
                    for (int t = pq; t < r; t += pstep) {
                        const uint64_t ct = sN[t];
                        uint64_t y = sU[t * TW + wq];
                        for (int g = g0; g < g1; g++)
                            y ^= sT[((g - g0) * esz + (int)((ct >> (k * g)) & kmask)) * TW + wq];
                        sU[t * TW + wq] = y;
                    }
                }
            }
            if (act) {
                for (int g = g0; g < g1; g++) {
                    const uint64_t *T =
                        sT + ((size_t)(g - g0) * esz + ((c >> (k * g)) & kmask)) * TW + wb;
#pragma unroll
                    for (int w = 0; w < M4_TWMAX; w++)
                        if (w < wn) x[w] ^= T[w];
                }
            }
        }
        if (act) {
#pragma unroll
            for (int w = 0; w < M4_TWMAX; w++)
                if (w < wn) px[w] = x[w];
        }
    }
    if (pivots_here && pq < pstep && wq < tw_n)
        for (int t = pq; t < r; t += pstep) A[(int64_t)(R + t) * stride + w0 + wq] = sU[t * TW + wq];
}

// Estimated density of the rows [R, m) on the words [w0, nw) (the part left to
// eliminate), from up to 256 rows spread evenly over them: out[0] (float
// bits) = ones / entries, out[1] = R.
__global__ __launch_bounds__(256) void m4ri_density_kernel(const uint64_t *A, int64_t stride, int m,
                                                           int n, int w0, const int32_t *rk, int b,
                                                           int32_t *out) {
    __shared__ unsigned long long s_cnt;
    const int R = rk[b];
    const int rows = m - R;
    const int nw = (n + 63) / 64;
    const int S = min(rows, 256);
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    if ((int)threadIdx.x < S) {
        const int i = R + (int)(((int64_t)threadIdx.x * rows) / S);
        unsigned long long c = 0;
        for (int w = w0; w < nw; w++) c += __popcll(A[(int64_t)i * stride + w]);
        atomicAdd(&s_cnt, c);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double entries = (double)S * (double)(n - 64 * w0);
        const float d = entries > 0 ? (float)((double)s_cnt / entries) : 0.f;
        out[0] = __float_as_int(d);
        out[1] = R;
    }
}

// Columns of the rows [0, rows) of X (words [0, nw)) selected by the mask PM,
// packed into C (bit prefP[w] + t of a row <- the t-th selected bit of its word
// w).  C zero on entry.  One thread per (row, word).
__global__ void gather_cols_kernel(const uint64_t *X, int64_t sx, int rows, int nw,
                                   const uint64_t *PM, const int32_t *prefP, uint64_t *C,
                                   int64_t sc) {
    const int64_t total = (int64_t)rows * nw;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / nw), w = (int)(e % nw);
        const uint64_t pm = PM[w];
        if (!pm) continue;
        const uint64_t x = X[(int64_t)i * sx + w];
        uint64_t v = 0;
        int t = 0;
        for (uint64_t mm = pm; mm; mm &= mm - 1, t++)
            v |= ((x >> (__ffsll((unsigned long long)mm) - 1)) & 1ull) << t;
        if (!v) continue;
        const int off = prefP[w], o = off >> 6, sh = off & 63;
        atomicOr((unsigned long long *)&C[(int64_t)i * sc + o], v << sh);
        if (sh && sh + t > 64) atomicOr((unsigned long long *)&C[(int64_t)i * sc + o + 1], v >> (64 - sh));
    }
}

// The hybrid's result bookkeeping: Q[R + i] = c0 + Q2[i] for i < r2, Q[i] = i
// for R + r2 <= i < n, rank = R + r2, and ext = {R, R + r2}.
__global__ void mp_finish_kernel(int32_t *Q, int32_t *rank, int32_t *ext, const int32_t *Q2,
                                 const int32_t *rank2, int R, int c0, int n) {
    const int r2 = *rank2;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n - R; i += gridDim.x * blockDim.x) {
        if (i < r2) Q[R + i] = c0 + Q2[i];
        else Q[R + i] = R + i;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *rank = R + r2;
        ext[0] = R;
        ext[1] = R + r2;
    }
}

hipError_t launch_m4ri_prep(const int32_t *info, const int32_t *rk, int b, void *rec,
                            hipStream_t st) {
    hipLaunchKernelGGL(m4ri_prep_kernel, dim3(1), dim3(64), 0, st,
                       reinterpret_cast<const PanelInfo *>(info), rk, b,
                       reinterpret_cast<M4riRec *>(rec));
    return hipGetLastError();
}

hipError_t launch_m4ri_update(uint64_t *A, int64_t stride, int m, int wc, const int32_t *rk, int b,
                              int w_lo, int w_hi, int k, int tables, const uint64_t *linv,
                              const void *rec, uint64_t *cbuf, const uint64_t *Bbuf,
                              int64_t bstride, int target_blocks, hipStream_t st) {
    const M4riRec *rc = reinterpret_cast<const M4riRec *>(rec);
    int mb = (m + M4_THREADS - 1) / M4_THREADS;
    mb = std::max(1, std::min(mb, target_blocks));
    hipLaunchKernelGGL(m4ri_mult_kernel, dim3(mb), dim3(M4_THREADS), 0, st, A, stride, m, wc, rk, b,
                       linv, rc, cbuf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || w_hi <= w_lo) return e;
    int TW = m4ri_tile_words(k, tables);
    if (TW > w_hi - w_lo) TW = w_hi - w_lo;
    const int ny = (w_hi - w_lo + TW - 1) / TW;
    const size_t lds = m4ri_lds_bytes(k, tables, TW);
    if (lds > (size_t)M4_LDS_MAX) return hipErrorInvalidValue;
    const int occ = std::max(1, (int)((160 * 1024) / lds));
    const int lg_tpr = TW >= 4 ? 2 : (TW >= 2 ? 1 : 0);
    const int rpb = M4_THREADS >> lg_tpr;
    int nx = (m + rpb - 1) / rpb;
    const int fit = std::max(1, target_blocks * occ / ny);
    if (nx > fit) nx = fit;
    if (nx < 1) nx = 1;
    static bool attr_set = false;
    if (!attr_set) {
        e = hipFuncSetAttribute((const void *)m4ri_update_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, M4_LDS_MAX);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(m4ri_update_kernel, dim3(nx, ny), dim3(M4_THREADS), lds, st, A, stride, m, rk,
                       b, w_lo, w_hi, k, tables, TW, lg_tpr, rc, cbuf, Bbuf, bstride);
    return hipGetLastError();
}

hipError_t launch_m4ri_density(const uint64_t *A, int64_t stride, int m, int n, int w0,
                               const int32_t *rk, int b, int32_t *out, hipStream_t st) {
    hipLaunchKernelGGL(m4ri_density_kernel, dim3(1), dim3(256), 0, st, A, stride, m, n, w0, rk, b,
                       out);
    return hipGetLastError();
}

hipError_t launch_gather_cols(const uint64_t *X, int64_t sx, int rows, int nw, const uint64_t *PM,
                              const int32_t *prefP, uint64_t *C, int64_t sc, hipStream_t st) {
    const int64_t total = (int64_t)rows * nw;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, sx, rows, nw,
                       PM, prefP, C, sc);
    return hipGetLastError();
}

hipError_t launch_mp_finish(int32_t *Q, int32_t *rank, int32_t *ext, const int32_t *Q2,
                            const int32_t *rank2, int R, int c0, int n, hipStream_t st) {
    int blocks = (n - R + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(mp_finish_kernel, dim3(blocks), dim3(256), 0, st, Q, rank, ext, Q2, rank2, R,
                       c0, n);
    return hipGetLastError();
}

}  // namespace gf2

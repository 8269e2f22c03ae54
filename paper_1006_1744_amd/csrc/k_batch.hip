// Batched PLS: many independent matrices of uneven shape in one persistent
// launch.  Each block of 256 threads takes the next matrix from a queue
// (largest estimated cost first) and factors it alone with the MMPF base case
// of Section 4.1 over all of its columns: for every 64-column panel, the panel
// search (PlsSubmatrix re-planned for one wave), the final pass of the pending
// pivots and the "compress L" swaps, the moves of the pivot rows' other words,
// then the table-driven solve of the pivot rows and update of the rows below
// (MakeTable / AddRowsFromTable with the block's k and table count); at the
// end the L columns of panels with fewer than 64 pivots are compressed.  The
// result is that of Gaussian PLS (Appendix A) for every matrix.
//
// The queue order comes from a counting sort of the matrices by a cost bucket
// (floor(log2(m * words^2))), built on the device so that the whole call is
// graph-capturable; the order only affects load balance.
#include "../../include/gf2pls.h"
#include "gf2_panel.h"

namespace gf2 {

constexpr int BT_THREADS = LEAF_THREADS;
constexpr int BT_MAXW = GF2_BATCH_MAX_N / 64;
constexpr int BT_TWMAX = 8;
constexpr int BT_TABLE_LDS = 16 * 1024;   // B tables of one pass
constexpr int BT_MOVE_W = 8;              // words per staged move chunk
constexpr int BT_BUCKETS = 64;

struct BatchPostLds {
    uint64_t sT[8][256];
    uint64_t sU[64];
    int32_t sQ[64];
    uint64_t stage[kMaxMoved * BT_MOVE_W];
    int32_t sDst[kMaxMoved], sSrc[kMaxMoved];
};

struct BatchUpdLds {
    uint64_t sLT[8 * 256];   // combinations of 8 rows of L^{-1}
    uint64_t sInv[64];
    uint64_t sB[64 * BT_TWMAX];
    uint64_t sTab[BT_TABLE_LDS / 8];
};

struct BatchLds {
    union {
        SearchLds search;
        BatchPostLds post;
        BatchUpdLds upd;
    } u;
    PanelInfo info;
    int32_t rk[BT_MAXW + 1];
    int job;
};

__device__ inline int batch_tile_words(int k, int tables) {
    const int tw = BT_TABLE_LDS / (tables * (1 << k) * 8);
    return tw < 1 ? 1 : (tw > BT_TWMAX ? BT_TWMAX : tw);
}

// Final pass and moves after the search of panel b (rows [R, m)).
__device__ void batch_post(uint64_t *A, int64_t stride, int m, int nw, int b, int R, BatchLds &S) {
    BatchPostLds &L = S.u.post;
    const PanelInfo &I = S.info;
    const int tid = threadIdx.x;
    const int mrem = m - R;
    const int r = I.r, F = I.F, pa = I.pa, cmp = I.compress;
    const bool pend = F < mrem && r > pa;
    if (pend || cmp) {
        if (tid < 64) {
            L.sU[tid] = I.u[tid];
            L.sQ[tid] = I.q[tid];
        }
        __syncthreads();
        if (pend) build_tables<BT_THREADS>(L.sU, L.sQ, pa, r, L.sT, tid);
        __syncthreads();
        uint64_t *col = A + (int64_t)R * stride + b;
        for (int o = tid; o < mrem; o += BT_THREADS) {
            const uint64_t v = col[(int64_t)o * stride];
            uint64_t w = v;
            if (pend && o >= F) w = apply_tables(w, L.sQ, pa, r, L.sT);
            if (cmp) {
                const int lim = min(o + 1, r);
                for (int s2 = 0; s2 < lim; s2++) {
                    const int qs = L.sQ[s2];
                    if (qs != s2) {
                        const uint64_t d = ((w >> s2) ^ (w >> qs)) & 1ull;
                        w ^= (d << s2) | (d << qs);
                    }
                }
            }
            if (w != v) col[(int64_t)o * stride] = w;
        }
    }
    const int nk = I.moved[0];
    if (nk > 0 && nw > 1) {
        if (tid < nk) {
            L.sDst[tid] = I.moved[1 + 2 * tid];
            L.sSrc[tid] = I.moved[2 + 2 * tid];
        }
        __syncthreads();
        for (int w0 = 0; w0 < nw; w0 += BT_MOVE_W) {
            for (int e = tid; e < nk * BT_MOVE_W; e += BT_THREADS) {
                const int kk = e / BT_MOVE_W, w = w0 + e % BT_MOVE_W;
                if (w < nw && w != b) L.stage[e] = A[(int64_t)(R + L.sSrc[kk]) * stride + w];
            }
            __syncthreads();
            for (int e = tid; e < nk * BT_MOVE_W; e += BT_THREADS) {
                const int kk = e / BT_MOVE_W, w = w0 + e % BT_MOVE_W;
                if (w < nw && w != b) A[(int64_t)(R + L.sDst[kk]) * stride + w] = L.stage[e];
            }
            __syncthreads();
        }
    }
    __syncthreads();
}

// Solve of the pivot rows [R, R + r) and update of the rows below on words
// [b + 1, nw): U = L^{-1} B for the pivot rows, x += (l L^{-1}) B below, B the
// pivot rows' words staged in LDS before any is rewritten.
__device__ void batch_update(uint64_t *A, int64_t stride, int m, int nw, int b, int R, int r,
                             int k, int tables, BatchLds &S) {
    BatchUpdLds &U = S.u.upd;
    const int tid = threadIdx.x;
    const int R1 = R + r;
    if (tid < 64) U.sInv[tid] = S.info.linv[tid];
    __syncthreads();
    build_tables_8x8<BT_THREADS>(U.sInv, U.sLT, tid);
    const int TW = batch_tile_words(k, tables);
    const int ng = (r + k - 1) / k, npass = (ng + tables - 1) / tables;
    const int esz = 1 << k;
    const uint32_t kmask = (1u << k) - 1;
    const int wq = tid % TW, pq = tid / TW, pstep = BT_THREADS / TW;
    for (int w0 = b + 1; w0 < nw; w0 += TW) {
        const int tw_n = min(TW, nw - w0);
        if (pq < pstep)
            for (int t = pq; t < r; t += pstep)
                U.sB[t * TW + wq] = wq < tw_n ? A[(int64_t)(R + t) * stride + w0 + wq] : 0ull;
        __syncthreads();
        uint64_t y0 = 0, y1 = 0;   // pivot outputs (t = pq, pq + pstep)
        for (int pass = 0; pass < npass; pass++) {
            const int g0 = pass * tables, g1 = min(ng, g0 + tables);
            if (pass > 0) __syncthreads();
            build_group_tables(U.sB + (size_t)g0 * k * TW, r - g0 * k, k, g1 - g0, U.sTab, TW, tid,
                               BT_THREADS);
            if (pq < pstep && wq < tw_n) {
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    const int t = pq + j * pstep;
                    if (t < r) {
                        const uint64_t ct = U.sInv[t];
                        uint64_t y = 0;
                        for (int g = g0; g < g1; g++)
                            y ^= U.sTab[((g - g0) * esz + (int)((ct >> (k * g)) & kmask)) * TW + wq];
                        if (j == 0) y0 ^= y; else y1 ^= y;
                    }
                }
            }
            for (int i = R1 + tid; i < m; i += BT_THREADS) {
                const uint64_t l = A[(int64_t)i * stride + b];
                uint64_t *px = A + (int64_t)i * stride + w0;
                uint64_t x[BT_TWMAX];
#pragma unroll
                for (int w = 0; w < BT_TWMAX; w++)
                    if (w < tw_n) x[w] = px[w];
                uint64_t c = 0;
#pragma unroll
                for (int g8 = 0; g8 < 8; g8++) c ^= U.sLT[g8 * 256 + (int)((l >> (8 * g8)) & 255)];
                for (int g = g0; g < g1; g++) {
                    const uint64_t *T = U.sTab + ((size_t)(g - g0) * esz + ((c >> (k * g)) & kmask)) * TW;
#pragma unroll
                    for (int w = 0; w < BT_TWMAX; w++)
                        if (w < tw_n) x[w] ^= T[w];
                }
#pragma unroll
                for (int w = 0; w < BT_TWMAX; w++)
                    if (w < tw_n) px[w] = x[w];
            }
        }
        if (pq < pstep && wq < tw_n) {
            if (pq < r) A[(int64_t)(R + pq) * stride + w0 + wq] = y0;
            if (pq + pstep < r) A[(int64_t)(R + pq + pstep) * stride + w0 + wq] = y1;
        }
        __syncthreads();
    }
}

// PLS of one matrix by the whole block; returns the rank.
__device__ int batch_pls_one(uint64_t *A, int64_t stride, int m, int n, int32_t *P, int32_t *Q,
                             int k, int tables, BatchLds &S) {
    const int tid = threadIdx.x;
    const int nw = (n + 63) / 64;
    int R = 0;
    if (tid == 0) S.rk[0] = 0;
    for (int b = 0; b < nw; b++) {
        __syncthreads();   // keeps each panel's thread-0 steps inside its own iteration
        int r = 0;
        if (R < m) {
            r = panel_search(A, stride, m, n, b, R, P, Q, &S.info, S.u.search);
            batch_post(A, stride, m, nw, b, R, S);
            if (r > 0 && b + 1 < nw) batch_update(A, stride, m, nw, b, R, r, k, tables, S);
        }
        R += r;
        if (tid == 0) S.rk[b + 1] = R;
    }
    __syncthreads();
    // L columns of panels with fewer than 64 pivots: innermost split first
    const int Re = S.rk[nw];
    bool any = false;
    for (int p = 0; p + 1 < nw; p++)
        if (S.rk[p + 1] - S.rk[p] < 64 && Re > S.rk[p + 1]) any = true;
    if (any)
        for (int i = S.rk[1] + tid; i < m; i += BT_THREADS) {
            uint64_t *row = A + (int64_t)i * stride;
            for (int p = nw - 2; p >= 0; p--) {
                const int Rp = S.rk[p], Rm = S.rk[p + 1];
                const int r0 = Rm - Rp, r1 = Re - Rm;
                if (r0 < 64 && r1 > 0 && i >= Rm) shift_row(row, stride, 64 * p, 64, r0, r1, i - Rm);
            }
        }
    const int mx = m > n ? m : n;
    for (int i = R + tid; i < mx; i += BT_THREADS) {
        if (i < m) P[i] = i;
        if (i < n) Q[i] = i;
    }
    __syncthreads();
    return R;
}

__device__ inline bool batch_item_ok(const gf2_batch_item &it) {
    if (it.m < 0 || it.n < 0 || it.n > GF2_BATCH_MAX_N || it.m > GF2_BATCH_MAX_M) return false;
    if (it.stride < (it.n + 63) / 64) return false;
    if (it.m > 0 && it.n > 0 && (!it.words || ((uintptr_t)it.words & 7))) return false;
    if (it.m > 0 && !it.P) return false;
    if (it.n > 0 && !it.Q) return false;
    return true;
}

__device__ inline bool batch_sched_ok(const gf2_sched &s) {
    return s.k >= 4 && s.k <= 8 &&
           (s.tables == 1 || s.tables == 2 || s.tables == 4 || s.tables == 8);
}

// The loop below is written so that every thread runs every iteration in step:
// each iteration opens with a barrier (which the compiler may not duplicate),
// so a "thread 0 only" test at the end of one iteration and the one at the
// start of the next cannot be merged into a second loop entry, and the job
// index is broadcast from one lane so that the exit test is uniform.
__global__ __launch_bounds__(BT_THREADS) void pls_batched_kernel(
    const gf2_batch_item *items, int count, const int32_t *order, int32_t *counter,
    int32_t *ranks, const gf2_sched *per, gf2_sched def) {
    __shared__ BatchLds S;
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) S.job = atomicAdd(counter, 1);
        __syncthreads();
        const int jq = __builtin_amdgcn_readfirstlane(S.job);
        if (jq >= count) break;
        const int j = order[jq];
        const gf2_batch_item it = items[j];
        int rank = GF2_E_ARG;
        if (batch_item_ok(it)) {
            gf2_sched s = def;
            if (per) {
                const gf2_sched pj = per[j];
                if (batch_sched_ok(pj)) s = pj;
            }
            if (it.m > 0 && it.n > 0) {
                rank = batch_pls_one(it.words, it.stride, (int)it.m, (int)it.n, it.P, it.Q, s.k,
                                     s.tables, S);
            } else {
                for (int i = threadIdx.x; i < it.m; i += BT_THREADS) it.P[i] = i;
                for (int i = threadIdx.x; i < it.n; i += BT_THREADS) it.Q[i] = i;
                rank = 0;
            }
        }
        if (threadIdx.x == 0) ranks[j] = rank;
    }
}

// --------------------------------------------------------------- queue order
__device__ inline int batch_bucket(const gf2_batch_item &it) {
    // sizes outside the batched range (rejected later) count as the largest
    if (it.m > GF2_BATCH_MAX_M || it.n > GF2_BATCH_MAX_N) return 0;
    const unsigned long long nw = it.n > 0 ? (unsigned long long)(it.n + 63) / 64 : 1;
    const unsigned long long cost = (it.m > 0 ? (unsigned long long)it.m : 1ull) * nw * nw;
    const int lg = 63 - __clzll(cost);   // cost >= 1 and < 2^37
    return BT_BUCKETS - 1 - min(max(lg, 0), BT_BUCKETS - 1);   // larger cost, earlier
}

__global__ void batch_hist_kernel(const gf2_batch_item *items, int count, int32_t *hist) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < count) atomicAdd(&hist[batch_bucket(items[j])], 1);
}

__global__ void batch_scan_kernel(const int32_t *hist, int32_t *cursor, int32_t *counter) {
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < BT_BUCKETS; i++) {
            cursor[i] = acc;
            acc += hist[i];
        }
        *counter = 0;
    }
}

__global__ void batch_scatter_kernel(const gf2_batch_item *items, int count, int32_t *cursor,
                                     int32_t *order) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < count) order[atomicAdd(&cursor[batch_bucket(items[j])], 1)] = j;
}

// Copy of every item's words from `src` to `dst` (same shapes), one block per
// item: restores the inputs between timed runs.
__global__ void batch_copy_kernel(const gf2_batch_item *src, const gf2_batch_item *dst, int count) {
    for (int j = blockIdx.x; j < count; j += gridDim.x) {
        const gf2_batch_item a = src[j], b = dst[j];
        if (a.m != b.m || a.n != b.n || a.m <= 0 || a.n <= 0 || !a.words || !b.words) continue;
        const int64_t nw = (a.n + 63) / 64;
        for (int64_t e = threadIdx.x; e < a.m * nw; e += blockDim.x) {
            const int64_t i = e / nw, w = e % nw;
            b.words[i * b.stride + w] = a.words[i * a.stride + w];
        }
    }
}

hipError_t launch_batch_copy(const gf2_batch_item *src, const gf2_batch_item *dst, int count,
                             hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int grid = count < 4096 ? count : 4096;
    hipLaunchKernelGGL(batch_copy_kernel, dim3(grid), dim3(256), 0, st, src, dst, count);
    return hipGetLastError();
}

size_t batch_ws_bytes(int64_t count) {
    return (size_t)(2 * BT_BUCKETS + 64) * 4 + (size_t)count * 4;
}

hipError_t launch_pls_batched(const gf2_batch_item *items, int count, int32_t *ranks,
                              const gf2_sched *per, gf2_sched def, int32_t *ws, int grid,
                              hipStream_t st) {
    int32_t *hist = ws, *cursor = ws + BT_BUCKETS, *counter = ws + 2 * BT_BUCKETS;
    int32_t *order = ws + 2 * BT_BUCKETS + 64;
    hipError_t e = launch_fill_i32(hist, 0, BT_BUCKETS, st);
    if (e != hipSuccess) return e;
    const int nb = (count + 255) / 256;
    hipLaunchKernelGGL(batch_hist_kernel, dim3(nb), dim3(256), 0, st, items, count, hist);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(batch_scan_kernel, dim3(1), dim3(64), 0, st, hist, cursor, counter);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(batch_scatter_kernel, dim3(nb), dim3(256), 0, st, items, count, cursor,
                       order);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(pls_batched_kernel, dim3(grid), dim3(BT_THREADS), 0, st, items, count, order,
                       counter, ranks, per, def);
    return hipGetLastError();
}

int batch_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)pls_batched_kernel,
                                                     BT_THREADS, 0) != hipSuccess)
        return 1;
    return n < 1 ? 1 : n;
}

}  // namespace gf2

// Kernels of the linear-system solver and the null-space basis built on a PLS
// decomposition (the decomposition as the building block for solving systems,
// abstract and Section 1).  With P A = L S:
//   A X = B  <=>  L S X = P B:  Y = P B; Y[0, r) <- L_top^{-1} Y[0, r) (forward
//   substitution); the system is consistent exactly when Y[r, m) equals
//   L_bottom Y[0, r); then X[Q[i]] = (U_Q^{-1} Y[0, r))[i] with U_Q = S[:, Q] and
//   every non-pivot entry zero (back substitution).
//   A x = 0  <=>  S x = 0: one basis vector per non-pivot column f, x[f] = 1,
//   x[Q] = U_Q^{-1} S[:, f], i.e. the non-pivot columns of the RREF transposed.
// The triangular solves and products reuse the kernels of the decomposition;
// the kernels here turn the transposition vector P into a gather map, move rows
// and scatter results by the pivot columns.
#include "gf2_internal.h"

namespace gf2 {

namespace {
__device__ inline int clamp_rank_s(const int32_t *rank, int rmax) {
    return min(max(*rank, 0), rmax);
}

__device__ inline uint64_t pdep_bits(uint64_t x, uint64_t mask) {
    uint64_t out = 0;
    int k = 0;
    while (mask) {
        const int p = __ffsll((unsigned long long)mask) - 1;
        out |= ((x >> k) & 1ull) << p;
        k++;
        mask &= mask - 1;
    }
    return out;
}

// Bits [off, off + cnt) of a packed row (cnt <= 64), as the low bits of a word.
__device__ inline uint64_t read_bits(const uint64_t *row, int off, int cnt) {
    if (cnt <= 0) return 0ull;
    const int o = off >> 6, sh = off & 63;
    uint64_t v = row[o] >> sh;
    if (sh && sh + cnt > 64) v |= row[o + 1] << (64 - sh);
    return cnt == 64 ? v : (v & ((1ull << cnt) - 1));
}
}  // namespace

// ------------------------------------------------------ transpositions -> map
// Step j < r exchanged positions j and P[j] >= j.  A value's trajectory: it
// stays at its position p until the first later step that touches p, either a
// step j < p with P[j] = p (the value moves to j, where no later step reaches:
// final) or step p itself (the value moves to P[p] and waits there, final at p
// when P[p] = p).  The steps targeting each position are listed once (counting
// sort), and every value walks its own trajectory; the result is
// perm[final position] = original position.

// cnt[P[j]] += 1 for every j < r with P[j] != j (cnt zero on entry).
__global__ void swap_count_kernel(const int32_t *P, const int32_t *rank, int m, int rmax,
                                  int32_t *cnt) {
    const int r = clamp_rank_s(rank, rmax);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < r; j += gridDim.x * blockDim.x) {
        const int p = P[j];
        if (p != j && p > j && p < m) atomicAdd(&cnt[p], 1);
    }
}

// Exclusive prefix sums of cnt[0, m) into off[0, m] (one block), and fill = 0.
__global__ __launch_bounds__(1024) void swap_scan_kernel(const int32_t *cnt, int32_t *off,
                                                         int32_t *fill, int m) {
    __shared__ int32_t s[1024];
    const int tid = threadIdx.x;
    const int per = (m + 1023) / 1024;
    const int a = tid * per, b = min(m, a + per);
    int c = 0;
    for (int i = a; i < b; i++) c += cnt[i];
    s[tid] = c;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int v = tid >= d ? s[tid - d] : 0;
        __syncthreads();
        s[tid] += v;
        __syncthreads();
    }
    int e = s[tid] - c;
    for (int i = a; i < b; i++) {
        off[i] = e;
        e += cnt[i];
        fill[i] = 0;
    }
    if (tid == 1023) off[m] = s[1023];
}

__global__ void swap_fill_kernel(const int32_t *P, const int32_t *rank, int m, int rmax,
                                 const int32_t *off, int32_t *fill, int32_t *list) {
    const int r = clamp_rank_s(rank, rmax);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < r; j += gridDim.x * blockDim.x) {
        const int p = P[j];
        if (p != j && p > j && p < m) list[off[p] + atomicAdd(&fill[p], 1)] = j;
    }
}

__global__ void swap_walk_kernel(const int32_t *P, const int32_t *rank, int m, int rmax,
                                 const int32_t *off, const int32_t *list, int32_t *perm) {
    const int r = clamp_rank_s(rank, rmax);
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < m; x += gridDim.x * blockDim.x) {
        int pos = x, time = 0;
        while (true) {
            // first step in [time, pos) that targets pos
            int e = 0x7fffffff;
            for (int k = off[pos]; k < off[pos + 1]; k++) {
                const int j = list[k];
                if (j >= time && j < e) e = j;
            }
            if (e != 0x7fffffff) { pos = e; break; }
            if (pos >= r) break;
            const int p = P[pos];
            if (p == pos || p < pos || p >= m) break;
            time = pos + 1;
            pos = p;
        }
        perm[pos] = x;
    }
}

// Y[i] <- B[perm[i]] (nrw words per row).
__global__ void gather_rows_kernel(uint64_t *Y, int64_t sy, const uint64_t *B, int64_t sb,
                                   const int32_t *perm, int m, int nrw) {
    const int64_t total = (int64_t)m * nrw;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / nrw), w = (int)(e % nrw);
        Y[(int64_t)i * sy + w] = B[(int64_t)perm[i] * sb + w];
    }
}

// ext = {0, r, nrw}: row extents of the forward and back substitutions.
__global__ void solve_extents_kernel(const int32_t *rank, int rmax, int nrw, int32_t *ext) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ext[0] = 0;
        ext[1] = clamp_rank_s(rank, rmax);
        ext[2] = nrw;
    }
}

// bad[w] |= OR of Y rows [r, m) on word w (bad zero on entry): a set bit marks
// a right-hand side whose remaining rows L_bottom Y_top did not cancel.
__global__ void consistency_kernel(const uint64_t *Y, int64_t sy, int m, int nrw,
                                   const int32_t *ext, uint64_t *bad) {
    const int r = ext[1];
    const int w = blockIdx.y;
    uint64_t acc = 0;
    for (int i = r + blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
        acc |= Y[(int64_t)i * sy + w];
    // one atomic per wave
    for (int d = 32; d >= 1; d >>= 1) acc |= __shfl_xor(acc, d);
    if ((threadIdx.x & 63) == 0 && acc) atomicOr((unsigned long long *)&bad[w], acc);
}

// X row j (j < n): Y row i when j = Q[i] is the i-th pivot column (i from the
// pivot mask's prefix counts), else zero.
__global__ void solve_scatter_kernel(uint64_t *X, int64_t sx, int n, int nrw, const uint64_t *Y,
                                     int64_t sy, const uint64_t *PM, const int32_t *prefP) {
    const int64_t total = (int64_t)n * nrw;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / nrw), w = (int)(e % nrw);
        const uint64_t pm = PM[j >> 6];
        uint64_t v = 0;
        if ((pm >> (j & 63)) & 1ull) {
            const int i = prefP[j >> 6] + __popcll(pm & ((1ull << (j & 63)) - 1));
            v = Y[(int64_t)i * sy + w];
        }
        X[(int64_t)j * sx + w] = v;
    }
}

// Null-space basis row j < n - r: a one at the j-th non-pivot column N[j] and,
// at pivot column Q[i], bit i of row j of XT (the transposed solved block
// U_Q^{-1} S[:, N]); rows n - r .. n - 1 zero.  One thread per (row, word).
__global__ void kernel_scatter_kernel(uint64_t *K, int64_t sk, int n, const uint64_t *XT,
                                      int64_t sxt, const uint64_t *PM, const uint64_t *NM,
                                      const int32_t *prefP, const int32_t *prefN,
                                      const int32_t *ext) {
    const int r = ext[1];
    const int nw = (n + 63) / 64;
    const int64_t total = (int64_t)n * nw;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / nw), w = (int)(e % nw);
        uint64_t v = 0;
        if (j < n - r) {
            const uint64_t pm = PM[w];
            const int cnt = __popcll(pm);
            if (cnt) v = pdep_bits(read_bits(XT + (int64_t)j * sxt, prefP[w], cnt), pm);
            // the j-th non-pivot column lies in word w when prefN[w] <= j < prefN[w + 1]
            if (prefN[w] <= j && j < prefN[w + 1]) {
                uint64_t nm = NM[w];
                for (int t = prefN[w]; t < j; t++) nm &= nm - 1;
                v |= nm & (~nm + 1);
            }
        }
        K[(int64_t)j * sk + w] = v;
    }
}

namespace {
int blocks_for(int64_t total, int64_t cap) {
    int64_t b = (total + 255) / 256;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}
}  // namespace

hipError_t launch_perm_from_swaps(const int32_t *P, const int32_t *rank, int m, int rmax,
                                  int32_t *cnt, int32_t *off, int32_t *fill, int32_t *list,
                                  int32_t *perm, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipError_t e = launch_fill_i32(cnt, 0, m, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(swap_count_kernel, dim3(blocks_for(rmax, 1024)), dim3(256), 0, st, P, rank, m,
                       rmax, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(swap_scan_kernel, dim3(1), dim3(1024), 0, st, cnt, off, fill, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(swap_fill_kernel, dim3(blocks_for(rmax, 1024)), dim3(256), 0, st, P, rank, m,
                       rmax, off, fill, list);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(swap_walk_kernel, dim3(blocks_for(m, 4096)), dim3(256), 0, st, P, rank, m,
                       rmax, off, list, perm);
    return hipGetLastError();
}

hipError_t launch_gather_rows(uint64_t *Y, int64_t sy, const uint64_t *B, int64_t sb,
                              const int32_t *perm, int m, int nrw, hipStream_t st) {
    if ((int64_t)m * nrw <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for((int64_t)m * nrw, 8192)), dim3(256), 0, st,
                       Y, sy, B, sb, perm, m, nrw);
    return hipGetLastError();
}

hipError_t launch_solve_extents(const int32_t *rank, int rmax, int nrw, int32_t *ext,
                                hipStream_t st) {
    hipLaunchKernelGGL(solve_extents_kernel, dim3(1), dim3(64), 0, st, rank, rmax, nrw, ext);
    return hipGetLastError();
}

hipError_t launch_consistency(const uint64_t *Y, int64_t sy, int m, int nrw, const int32_t *ext,
                              uint64_t *bad, hipStream_t st) {
    if (nrw <= 0) return hipSuccess;
    hipError_t e = launch_zero_rows(bad, nrw, 1, nrw, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(consistency_kernel, dim3(blocks_for(m, 256), nrw), dim3(256), 0, st, Y, sy, m,
                       nrw, ext, bad);
    return hipGetLastError();
}

hipError_t launch_solve_scatter(uint64_t *X, int64_t sx, int n, int nrw, const uint64_t *Y,
                                int64_t sy, const uint64_t *PM, const int32_t *prefP,
                                hipStream_t st) {
    if ((int64_t)n * nrw <= 0) return hipSuccess;
    hipLaunchKernelGGL(solve_scatter_kernel, dim3(blocks_for((int64_t)n * nrw, 8192)), dim3(256), 0,
                       st, X, sx, n, nrw, Y, sy, PM, prefP);
    return hipGetLastError();
}

hipError_t launch_kernel_scatter(uint64_t *K, int64_t sk, int n, const uint64_t *XT, int64_t sxt,
                                 const uint64_t *PM, const uint64_t *NM, const int32_t *prefP,
                                 const int32_t *prefN, const int32_t *ext, hipStream_t st) {
    const int nw = (n + 63) / 64;
    if ((int64_t)n * nw <= 0) return hipSuccess;
    hipLaunchKernelGGL(kernel_scatter_kernel, dim3(blocks_for((int64_t)n * nw, 16384)), dim3(256), 0,
                       st, K, sk, n, XT, sxt, PM, NM, prefP, prefN, ext);
    return hipGetLastError();
}

}  // namespace gf2

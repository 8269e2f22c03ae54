// Reduced row echelon form from a PLS decomposition (the RREF timed together
// with the decomposition in the paper's Table 1; Definition of the RREF,
// Section 2).  With S the echelon rows (pivot i at column Q[i]) and U = S[:, Q]
// (unit upper triangular), R = U^{-1} S: R[:, Q] = I and the non-pivot columns
// are U^{-1} S[:, N].  The kernels here gather S[:, Q] and S[:, N] into compact
// matrices, and scatter the solved block back; the solve itself reuses the
// triangular-solve and product kernels.
#include "gf2_internal.h"

namespace gf2 {

__device__ inline uint64_t pext64(uint64_t x, uint64_t mask) {
    if (mask == ~0ull) return x;
    uint64_t out = 0;
    int k = 0;
    while (mask) {
        int p = __ffsll((unsigned long long)mask) - 1;
        out |= ((x >> p) & 1ull) << k;
        k++;
        mask &= mask - 1;
    }
    return out;
}

__device__ inline uint64_t pdep64(uint64_t x, uint64_t mask) {
    if (mask == ~0ull) return x;
    uint64_t out = 0;
    int k = 0;
    while (mask) {
        int p = __ffsll((unsigned long long)mask) - 1;
        out |= ((x >> k) & 1ull) << p;
        k++;
        mask &= mask - 1;
    }
    return out;
}

// A rank outside [0, rmax] (not a gf2_pls result) is clamped into it.
__device__ inline int clamp_rank(const int32_t *rank, int rmax) {
    return min(max(*rank, 0), rmax);
}

// Pivot mask from Q[0..r): set bit Q[t].  PM must be zero on entry.
__global__ void pivot_mask_kernel(uint64_t *PM, const int32_t *Q, const int32_t *rank, int rmax) {
    const int r = clamp_rank(rank, rmax);
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < r; t += gridDim.x * blockDim.x) {
        int q = Q[t];
        atomicOr((unsigned long long *)&PM[q >> 6], 1ull << (q & 63));
    }
}

// NM = ~PM inside [0, n); exclusive prefix sums of popcounts (one block).
// Also the solve's extents rr = {0, r, ceil((n - r) / 64)}.
__global__ __launch_bounds__(1024) void mask_prefix_kernel(const uint64_t *PM, uint64_t *NM,
                                                           int32_t *prefP, int32_t *prefN, int n,
                                                           const int32_t *rank, int rmax,
                                                           int32_t *rr) {
    __shared__ int32_t sp[1024], sn[1024];
    const int nw = (n + 63) / 64;
    const int tid = threadIdx.x;
    if (tid == 0) {
        const int r = clamp_rank(rank, rmax);
        rr[0] = 0;
        rr[1] = r;
        rr[2] = (n - r + 63) / 64;
    }
    const int per = (nw + 1023) / 1024;
    const int w0 = tid * per, w1 = min(nw, w0 + per);
    int cp = 0, cn = 0;
    for (int w = w0; w < w1; w++) {
        uint64_t valid = (w == nw - 1 && (n & 63)) ? ((1ull << (n & 63)) - 1) : ~0ull;
        uint64_t nm = ~PM[w] & valid;
        NM[w] = nm;
        cp += __popcll(PM[w]);
        cn += __popcll(nm);
    }
    sp[tid] = cp;
    sn[tid] = cn;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int vp = tid >= off ? sp[tid - off] : 0;
        int vn = tid >= off ? sn[tid - off] : 0;
        __syncthreads();
        sp[tid] += vp;
        sn[tid] += vn;
        __syncthreads();
    }
    int ep = sp[tid] - cp, en = sn[tid] - cn;   // exclusive
    for (int w = w0; w < w1; w++) {
        prefP[w] = ep;
        prefN[w] = en;
        ep += __popcll(PM[w]);
        en += __popcll(NM[w]);
    }
    if (tid == 1023) {
        prefP[nw] = sp[1023];
        prefN[nw] = sn[1023];
    }
}

__device__ inline void or_bits(uint64_t *row, int off, int cnt, uint64_t v) {
    if (cnt <= 0 || v == 0) return;
    int o = off >> 6, sh = off & 63;
    atomicOr((unsigned long long *)&row[o], v << sh);
    if (sh && sh + cnt > 64) atomicOr((unsigned long long *)&row[o + 1], v >> (64 - sh));
}

// Row i < r of S (pivot one at Q[i], zeros left of it, the stored bits right of
// it) compressed by PM into Uc and by NM into Xc.  Uc, Xc zero on entry.  One
// thread per (row, word), the word index fastest, so neighbouring threads read
// neighbouring words of a row and OR into neighbouring words of its compact rows.
// Xc == nullptr: U_Q alone (the solver needs it whatever the non-pivot columns).
__global__ void rref_gather_kernel(const uint64_t *Ap, int64_t sap, const int32_t *Q, int nw,
                                   const uint64_t *PM, const uint64_t *NM, const int32_t *prefP,
                                   const int32_t *prefN, uint64_t *Uc, int64_t su, uint64_t *Xc,
                                   int64_t sx, const int32_t *rr) {
    if (Xc && rr[2] == 0) return;   // no non-pivot column: nothing to solve
    const int r = rr[1];
    const int64_t total = (int64_t)r * nw;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / nw), w = (int)(e % nw);
        const int q = Q[i];
        const int qw = q >> 6;
        if (w < qw) continue;   // S is zero left of the pivot word
        const uint64_t pm = PM[w], nm = NM[w];
        const int cpp = __popcll(pm), cnn = __popcll(nm);
        uint64_t x = Ap[(int64_t)i * sap + w];
        if (w == qw) {
            const int qb = q & 63;
            uint64_t above = qb == 63 ? 0ull : (~0ull << (qb + 1));
            x = (x & above) | (1ull << qb);
        }
        if (cpp) or_bits(Uc + (int64_t)i * su, prefP[w], cpp, pext64(x, pm));
        if (cnn && Xc) or_bits(Xc + (int64_t)i * sx, prefN[w], cnn, pext64(x, nm));
    }
}

// R row i: pivot one at Q[i] (i < r) and the solved non-pivot bits spread back
// by NM; rows >= r are zero.  One thread per (row, word), the word index fastest.
__global__ void rref_scatter_kernel(uint64_t *R, int64_t sr, int m, const int32_t *Q,
                                    const int32_t *rr, const uint64_t *NM, const int32_t *prefN,
                                    const uint64_t *Xc, int64_t sx, int nw) {
    const int r = rr[1];
    const int64_t total = (int64_t)m * nw;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / nw), w = (int)(e % nw);
        uint64_t out = 0;
        if (i < r) {
            const uint64_t nm = NM[w];
            const int cnt = __popcll(nm), off = prefN[w];
            if (cnt) {
                const uint64_t *xr = Xc + (int64_t)i * sx;
                int o = off >> 6, sh = off & 63;
                uint64_t v = xr[o] >> sh;
                if (sh && sh + cnt > 64) v |= xr[o + 1] << (64 - sh);
                out = pdep64(v, nm);
            }
            const int q = Q[i];
            if ((q >> 6) == w) out |= 1ull << (q & 63);
        }
        R[(int64_t)i * sr + w] = out;
    }
}

// Uc rows [0, r) x ceil(r / 64) words and Xc rows [0, r) x rr[2] words <- 0
// (nothing when there is no non-pivot column; Uc alone when Xc is null).
__global__ void rref_zero_kernel(uint64_t *Uc, int64_t su, uint64_t *Xc, int64_t sx,
                                 const int32_t *rr) {
    const int r = rr[1], nu = (r + 63) / 64;
    const int nx = Xc ? rr[2] : 0;
    if (Xc && nx == 0) return;
    const int64_t tu = (int64_t)r * nu, total = tu + (int64_t)r * nx;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e < tu)
            Uc[(e / nu) * su + (e % nu)] = 0ull;
        else
            Xc[((e - tu) / nx) * sx + ((e - tu) % nx)] = 0ull;
    }
}

hipError_t launch_rref_zero(uint64_t *Uc, int64_t su, uint64_t *Xc, int64_t sx, int rmax,
                            const int32_t *rr, hipStream_t st) {
    if (rmax <= 0) return hipSuccess;
    int64_t blocks = ((int64_t)rmax * (su + sx) + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(rref_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Uc, su, Xc, sx,
                       rr);
    return hipGetLastError();
}

__global__ void zero_rows_kernel(uint64_t *X, int64_t sx, int rows, int words) {
    int64_t total = (int64_t)rows * words;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x)
        X[(e / words) * sx + (e % words)] = 0ull;
}

hipError_t launch_zero_rows(uint64_t *X, int64_t sx, int rows, int words, hipStream_t st) {
    int64_t total = (int64_t)rows * words;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(zero_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, sx, rows,
                       words);
    return hipGetLastError();
}

hipError_t launch_rref_masks(uint64_t *PM, uint64_t *NM, int32_t *prefP, int32_t *prefN,
                             const int32_t *Q, const int32_t *rank, int n, int rmax, int32_t *rr,
                             hipStream_t st) {
    const int nw = (n + 63) / 64;
    hipError_t e = launch_zero_rows(PM, nw, 1, nw, st);
    if (e != hipSuccess) return e;
    int blocks = (rmax + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(pivot_mask_kernel, dim3(blocks), dim3(256), 0, st, PM, Q, rank, rmax);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(mask_prefix_kernel, dim3(1), dim3(1024), 0, st, PM, NM, prefP, prefN, n, rank,
                       rmax, rr);
    return hipGetLastError();
}

hipError_t launch_rref_gather(const uint64_t *Ap, int64_t sap, const int32_t *Q, int rmax, int n,
                              const uint64_t *PM, const uint64_t *NM, const int32_t *prefP,
                              const int32_t *prefN, uint64_t *Uc, int64_t su, uint64_t *Xc,
                              int64_t sx, const int32_t *rr, hipStream_t st) {
    if (rmax <= 0) return hipSuccess;
    const int nw = (n + 63) / 64;
    int64_t blocks = ((int64_t)rmax * nw + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(rref_gather_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Ap, sap, Q, nw,
                       PM, NM, prefP, prefN, Uc, su, Xc, sx, rr);
    return hipGetLastError();
}

hipError_t launch_rref_scatter(uint64_t *R, int64_t sr, int m, int n, const int32_t *Q,
                               const int32_t *rr, const uint64_t *NM, const int32_t *prefN,
                               const uint64_t *Xc, int64_t sx, hipStream_t st) {
    const int nw = (n + 63) / 64;
    if (m <= 0 || nw <= 0) return hipSuccess;
    int64_t blocks = ((int64_t)m * nw + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(rref_scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, st, R, sr, m, Q, rr,
                       NM, prefN, Xc, sx, nw);
    return hipGetLastError();
}

// Explicit factors from the compressed in-place result: L (m x r, unit lower
// trapezoidal: row i holds the stored bits of columns < min(i, r) and a one at
// column i when i < r) and S (r x n: one at Q[i], zeros left of it, the stored
// bits right of it).  One thread per output word.
__global__ void unpack_kernel(const uint64_t *A, int64_t sa, int m, int n, const int32_t *Q,
                              const int32_t *rank, uint64_t *L, int64_t sl, int lwords, uint64_t *S,
                              int64_t ss, int swords) {
    const int r = *rank;
    const int64_t totL = (int64_t)m * lwords, totS = (int64_t)r * swords;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < totL + totS;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e < totL) {
            const int i = (int)(e / lwords), w = (int)(e % lwords);
            const int k = min(i, r);   // stored L bits: columns [0, k)
            uint64_t v = 0;
            if (64 * w < k) {
                v = A[(int64_t)i * sa + w];
                const int hi = k - 64 * w;
                if (hi < 64) v &= (1ull << hi) - 1;
            }
            if (i < r && (i >> 6) == w) v |= 1ull << (i & 63);
            if (64 * w >= r) v = 0;
            else if (r - 64 * w < 64) v &= (1ull << (r - 64 * w)) - 1;
            L[(int64_t)i * sl + w] = v;
        } else {
            const int64_t f = e - totL;
            const int i = (int)(f / swords), w = (int)(f % swords);
            const int q = Q[i];
            uint64_t v = A[(int64_t)i * sa + w];
            // keep columns > q, set column q, clear the rest
            const int lo = q + 1 - 64 * w;   // first kept bit in this word
            if (lo >= 64) v = 0;
            else if (lo > 0) v &= ~0ull << lo;
            if ((q >> 6) == w) v |= 1ull << (q & 63);
            if (64 * w + 64 > n) v &= n - 64 * w >= 64 ? ~0ull : ((1ull << (n - 64 * w)) - 1);
            S[(int64_t)i * ss + w] = v;
        }
    }
}

hipError_t launch_unpack(const uint64_t *A, int64_t sa, int m, int n, const int32_t *Q,
                         const int32_t *rank, uint64_t *L, int64_t sl, int lwords, uint64_t *S,
                         int64_t ss, int swords, int64_t max_words, hipStream_t st) {
    if (max_words <= 0) return hipSuccess;
    int64_t blocks = (max_words + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(unpack_kernel, dim3((unsigned)blocks), dim3(256), 0, st, A, sa, m, n, Q, rank,
                       L, sl, lwords, S, ss, swords);
    return hipGetLastError();
}

}  // namespace gf2

// Learned cost model: an fp32 multilayer perceptron 4 -> 64 -> 64 -> S (ReLU)
// mapping the features of a problem to predicted log run times of S candidate
// schedules; the predicted schedule is the argmin.  Training minimises the
// masked mean squared error over the (problem, schedule) pairs that were
// timed, with Adam.  Everything here is plain fp32 on the vector units: the
// network is tiny and is not on the decomposition's hot path.
//
// Parameters, one contiguous fp32 array:  W1[4][64] b1[64] W2[64][64] b2[64]
// W3[64][S] b3[S]  (W[a][j] connects input a to output j).
// Input features per problem (raw): log2 m, log2 n, density, rank estimate /
// min(m, n); the network sees them scaled as (f0/16, f1/16, f2, f3).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/gf2pls.h"
#include "gf2_internal.h"

namespace gf2 {

constexpr int MLP_H = 64;
constexpr int MLP_BS = 16;        // problems per block
constexpr int MLP_THREADS = 256;

__host__ __device__ inline int64_t mlp_params(int S) {
    return 4 * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + (int64_t)MLP_H * S + S;
}

struct MlpView {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};

__device__ inline MlpView mlp_view(const float *p, int S) {
    MlpView v;
    v.W1 = p;
    v.b1 = v.W1 + 4 * MLP_H;
    v.W2 = v.b1 + MLP_H;
    v.b2 = v.W2 + MLP_H * MLP_H;
    v.W3 = v.b2 + MLP_H;
    v.b3 = v.W3 + MLP_H * S;
    return v;
}

// LDS: parameters, then per-block activations.
__host__ __device__ inline size_t mlp_lds_floats(int S) {
    return (size_t)mlp_params(S) + MLP_BS * 4 + 3 * MLP_BS * MLP_H + 3 * (size_t)MLP_BS * S;
}

struct MlpLds {
    float *par, *X, *H1, *H2, *D, *Y, *T, *M;
};

__device__ inline MlpLds mlp_lds(float *base, int S) {
    MlpLds L;
    L.par = base;
    L.X = L.par + mlp_params(S);
    L.H1 = L.X + MLP_BS * 4;
    L.H2 = L.H1 + MLP_BS * MLP_H;
    L.D = L.H2 + MLP_BS * MLP_H;
    L.Y = L.D + MLP_BS * MLP_H;
    L.T = L.Y + MLP_BS * S;
    L.M = L.T + MLP_BS * S;
    return L;
}

// Loads the parameters and the block's (scaled) features, then the forward
// pass into H1, H2 (post-ReLU) and Y.  nb = problems in this block.
__device__ void mlp_forward_block(const float *params, int S, const float *feats, int i0, int nb,
                                  const MlpLds &L) {
    const int tid = threadIdx.x;
    const int64_t np = mlp_params(S);
    for (int64_t e = tid; e < np; e += MLP_THREADS) L.par[e] = params[e];
    for (int e = tid; e < MLP_BS * 4; e += MLP_THREADS) {
        const int i = e / 4, a = e % 4;
        float f = i < nb ? feats[(int64_t)(i0 + i) * 4 + a] : 0.f;
        if (a < 2) f *= (1.0f / 16.0f);
        L.X[e] = f;
    }
    __syncthreads();
    const MlpView w = mlp_view(L.par, S);
    for (int e = tid; e < MLP_BS * MLP_H; e += MLP_THREADS) {
        const int i = e / MLP_H, j = e % MLP_H;
        float acc = w.b1[j];
        for (int a = 0; a < 4; a++) acc += L.X[i * 4 + a] * w.W1[a * MLP_H + j];
        L.H1[e] = acc > 0.f ? acc : 0.f;
    }
    __syncthreads();
    for (int e = tid; e < MLP_BS * MLP_H; e += MLP_THREADS) {
        const int i = e / MLP_H, j = e % MLP_H;
        float acc = w.b2[j];
        for (int a = 0; a < MLP_H; a++) acc += L.H1[i * MLP_H + a] * w.W2[a * MLP_H + j];
        L.H2[e] = acc > 0.f ? acc : 0.f;
    }
    __syncthreads();
    for (int e = tid; e < MLP_BS * S; e += MLP_THREADS) {
        const int i = e / S, s = e % S;
        float acc = w.b3[s];
        for (int a = 0; a < MLP_H; a++) acc += L.H2[i * MLP_H + a] * w.W3[a * S + s];
        L.Y[e] = acc;
    }
    __syncthreads();
}

__global__ __launch_bounds__(MLP_THREADS) void mlp_forward_kernel(const float *params, int S,
                                                                   const float *feats, int N,
                                                                   float *out) {
    extern __shared__ float mlp_lds_base[];
    const MlpLds L = mlp_lds(mlp_lds_base, S);
    const int i0 = blockIdx.x * MLP_BS;
    const int nb = min(MLP_BS, N - i0);
    mlp_forward_block(params, S, feats, i0, nb, L);
    for (int e = threadIdx.x; e < nb * S; e += MLP_THREADS) out[(int64_t)i0 * S + e] = L.Y[e];
}

// Per-block gradient of  loss = inv_count * sum_{i,s} M[i][s] (Y[i][s] - T[i][s])^2
// written to part[block][0 .. P) with the block's loss at part[block][P].
// Every sum runs over a fixed index order, so the result is deterministic.
__global__ __launch_bounds__(MLP_THREADS) void mlp_grad_kernel(const float *params, int S,
                                                                const float *feats,
                                                                const float *target,
                                                                const float *mask, int N,
                                                                float inv_count, float *part) {
    extern __shared__ float mlp_lds_base[];
    const MlpLds L = mlp_lds(mlp_lds_base, S);
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * MLP_BS;
    const int nb = min(MLP_BS, N - i0);
    const int64_t P = mlp_params(S);
    float *g = part + (int64_t)blockIdx.x * (P + 1);
    for (int e = tid; e < MLP_BS * S; e += MLP_THREADS) {
        const int i = e / S;
        L.T[e] = i < nb ? target[(int64_t)i0 * S + e] : 0.f;
        L.M[e] = i < nb ? mask[(int64_t)i0 * S + e] : 0.f;
    }
    mlp_forward_block(params, S, feats, i0, nb, L);
    const MlpView w = mlp_view(L.par, S);
    // dY (in place of Y) and the block's loss
    __shared__ float red[MLP_THREADS];
    float lpart = 0.f;
    for (int e = tid; e < MLP_BS * S; e += MLP_THREADS) {
        const float d = L.Y[e] - L.T[e];
        lpart += L.M[e] * d * d;
        L.Y[e] = 2.f * L.M[e] * d * inv_count;
    }
    red[tid] = lpart;
    __syncthreads();
    if (tid == 0) {
        float s = 0.f;
        for (int t = 0; t < MLP_THREADS; t++) s += red[t];
        g[P] = s * inv_count;
    }
    const int64_t oW1 = 0, ob1 = 4 * MLP_H, oW2 = ob1 + MLP_H, ob2 = oW2 + MLP_H * MLP_H,
                  oW3 = ob2 + MLP_H, ob3 = oW3 + (int64_t)MLP_H * S;
    // output layer
    for (int e = tid; e < MLP_H * S; e += MLP_THREADS) {
        const int a = e / S, s = e % S;
        float acc = 0.f;
        for (int i = 0; i < MLP_BS; i++) acc += L.H2[i * MLP_H + a] * L.Y[i * S + s];
        g[oW3 + e] = acc;
    }
    for (int s = tid; s < S; s += MLP_THREADS) {
        float acc = 0.f;
        for (int i = 0; i < MLP_BS; i++) acc += L.Y[i * S + s];
        g[ob3 + s] = acc;
    }
    for (int e = tid; e < MLP_BS * MLP_H; e += MLP_THREADS) {
        const int i = e / MLP_H, a = e % MLP_H;
        float acc = 0.f;
        for (int s = 0; s < S; s++) acc += L.Y[i * S + s] * w.W3[a * S + s];
        L.D[e] = L.H2[e] > 0.f ? acc : 0.f;
    }
    __syncthreads();
    // second layer
    for (int e = tid; e < MLP_H * MLP_H; e += MLP_THREADS) {
        const int a = e / MLP_H, b = e % MLP_H;
        float acc = 0.f;
        for (int i = 0; i < MLP_BS; i++) acc += L.H1[i * MLP_H + a] * L.D[i * MLP_H + b];
        g[oW2 + e] = acc;
    }
    for (int b = tid; b < MLP_H; b += MLP_THREADS) {
        float acc = 0.f;
        for (int i = 0; i < MLP_BS; i++) acc += L.D[i * MLP_H + b];
        g[ob2 + b] = acc;
    }
    // dH1 (into H2's storage, which is no longer needed)
    for (int e = tid; e < MLP_BS * MLP_H; e += MLP_THREADS) {
        const int i = e / MLP_H, a = e % MLP_H;
        float acc = 0.f;
        for (int b = 0; b < MLP_H; b++) acc += L.D[i * MLP_H + b] * w.W2[a * MLP_H + b];
        L.H2[e] = L.H1[e] > 0.f ? acc : 0.f;
    }
    __syncthreads();
    // first layer
    for (int e = tid; e < 4 * MLP_H; e += MLP_THREADS) {
        const int a = e / MLP_H, j = e % MLP_H;
        float acc = 0.f;
        for (int i = 0; i < MLP_BS; i++) acc += L.X[i * 4 + a] * L.H2[i * MLP_H + j];
        g[oW1 + e] = acc;
    }
    for (int j = tid; j < MLP_H; j += MLP_THREADS) {
        float acc = 0.f;
        for (int i = 0; i < MLP_BS; i++) acc += L.H2[i * MLP_H + j];
        g[ob1 + j] = acc;
    }
}

// out[p] = sum over blocks b (in order) of part[b][p], p in [0, P]
__global__ void mlp_reduce_kernel(const float *part, int nblk, int64_t width, float *out) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < width;
         p += (int64_t)gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (int b = 0; b < nblk; b++) acc += part[(int64_t)b * width + p];
        out[p] = acc;
    }
}

// Adam (Kingma & Ba, Algorithm 1) with bias correction; step t >= 1.
__global__ void mlp_adam_kernel(float *params, const float *grad, float *m1, float *m2, int64_t P,
                                float lr, float beta1, float beta2, float eps, float c1, float c2) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
         p += (int64_t)gridDim.x * blockDim.x) {
        const float gp = grad[p];
        const float a = beta1 * m1[p] + (1.f - beta1) * gp;
        const float b = beta2 * m2[p] + (1.f - beta2) * gp * gp;
        m1[p] = a;
        m2[p] = b;
        params[p] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
    }
}

// Uniform(-lim, lim) weights with lim = sqrt(6 / fan_in), zero biases; the
// uniform draws come from SplitMix64 (Steele, Lea and Flood) at counter p.
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void mlp_init_kernel(float *params, int S, uint64_t seed) {
    const int64_t P = mlp_params(S);
    const int64_t ob1 = 4 * MLP_H, oW2 = ob1 + MLP_H, ob2 = oW2 + MLP_H * MLP_H,
                  oW3 = ob2 + MLP_H, ob3 = oW3 + (int64_t)MLP_H * S;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
         p += (int64_t)gridDim.x * blockDim.x) {
        float fan = 0.f;
        if (p < ob1) fan = 4.f;
        else if (p >= oW2 && p < ob2) fan = MLP_H;
        else if (p >= oW3 && p < ob3) fan = MLP_H;
        if (fan == 0.f) {
            params[p] = 0.f;
            continue;
        }
        const float u = (float)(splitmix64_at(seed, (uint64_t)p) >> 40) * (1.0f / 16777216.0f);
        params[p] = (2.f * u - 1.f) * sqrtf(6.f / fan);
    }
}

// Forward pass, then per problem the candidate with the smallest predicted log
// time (the first on ties); out[i] = table[argmin].
__global__ __launch_bounds__(MLP_THREADS) void costmodel_predict_kernel(
    const float *params, int S, const float *feats, int N, const gf2_sched *table,
    gf2_sched *out) {
    extern __shared__ float mlp_lds_base[];
    const MlpLds L = mlp_lds(mlp_lds_base, S);
    const int i0 = blockIdx.x * MLP_BS;
    const int nb = min(MLP_BS, N - i0);
    mlp_forward_block(params, S, feats, i0, nb, L);
    for (int i = threadIdx.x; i < nb; i += MLP_THREADS) {
        int best = 0;
        float bv = L.Y[i * S];
        for (int s = 1; s < S; s++)
            if (L.Y[i * S + s] < bv) {
                bv = L.Y[i * S + s];
                best = s;
            }
        out[i0 + i] = table[best];
    }
}

// Features of problem i from its matrix: (log2 m, log2 n, density, rank
// estimate / min(m, n)); the density counts the ones of up to 256 rows spread
// evenly over the matrix (all of its words), the rank estimate is the caller's
// hint when positive, else min(m, n).  One block per problem.
__global__ __launch_bounds__(256) void features_kernel(const gf2_batch_item *items, int count,
                                                       const int32_t *r_hint, float *feats) {
    __shared__ unsigned long long s_cnt;
    const int i = blockIdx.x;
    if (i >= count) return;
    const gf2_batch_item it = items[i];
    const int64_t m = it.m, n = it.n;
    float *f = feats + 4 * (int64_t)i;
    if (m <= 0 || n <= 0 || !it.words || it.stride < (n + 63) / 64) {
        if (threadIdx.x < 4) f[threadIdx.x] = 0.f;
        return;
    }
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int S = (int)min<int64_t>(m, 256);
    const int64_t nw = (n + 63) / 64;
    if ((int)threadIdx.x < S) {
        const int64_t row = ((int64_t)threadIdx.x * m) / S;
        const uint64_t *pr = it.words + row * it.stride;
        unsigned long long c = 0;
        for (int64_t w = 0; w < nw; w++) {
            uint64_t x = pr[w];
            if (w == nw - 1 && (n & 63)) x &= (1ull << (n & 63)) - 1;
            c += __popcll(x);
        }
        atomicAdd(&s_cnt, c);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double mn = (double)min(m, n);
        const int hint = r_hint ? r_hint[i] : 0;
        f[0] = (float)log2((double)m);
        f[1] = (float)log2((double)n);
        f[2] = (float)((double)s_cnt / ((double)S * (double)n));
        f[3] = (float)((hint > 0 ? min((double)hint, mn) : mn) / mn);
    }
}

// ------------------------------------------------------------------ launchers
int64_t mlp_param_count(int S) { return mlp_params(S); }

hipError_t launch_features(const gf2_batch_item *items, int count, const int32_t *r_hint,
                           float *feats, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel, dim3(count), dim3(256), 0, st, items, count, r_hint, feats);
    return hipGetLastError();
}
size_t mlp_lds_bytes(int S) { return mlp_lds_floats(S) * sizeof(float); }
int mlp_blocks(int64_t N) { return (int)((N + MLP_BS - 1) / MLP_BS); }

static hipError_t mlp_set_lds(const void *k) {
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)mlp_lds_bytes(GF2_MLP_MAX_S));
}

hipError_t mlp_prepare() {
    hipError_t e;
    if ((e = mlp_set_lds((const void *)mlp_forward_kernel)) != hipSuccess) return e;
    if ((e = mlp_set_lds((const void *)mlp_grad_kernel)) != hipSuccess) return e;
    return mlp_set_lds((const void *)costmodel_predict_kernel);
}

hipError_t launch_mlp_init(float *params, int S, uint64_t seed, hipStream_t st) {
    hipLaunchKernelGGL(mlp_init_kernel, dim3(64), dim3(256), 0, st, params, S, seed);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *params, int S, const float *feats, int N, float *out,
                              hipStream_t st) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(mlp_blocks(N)), dim3(MLP_THREADS),
                       mlp_lds_bytes(S), st, params, S, feats, N, out);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *params, int S, const float *feats, const float *target,
                           const float *mask, int N, float inv_count, float *part, float *grad,
                           hipStream_t st) {
    if (N <= 0) return hipSuccess;
    const int nblk = mlp_blocks(N);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(MLP_THREADS), mlp_lds_bytes(S), st,
                       params, S, feats, target, mask, N, inv_count, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t width = mlp_params(S) + 1;
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((unsigned)((width + 255) / 256)), dim3(256), 0, st,
                       part, nblk, width, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *params, const float *grad, float *m1, float *m2, int S, float lr,
                           float beta1, float beta2, float eps, int step, hipStream_t st) {
    const int64_t P = mlp_params(S);
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, params,
                       grad, m1, m2, P, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_costmodel_predict(const float *params, int S, const float *feats, int N,
                                    const gf2_sched *table, gf2_sched *out, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(costmodel_predict_kernel, dim3(mlp_blocks(N)), dim3(MLP_THREADS),
                       mlp_lds_bytes(S), st, params, S, feats, N, table, out);
    return hipGetLastError();
}

}  // namespace gf2

// C-ABI of the learned cost model (kernels in k_mlp.hip).
#include <hip/hip_runtime.h>

#include "../../include/gf2pls.h"
#include "gf2_internal.h"

namespace gf2 {
int64_t mlp_param_count(int S);
int mlp_blocks(int64_t N);
hipError_t launch_mlp_init(float *params, int S, uint64_t seed, hipStream_t st);
hipError_t launch_mlp_forward(const float *params, int S, const float *feats, int N, float *out,
                              hipStream_t st);
hipError_t launch_mlp_grad(const float *params, int S, const float *feats, const float *target,
                           const float *mask, int N, float inv_count, float *part, float *grad,
                           hipStream_t st);
hipError_t launch_mlp_adam(float *params, const float *grad, float *m1, float *m2, int S, float lr,
                           float beta1, float beta2, float eps, int step, hipStream_t st);
hipError_t launch_costmodel_predict(const float *params, int S, const float *feats, int N,
                                    const gf2_sched *table, gf2_sched *out, hipStream_t st);
hipError_t launch_features(const gf2_batch_item *items, int count, const int32_t *r_hint,
                           float *feats, hipStream_t st);
}  // namespace gf2

namespace {
bool net_ok(const gf2_mlp &net) { return net.params && net.S >= 1 && net.S <= GF2_MLP_MAX_S; }
bool n_ok(int64_t N) { return N >= 0 && N <= ((int64_t)1 << 28); }
int hip_rc(hipError_t e) { return e == hipSuccess ? GF2_OK : GF2_E_HIP; }
}  // namespace

extern "C" {

int64_t gf2_mlp_param_count(int S) {
    if (S < 1 || S > GF2_MLP_MAX_S) return GF2_E_ARG;
    return gf2::mlp_param_count(S);
}

int gf2_mlp_init(gf2_ctx *ctx, gf2_mlp net, uint64_t seed, void *stream) {
    if (!ctx || !net_ok(net)) return GF2_E_ARG;
    return hip_rc(gf2::launch_mlp_init(net.params, net.S, seed, (hipStream_t)stream));
}

int gf2_mlp_forward(gf2_ctx *ctx, gf2_mlp net, const float *feats, int64_t N, float *out,
                    void *stream) {
    if (!ctx || !net_ok(net) || !n_ok(N) || (N > 0 && (!feats || !out))) return GF2_E_ARG;
    return hip_rc(gf2::launch_mlp_forward(net.params, net.S, feats, (int)N, out,
                                          (hipStream_t)stream));
}

size_t gf2_mlp_grad_workspace_bytes(int S, int64_t N) {
    if (S < 1 || S > GF2_MLP_MAX_S || !n_ok(N)) return 0;
    return (size_t)gf2::mlp_blocks(N > 0 ? N : 1) * (size_t)(gf2::mlp_param_count(S) + 1) * 4;
}

int gf2_mlp_grad(gf2_ctx *ctx, gf2_mlp net, const float *feats, const float *target,
                 const float *mask, int64_t N, float inv_count, float *grad, void *ws,
                 size_t ws_bytes, void *stream) {
    if (!ctx || !net_ok(net) || !n_ok(N) || N == 0 || !feats || !target || !mask || !grad)
        return GF2_E_ARG;
    if (!ws || ws_bytes < gf2_mlp_grad_workspace_bytes(net.S, N)) return GF2_E_WORKSPACE;
    return hip_rc(gf2::launch_mlp_grad(net.params, net.S, feats, target, mask, (int)N, inv_count,
                                       (float *)ws, grad, (hipStream_t)stream));
}

int gf2_mlp_adam(gf2_ctx *ctx, gf2_mlp net, const float *grad, float *m1, float *m2, float lr,
                 float beta1, float beta2, float eps, int step, void *stream) {
    if (!ctx || !net_ok(net) || !grad || !m1 || !m2 || step < 1) return GF2_E_ARG;
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f)) return GF2_E_ARG;
    return hip_rc(gf2::launch_mlp_adam(net.params, grad, m1, m2, net.S, lr, beta1, beta2, eps, step,
                                       (hipStream_t)stream));
}

int gf2_costmodel_predict(gf2_ctx *ctx, gf2_mlp net, const float *feats, int64_t N,
                          const gf2_sched *table, gf2_sched *out, void *stream) {
    if (!ctx || !net_ok(net) || !n_ok(N) || (N > 0 && (!feats || !table || !out))) return GF2_E_ARG;
    return hip_rc(gf2::launch_costmodel_predict(net.params, net.S, feats, (int)N, table, out,
                                                (hipStream_t)stream));
}

int gf2_features(gf2_ctx *ctx, const gf2_batch_item *items, int64_t count, const int32_t *r_hint,
                 float *feats, void *stream) {
    if (!ctx || count < 0 || count > ((int64_t)1 << 30)) return GF2_E_ARG;
    if (count == 0) return GF2_OK;
    if (!items || !feats) return GF2_E_ARG;
    if (((uintptr_t)items & 7) != 0 || ((uintptr_t)feats & 3) != 0) return GF2_E_ALIGN;
    return hip_rc(gf2::launch_features(items, (int)count, r_hint, feats, (hipStream_t)stream));
}

}  // extern "C"

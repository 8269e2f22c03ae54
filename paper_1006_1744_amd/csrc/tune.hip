// Autotuner: candidate schedules for a problem shape and their measured times.
// A schedule (strip width k, tables per pass, recursion cutoff, Schur variant)
// never changes a result bit, only the time, so the tuner simply runs every
// candidate on a trial problem, restoring the input from a pristine copy
// before each run, and keeps the fastest.  The fixed default schedule is the
// answer when there is nothing to time.  Timing uses HIP events on the call's
// stream and waits for them, so a tuning call is not graph-capturable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/gf2pls.h"
#include "gf2_internal.h"

namespace {

constexpr int kCutoffs[] = {256, 512, 1024, 2048, 4096};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    bool init() { return hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess; }
};

bool same_shape(const gf2_mat &x, const gf2_mat &y) { return x.m == y.m && x.n == y.n; }

}  // namespace

extern "C" {

int gf2_sched_candidates(int64_t m, int64_t n, int batched, gf2_sched *out, int max) {
    (void)m;
    if (n < 0 || max < 0 || (max > 0 && !out)) return GF2_E_ARG;
    gf2_sched d;
    gf2_default_sched(&d);
    const int64_t ncols = 64 * ((n + 63) / 64);
    std::vector<gf2_sched> c;
    for (int k = 4; k <= 8; k++)
        for (int t : {1, 2, 4, 8}) {
            if (batched) {
                c.push_back({k, t, d.cutoff, d.schur});
                continue;
            }
            bool mmpf = false;
            for (int cut : kCutoffs) {
                if (cut >= ncols) {   // the whole width is one MMPF block: no Schur products
                    if (!mmpf) c.push_back({k, t, cut, d.schur});
                    mmpf = true;
                    continue;
                }
                c.push_back({k, t, cut, GF2_SCHUR_XOR});
                c.push_back({k, t, cut, GF2_SCHUR_MFMA});
                c.push_back({k, t, cut, GF2_SCHUR_FP4});
            }
        }
    const int cnt = (int)c.size();
    for (int i = 0; i < std::min(cnt, max); i++) out[i] = c[i];
    return cnt;
}

size_t gf2_autotune_workspace_bytes(int64_t m, int64_t n, const gf2_sched *cands, int ncand) {
    if (m < 0 || n < 0 || ncand < 0 || (ncand > 0 && !cands)) return 0;
    size_t ws = 0;
    for (int i = 0; i < ncand; i++) ws = std::max(ws, gf2_pls_workspace_bytes(m, n, &cands[i]));
    return align256(ws) + align256((size_t)std::max<int64_t>(m, 1) * 4) +
           align256((size_t)std::max<int64_t>(n, 1) * 4) + 256;
}

int gf2_autotune(gf2_ctx *ctx, gf2_mat A_trial, gf2_mat A_work, const gf2_sched *cands, int ncand,
                 int reps, float *ms_out, gf2_sched *best, void *ws, size_t ws_bytes,
                 void *stream) {
    if (!ctx || !best || ncand < 0 || reps < 1 || (ncand > 0 && (!cands || !ms_out)))
        return GF2_E_ARG;
    if (!same_shape(A_trial, A_work) || A_trial.words == A_work.words) return GF2_E_ARG;
    gf2_default_sched(best);
    if (ncand == 0) return GF2_OK;
    for (int i = 0; i < ncand; i++)
        if (!gf2_sched_valid(&cands[i])) return GF2_E_ARG;
    const size_t need = gf2_autotune_workspace_bytes(A_trial.m, A_trial.n, cands, ncand);
    if (!ws || ws_bytes < need) return GF2_E_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return GF2_E_ALIGN;
    size_t pls_ws = 0;
    for (int i = 0; i < ncand; i++)
        pls_ws = std::max(pls_ws, gf2_pls_workspace_bytes(A_trial.m, A_trial.n, &cands[i]));
    char *base = (char *)ws;
    int32_t *P = (int32_t *)(base + align256(pls_ws));
    int32_t *Q = (int32_t *)((char *)P + align256((size_t)std::max<int64_t>(A_trial.m, 1) * 4));
    int32_t *rank = (int32_t *)((char *)Q + align256((size_t)std::max<int64_t>(A_trial.n, 1) * 4));
    hipStream_t st = (hipStream_t)stream;
    EventPair ev;
    if (!ev.init()) return GF2_E_HIP;
    const int64_t nw = (A_trial.n + 63) / 64;
    float best_ms = 0.f;
    for (int i = 0; i < ncand; i++) {
        float tmin = 0.f;
        for (int r = 0; r < reps; r++) {
            if (gf2::launch_copy_words(A_work.words, A_work.stride, A_trial.words, A_trial.stride,
                                       A_trial.m, nw, st) != hipSuccess)
                return GF2_E_HIP;
            if (hipEventRecord(ev.a, st) != hipSuccess) return GF2_E_HIP;
            const int rc = gf2_pls(ctx, A_work, P, Q, rank, &cands[i], ws, pls_ws, stream);
            if (rc != GF2_OK) return rc;
            if (hipEventRecord(ev.b, st) != hipSuccess) return GF2_E_HIP;
            if (hipEventSynchronize(ev.b) != hipSuccess) return GF2_E_HIP;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess) return GF2_E_HIP;
            tmin = r == 0 ? ms : std::min(tmin, ms);
        }
        ms_out[i] = tmin;
        if (i == 0 || tmin < best_ms) {
            best_ms = tmin;
            *best = cands[i];
        }
    }
    return GF2_OK;
}

int gf2_autotune_batched(gf2_ctx *ctx, const gf2_batch_item *trial, const gf2_batch_item *work,
                         int64_t count, int32_t *ranks, const gf2_sched *cands, int ncand, int reps,
                         float *ms_out, gf2_sched *best, void *ws, size_t ws_bytes, void *stream) {
    if (!ctx || !best || ncand < 0 || reps < 1 || count < 0 || (ncand > 0 && (!cands || !ms_out)))
        return GF2_E_ARG;
    gf2_default_sched(best);
    if (ncand == 0 || count == 0) return GF2_OK;
    if (!trial || !work || !ranks || trial == work) return GF2_E_ARG;
    for (int i = 0; i < ncand; i++)
        if (!gf2_sched_valid(&cands[i])) return GF2_E_ARG;
    if (!ws || ws_bytes < gf2_pls_batched_workspace_bytes(count)) return GF2_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    EventPair ev;
    if (!ev.init()) return GF2_E_HIP;
    float best_ms = 0.f;
    for (int i = 0; i < ncand; i++) {
        float tmin = 0.f;
        for (int r = 0; r < reps; r++) {
            if (gf2::launch_batch_copy(trial, work, (int)count, st) != hipSuccess) return GF2_E_HIP;
            if (hipEventRecord(ev.a, st) != hipSuccess) return GF2_E_HIP;
            const int rc = gf2_pls_batched(ctx, work, count, ranks, nullptr, &cands[i], ws,
                                           ws_bytes, stream);
            if (rc != GF2_OK) return rc;
            if (hipEventRecord(ev.b, st) != hipSuccess) return GF2_E_HIP;
            if (hipEventSynchronize(ev.b) != hipSuccess) return GF2_E_HIP;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess) return GF2_E_HIP;
            tmin = r == 0 ? ms : std::min(tmin, ms);
        }
        ms_out[i] = tmin;
        if (i == 0 || tmin < best_ms) {
            best_ms = tmin;
            *best = cands[i];
        }
    }
    return GF2_OK;
}

}  // extern "C"

// C-ABI entry points of libgf2pls and the host-side driver of the recursion.
//
// gf2_pls follows the asymptotically fast PLS of Section 5: columns are split at
// word boundaries (Section 6: cuts along word boundaries), the left half is
// decomposed, the right half receives the row swaps (done eagerly inside the
// panel kernels), the triangular solve A_NE <- L_NW^{-1} A_NE and the Schur
// update A_SE <- A_SE + A_SW A_NE, then the right half is decomposed and the L
// columns are compressed.  Column blocks of at most `cutoff` columns use the
// MMPF base case of Section 4.1, with 64-column panels (PlsSubmatrix re-planned
// for one wave) followed by table-driven updates (MakeTable1 /
// AddRowsFromTable).  All launches go to one stream; data-dependent extents
// are read on the device, so the host never waits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/gf2pls.h"
#include "gf2_internal.h"

// Optional per-launch timing of the product kernels: events recorded on the
// launch stream around each launch, the kernel storing its dynamic M, K and N in
// a caller-provided device log.
struct ProfRec {
    hipEvent_t a, b;
    int slot;
};

// ints per launch in the device log: M, K and the column count N
constexpr int kProfInts = 3;

struct gf2_ctx {
    int device;
    int cus;
    int batch_bpc = 1;   // resident blocks per CU of the batched kernel
    int32_t *plog = nullptr;
    int64_t plog_cap = 0;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
    void *scratch = nullptr;   // this device's copy of `scratch` (device address)
    // learned schedule choice for calls without a schedule: one schedule per
    // cell of a half-log2 grid of (m, n) over [l_lo, l_hi]^2, row-major by m
    std::vector<gf2_sched> learned;
    float l_lo = 0.f, l_hi = -1.f, l_mn_hi = -1.f;
    int l_cells = 0;
};

// Scratch memory of gf2_pls_noalloc: one copy per device, held until the process
// ends.  Its name is a host-side stand-in; kernels only ever receive the device
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[GF2_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (current), looked up once per device.
hipError_t scratch_address(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

namespace gf2 {
int table_update_tile_words(int k, int tables);
}

using namespace gf2;

namespace {

constexpr int64_t kMaxDim = (int64_t)1 << 30;
constexpr int kMfmaMaxK = 65536;   // sums of 0/1 products: exact in int32 and in fp32 (< 2^24)
constexpr int kINF = 0x3fffffff;
constexpr int kBufWords = 16;       // widest base block worked on in a contiguous copy

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

bool sched_ok(const gf2_sched *s) {
    if (!s) return false;
    if (s->k < 4 || s->k > 8) return false;
    if (s->tables != 1 && s->tables != 2 && s->tables != 4 && s->tables != 8) return false;
    if (s->cutoff < 64 || (s->cutoff % 64) != 0) return false;
    if (s->schur != GF2_SCHUR_XOR && s->schur != GF2_SCHUR_MFMA && s->schur != GF2_SCHUR_FP4)
        return false;
    return true;
}

gf2_sched default_sched() {
    gf2_sched s;
    s.k = 8;
    s.tables = 8;
    s.cutoff = 2048;
    s.schur = GF2_SCHUR_FP4;
    return s;
}

// C rows `crows` (of C, default end m), words [cw, cw + nw) += A (same rows, K
// bits from word aw) * B (rows `brows` of Bsrc, default end kmrows, words
// [cw, cw + nw) of Bsrc), K <= kmax, split into chunks the MFMA sums keep exact.
hipEvent_t pool_event(gf2_ctx *ctx, size_t idx) {
    while (ctx->pool.size() <= idx) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ctx->pool.push_back(e);
    }
    return ctx->pool[idx];
}

// pre_transposed: Bt already holds B transposed (kmax <= kMfmaMaxK, row stride
// (kmax + 63) / 64 words, rows past K zero), so no transpose is launched.
// nwd (nullable, device): dynamic number of C words, at most nw.
hipError_t enqueue_gemm(gf2_ctx *ctx, uint64_t *C, int64_t sc, const uint64_t *Am, int64_t sa,
                        const uint64_t *Bsrc, int64_t sb, int m, int kmrows, RowRange crows,
                        int aw, int cw, int nw, RowRange brows, int kmax, int schur,
                        const int32_t *rk, uint64_t *Bt, hipStream_t st,
                        bool pre_transposed = false, const int32_t *nwd = nullptr) {
    if (pre_transposed && kmax > kMfmaMaxK) return hipErrorInvalidValue;
    for (int k0 = 0; k0 < kmax; k0 += kMfmaMaxK) {
        const int kc = std::min(kMfmaMaxK, kmax - k0);
        RowRange br = brows;
        br.a += k0;
        br.s = std::min(br.s - k0, kc);
        const int64_t sbt = (kc + 63) / 64;
        hipError_t e = hipSuccess;
        if (!pre_transposed)
            e = launch_transpose(Bsrc, sb, kmrows, br, cw, nw, kc, Bt, sbt, rk, st, nwd);
        if (e != hipSuccess) return e;
        int32_t *plog = nullptr;
        ProfRec rec{};
        const bool prof = ctx && ctx->plog && (int64_t)ctx->recs.size() < ctx->plog_cap;
        if (prof) {
            rec.slot = (int)ctx->recs.size();
            rec.a = pool_event(ctx, 2 * (size_t)rec.slot);
            rec.b = pool_event(ctx, 2 * (size_t)rec.slot + 1);
            if (!rec.a || !rec.b) return hipErrorOutOfMemory;
            plog = ctx->plog + kProfInts * rec.slot;
            if ((e = hipEventRecord(rec.a, st)) != hipSuccess) return e;
        }
        if (schur == GF2_SCHUR_MFMA || schur == GF2_SCHUR_FP4)
            e = launch_gemm_mfma(C, sc, Am, sa, m, crows, aw + k0 / 64, cw, nw, Bt, sbt, kc, br,
                                 kmrows, rk, plog, schur == GF2_SCHUR_FP4, st, nwd);
        else
            e = launch_gemm_xor(C, sc, Am, sa, m, crows, aw + k0 / 64, cw, nw, Bt, sbt, kc, br,
                                kmrows, rk, plog, st, nwd);
        if (e != hipSuccess) return e;
        if (prof) {
            if ((e = hipEventRecord(rec.b, st)) != hipSuccess) return e;
            ctx->recs.push_back(rec);
        }
    }
    return hipSuccess;
}

size_t gemm_bt_words(int nw, int kmax) {
    const int kc = std::min(kMfmaMaxK, kmax);
    return (size_t)nw * 64 * ((kc + 63) / 64);
}

#define GF2_TRY(x)                                   \
    do {                                             \
        hipError_t e_ = (x);                         \
        if (e_ != hipSuccess) return GF2_E_HIP;      \
    } while (0)

// The recursion, run either to size the workspace (dry) or to launch.
struct PlsDriver {
    bool dry = true;
    gf2_ctx *ctx = nullptr;
    uint64_t *A = nullptr;
    int64_t stride = 0;
    int m = 0, n = 0, nb = 0;
    gf2_sched s{};
    int32_t *rk = nullptr, *P = nullptr, *Q = nullptr, *info = nullptr;
    const uint64_t *linv = nullptr;   // L^{-1} rows inside the panel record
    uint64_t *Bt = nullptr;           // a node's Schur operand, written transposed by its TRSM
    uint64_t *Bt2 = nullptr;          // transposed operands of the products inside a TRSM
    int64_t bt_sbt = 0;               // row stride of Bt for the node being solved
    bool bt_fused = false;            // the node's TRSM writes Bt (else the product transposes)
    uint64_t *Bbuf = nullptr;         // staged pivot rows, 64 x bstride words
    uint64_t *linv_store = nullptr;   // per panel: L^{-1} of its pivot block (64 words)
    uint64_t *pbuf = nullptr;         // base block copy: m rows x pbuf_w words, contiguous
    int pbuf_w = 0;
    int64_t bstride = 0;
    int cus = 256;
    size_t bt_words = 0;   // capacity (launch) or requirement (dry)
    size_t bt2_words = 0;
    hipStream_t st = nullptr;
    hipError_t err = hipSuccess;

    void chk(hipError_t e) {
        if (err == hipSuccess && e != hipSuccess) err = e;
    }

    // C rows `crows`, C words [cw, cw + nw) += A (rows = crows, K bits from word aw)
    // times B (rows `brows`, same words as C), K <= kmax.  Inside a TRSM: B is
    // transposed into Bt2 first.
    void gemm(RowRange crows, int aw, int cw, int nw, RowRange brows, int kmax) {
        if (nw <= 0 || kmax <= 0) return;
        if (dry) {
            bt2_words = std::max(bt2_words, gemm_bt_words(nw, kmax));
            return;
        }
        chk(enqueue_gemm(ctx, A, stride, A, stride, A, stride, m, m, crows, aw, cw, nw, brows,
                         kmax, s.schur, rk, Bt2, st));
    }

    // A node's Schur product: when bt_fused, B was written transposed into Bt by
    // the TRSM that produced it (row stride bt_sbt = kmax / 64 words).
    void gemm_schur(RowRange crows, int aw, int cw, int nw, RowRange brows, int kmax) {
        if (nw <= 0 || kmax <= 0) return;
        if (dry) {
            bt_words = std::max(bt_words, gemm_bt_words(nw, kmax));
            return;
        }
        chk(enqueue_gemm(ctx, A, stride, A, stride, A, stride, m, m, crows, aw, cw, nw, brows,
                         kmax, s.schur, rk, Bt, st, bt_fused));
    }

    // rows [rk[ib] + a, min(rk[ie], rk[ib] + a + sz)) <- L^{-1} rows, L's block
    // starting at word lw0 + a / 64; right-hand side words [w_lo, w_hi).  The
    // solved rows also go to Bt, transposed, at K word a / 64 (row stride bt_sbt).
    void trsm_lower(int ib, int ie, int a, int sz, int lw0, int w_lo, int w_hi) {
        if (w_hi <= w_lo || sz <= 0) return;
        if (sz <= trsm_block_max_rows()) {
            if (!dry)
                chk(launch_trsm_block(A, stride, A, stride, m, row_range(ib, ie, a, sz),
                                      lw0 + a / 64, w_lo, w_hi, rk, 1, (sz + 63) / 64, linv_store,
                                      bt_fused ? Bt : nullptr, bt_sbt, a / 64, st));
            return;
        }
        const int h = (sz / 64 / 2) * 64;
        trsm_lower(ib, ie, a, h, lw0, w_lo, w_hi);
        gemm(row_range(ib, ie, a + h, sz - h), lw0 + a / 64, w_lo, w_hi - w_lo,
             row_range(ib, ie, a, h), h);
        trsm_lower(ib, ie, a + h, sz - h, lw0, w_lo, w_hi);
    }

    // MMPF base case on word columns [wb, wb + nwd): 64-column panels, each
    // followed by the table-driven solve of its pivot rows and update of the
    // rows below, on the block's remaining columns.
    void base(int wb, int nwd) {
        if (dry) bstride = std::max<int64_t>(bstride, nwd - 1);
        // a narrow block works on a contiguous copy of its words (rows of nwd words),
        // so the passes over the rows below a panel read whole segments in order
        const bool buffered = pbuf_w > 0 && nwd <= pbuf_w && nwd > 1;
        uint64_t *Ab = buffered ? pbuf - wb : A;
        const int64_t sb = buffered ? nwd : stride;
        const int blk_lo = buffered ? wb : 0, blk_hi = buffered ? wb + nwd : (int)stride;
        if (buffered && !dry) chk(launch_copy_rows(pbuf, nwd, 0, A, stride, wb, nwd, rk, wb, m, st));
        // search(0), then per panel: its post pass, and the update of the block's
        // remaining words fused with the next panel's search
        if (!dry) chk(launch_leaf_search(Ab, sb, m, n, wb, rk, wb, P, Q, info, st));
        for (int p = 0; p < nwd; p++) {
            const int wc = wb + p;
            const bool upd = p + 1 < nwd;
            if (dry) continue;
            chk(launch_panel_post(A, stride, Ab, sb, blk_lo, blk_hi, m, n, wc, rk, wc, info,
                                  upd ? Bbuf : nullptr, bstride, wc + 1, wb + nwd, linv_store,
                                  p > 0, st));
            if (upd)
                chk(launch_table_update_search(Ab, sb, m, n, wc, rk, wc, wc + 1, wb + nwd, s.k,
                                               s.tables, linv, Bbuf, bstride, P, Q, info, cus, st));
        }
        if (!dry) {
            if (buffered)
                chk(launch_compress_chain_out(A, stride, pbuf, m, wb, nwd, rk, st));
            else
                chk(launch_compress_chain(Ab, sb, m, wb, nwd, rk, stride, st));
        }
    }

    void node(int wb, int nwd) {
        if (nwd <= 0) return;
        if (nwd == 1 || (int64_t)nwd * 64 <= s.cutoff) {
            base(wb, nwd);
            return;
        }
        const int h = nwd / 2;
        node(wb, h);
        // A_NE <- L_NW^{-1} A_NE on the first half's pivot rows, also written
        // transposed into Bt for the Schur product when the solve runs one word
        // per block (below 512 words); wider ones leave it to the tiled transpose,
        // cheaper than the scattered writes at the end of every solve block there
        bt_sbt = h;
        bt_fused = nwd - h < 512;
        trsm_lower(wb, wb + h, 0, 64 * h, wb, wb + h, wb + nwd);
        // A_SE <- A_SE + A_SW A_NE
        gemm_schur(row_range(wb + h, -1, 0, kINF), wb, wb + h, nwd - h,
                   row_range(wb, wb + h, 0, 64 * h), 64 * h);
        node(wb + h, nwd - h);
        if (!dry)
            chk(launch_compress_shift(A, stride, m, 64 * wb, 64 * h, rk, wb, wb + h, wb + nwd, st));
    }

    void run() {
        if (!dry) chk(launch_fill_i32(rk, 0, nb + 1, st));
        node(0, nb);
    }
};

struct PlsLayout {
    size_t rk_off, info_off, bt_off, bt2_off, bb_off, linv_off, pbuf_off, total;
    int pbuf_w;
    size_t bt_words, bt2_words;
    int64_t bstride;
};

PlsLayout pls_layout(int64_t m, int64_t n, const gf2_sched &s) {
    PlsDriver d;
    d.dry = true;
    d.m = (int)m;
    d.n = (int)n;
    d.nb = (int)((n + 63) / 64);
    d.s = s;
    d.run();
    PlsLayout L;
    size_t off = 0;
    L.rk_off = off;
    off = align_up(off + (size_t)(d.nb + 2) * 4);
    L.info_off = off;
    off = align_up(off + panel_info_bytes());
    L.bt_off = off;
    L.bt_words = d.bt_words;
    off = align_up(off + d.bt_words * 8);
    L.bt2_off = off;
    L.bt2_words = d.bt2_words;
    off = align_up(off + d.bt2_words * 8);
    L.bb_off = off;
    L.bstride = std::max<int64_t>(d.bstride, 1);
    off = align_up(off + (size_t)64 * L.bstride * 8);
    L.linv_off = off;
    off = align_up(off + (size_t)(d.nb + 1) * 64 * 8);
    L.pbuf_w = std::min(std::min(s.cutoff / 64, kBufWords), d.nb);
    L.pbuf_off = off;
    off = align_up(off + (size_t)std::max<int64_t>(m, 1) * std::max(L.pbuf_w, 1) * 8);
    L.total = off;
    return L;
}

int check_mat(const gf2_mat &A) {
    if (A.m < 0 || A.n < 0 || A.m > kMaxDim || A.n > kMaxDim) return GF2_E_UNSUPPORTED;
    if (A.stride < (A.n + 63) / 64) return GF2_E_ALIGN;
    if ((A.m > 0 && A.n > 0) && !A.words) return GF2_E_ARG;
    if (((uintptr_t)A.words & 7) != 0) return GF2_E_ALIGN;
    if (A.stride > ((int64_t)1 << 40) / std::max<int64_t>(A.m, 1)) return GF2_E_UNSUPPORTED;
    return GF2_OK;
}

// The schedule of a call without one: the learned cell of (m, n) when the
// context holds a learned choice covering it, else the default.
gf2_sched choose_sched(const gf2_ctx *ctx, int64_t m, int64_t n, bool *learned = nullptr) {
    if (learned) *learned = false;
    if (!ctx || ctx->l_cells <= 0 || m <= 0 || n <= 0) return default_sched();
    const double lm = std::log2((double)m), ln = std::log2((double)n);
    if (lm < ctx->l_lo - 0.25 || lm > ctx->l_hi + 0.25 || ln < ctx->l_lo - 0.25 ||
        ln > ctx->l_hi + 0.25 || lm + ln > ctx->l_mn_hi + 0.25)
        return default_sched();
    const int im = std::min(ctx->l_cells - 1, std::max(0, (int)std::lround((lm - ctx->l_lo) * 2.0)));
    const int in = std::min(ctx->l_cells - 1, std::max(0, (int)std::lround((ln - ctx->l_lo) * 2.0)));
    const gf2_sched c = ctx->learned[(size_t)im * ctx->l_cells + in];
    if (!sched_ok(&c)) return default_sched();
    if (learned) *learned = true;
    return c;
}

// Launches the recursion for A with its workspace at `base` (layout L).
int pls_run(gf2_ctx *ctx, const gf2_mat &A, int32_t *P, int32_t *Q, int32_t *rank,
            const gf2_sched &ss, const PlsLayout &L, char *base, hipStream_t st) {
    if (hipSetDevice(ctx->device) != hipSuccess) return GF2_E_HIP;
    PlsDriver d;
    d.dry = false;
    d.ctx = ctx;
    d.A = A.words;
    d.stride = A.stride;
    d.m = (int)A.m;
    d.n = (int)A.n;
    d.nb = (int)((A.n + 63) / 64);
    d.s = ss;
    d.rk = (int32_t *)(base + L.rk_off);
    d.info = (int32_t *)(base + L.info_off);
    d.Bt = (uint64_t *)(base + L.bt_off);
    d.bt_words = L.bt_words;
    d.Bt2 = (uint64_t *)(base + L.bt2_off);
    d.bt2_words = L.bt2_words;
    d.Bbuf = (uint64_t *)(base + L.bb_off);
    d.bstride = L.bstride;
    d.linv = (const uint64_t *)(base + L.info_off + panel_info_linv_offset());
    d.linv_store = (uint64_t *)(base + L.linv_off);
    d.pbuf = (uint64_t *)(base + L.pbuf_off);
    d.pbuf_w = L.pbuf_w;
    d.cus = ctx->cus;
    d.P = P;
    d.Q = Q;
    d.st = st;
    if (A.m > 0 && A.n > 0) d.run();
    else d.chk(launch_fill_i32(d.rk, 0, d.nb + 1, st));
    d.chk(launch_finalize(P, Q, rank, d.rk, d.nb, d.m, d.n, st));
    return d.err == hipSuccess ? GF2_OK : GF2_E_HIP;
}

}  // namespace

extern "C" {

int gf2_ctx_create(gf2_ctx **out, int device) {
    if (!out) return GF2_E_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return GF2_E_HIP;
    if (device < 0 || device >= count) return GF2_E_ARG;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return GF2_E_HIP;
    if (hipSetDevice(device) != hipSuccess) return GF2_E_HIP;
    gf2_ctx *c = new gf2_ctx;
    c->device = device;
    c->cus = prop.multiProcessorCount;
    c->batch_bpc = batch_blocks_per_cu();
    if (scratch_address(device, &c->scratch) != hipSuccess) {
        delete c;
        return GF2_E_HIP;
    }
    if (mlp_prepare() != hipSuccess) {
        delete c;
        return GF2_E_HIP;
    }
    *out = c;
    return GF2_OK;
}

void gf2_ctx_destroy(gf2_ctx *ctx) {
    if (!ctx) return;
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    delete ctx;
}

int gf2_prof_enable(gf2_ctx *ctx, int32_t *dev_log, int64_t log_slots) {
    if (!ctx) return GF2_E_ARG;
    if (dev_log && log_slots <= 0) return GF2_E_ARG;
    ctx->plog = dev_log;
    ctx->plog_cap = dev_log ? log_slots : 0;
    ctx->recs.clear();
    return GF2_OK;
}

int gf2_prof_read_launches(gf2_ctx *ctx, gf2_prof_launch *out, int64_t max, int64_t *count) {
    if (!ctx || !count || (max > 0 && !out)) return GF2_E_ARG;
    *count = 0;
    if (ctx->recs.empty()) return GF2_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return GF2_E_HIP;
    if (hipEventSynchronize(ctx->recs.back().b) != hipSuccess) return GF2_E_HIP;
    std::vector<int32_t> log(kProfInts * ctx->recs.size());
    if (hipMemcpy(log.data(), ctx->plog, log.size() * sizeof(int32_t), hipMemcpyDeviceToHost) !=
        hipSuccess)
        return GF2_E_HIP;
    int64_t k = 0;
    for (const ProfRec &r : ctx->recs) {
        if (k >= max) break;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return GF2_E_HIP;
        out[k].ms = ms;
        out[k].m = log[kProfInts * r.slot];
        out[k].k = log[kProfInts * r.slot + 1];
        out[k].n = log[kProfInts * r.slot + 2];
        k++;
    }
    *count = k;
    return GF2_OK;
}

int gf2_prof_read(gf2_ctx *ctx, gf2_prof_stats *out) {
    if (!ctx || !out) return GF2_E_ARG;
    out->launches = 0;
    out->total_ms = 0.0;
    out->total_ops = 0.0;
    if (ctx->recs.empty()) return GF2_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return GF2_E_HIP;
    if (hipEventSynchronize(ctx->recs.back().b) != hipSuccess) return GF2_E_HIP;
    std::vector<int32_t> log(kProfInts * ctx->recs.size());
    if (hipMemcpy(log.data(), ctx->plog, log.size() * sizeof(int32_t), hipMemcpyDeviceToHost) !=
        hipSuccess)
        return GF2_E_HIP;
    for (const ProfRec &r : ctx->recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess) return GF2_E_HIP;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return GF2_E_HIP;
        out->launches += 1;
        out->total_ms += ms;
        out->total_ops += 2.0 * (double)log[kProfInts * r.slot] *
                          (double)log[kProfInts * r.slot + 2] * (double)log[kProfInts * r.slot + 1];
    }
    ctx->recs.clear();
    return GF2_OK;
}

const char *gf2_status_str(int status) {
    switch (status) {
        case GF2_OK: return "ok";
        case GF2_E_ARG: return "invalid argument";
        case GF2_E_ALIGN: return "stride or alignment";
        case GF2_E_WORKSPACE: return "workspace too small";
        case GF2_E_HIP: return "HIP runtime error";
        case GF2_E_UNSUPPORTED: return "unsupported size";
        default: return "unknown status";
    }
}

void gf2_default_sched(gf2_sched *out) {
    if (out) *out = default_sched();
}

int gf2_sched_valid(const gf2_sched *s) { return sched_ok(s) ? 1 : 0; }

size_t gf2_pls_workspace_bytes(int64_t m, int64_t n, const gf2_sched *s) {
    if (m < 0 || n < 0 || m > kMaxDim || n > kMaxDim) return 0;
    if (s) {
        if (!sched_ok(s)) return 0;
        return pls_layout(m, n, *s).total;
    }
    // no schedule: enough for any a context may choose (the cutoff alone sets
    // the layout; k, tables and the product variant do not)
    size_t need = pls_layout(m, n, default_sched()).total;
    for (int c = 256; c <= 4096; c *= 2) {
        gf2_sched t = default_sched();
        t.cutoff = c;
        need = std::max(need, pls_layout(m, n, t).total);
    }
    return need;
}

int gf2_pls(gf2_ctx *ctx, gf2_mat A, int32_t *P, int32_t *Q, int32_t *rank, const gf2_sched *s,
            void *ws, size_t ws_bytes, void *stream) {
    if (!ctx) return GF2_E_ARG;
    int rc = check_mat(A);
    if (rc != GF2_OK) return rc;
    gf2_sched ss = s ? *s : choose_sched(ctx, A.m, A.n);
    if (!sched_ok(&ss)) return GF2_E_ARG;
    if (!rank || (A.m > 0 && !P) || (A.n > 0 && !Q)) return GF2_E_ARG;
    PlsLayout L = pls_layout(A.m, A.n, ss);
    if (!ws || ws_bytes < L.total) return GF2_E_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return GF2_E_ALIGN;
    return pls_run(ctx, A, P, Q, rank, ss, L, (char *)ws, (hipStream_t)stream);
}

int gf2_pls_noalloc(gf2_ctx *ctx, gf2_mat A, int32_t *P, int32_t *Q, int32_t *rank,
                    const gf2_sched *s, void *stream) {
    if (!ctx) return GF2_E_ARG;
    int rc = check_mat(A);
    if (rc != GF2_OK) return rc;
    gf2_sched ss = s ? *s : choose_sched(ctx, A.m, A.n);
    if (!sched_ok(&ss)) return GF2_E_ARG;
    if (!rank || (A.m > 0 && !P) || (A.n > 0 && !Q)) return GF2_E_ARG;
    PlsLayout L = pls_layout(A.m, A.n, ss);
    if (L.total > (size_t)GF2_NOALLOC_SCRATCH_BYTES) return GF2_E_UNSUPPORTED;
    if (!ctx->scratch) return GF2_E_HIP;
    return pls_run(ctx, A, P, Q, rank, ss, L, (char *)ctx->scratch, (hipStream_t)stream);
}

size_t gf2_pls_noalloc_max_bytes(void) { return (size_t)GF2_NOALLOC_SCRATCH_BYTES; }

size_t gf2_ctx_set_learned_workspace_bytes(void) {
    const size_t cells = (size_t)GF2_LEARNED_MAX_CELLS * GF2_LEARNED_MAX_CELLS;
    return align_up(cells * 4 * sizeof(float)) + align_up(cells * sizeof(gf2_sched));
}

int gf2_ctx_set_learned(gf2_ctx *ctx, gf2_mlp net, const gf2_sched *table, float log2_lo,
                        float log2_hi, float log2_mn_hi, void *ws, size_t ws_bytes,
                        void *stream) {
    if (!ctx) return GF2_E_ARG;
    if (!net.params) {   // back to the default for every call without a schedule
        ctx->learned.clear();
        ctx->l_cells = 0;
        return GF2_OK;
    }
    if (net.S < 1 || net.S > GF2_MLP_MAX_S || !table) return GF2_E_ARG;
    if (!(log2_lo >= 0.f && log2_hi >= log2_lo && log2_hi <= 30.f)) return GF2_E_ARG;
    if (!(log2_mn_hi >= 2.f * log2_lo)) return GF2_E_ARG;
    const int cells = (int)std::lround((log2_hi - log2_lo) * 2.0f) + 1;
    if (cells > GF2_LEARNED_MAX_CELLS) return GF2_E_ARG;
    if (!ws || ws_bytes < gf2_ctx_set_learned_workspace_bytes()) return GF2_E_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return GF2_E_ALIGN;
    if (hipSetDevice(ctx->device) != hipSuccess) return GF2_E_HIP;
    const int N = cells * cells;
    std::vector<float> f((size_t)N * 4);
    for (int a = 0; a < cells; a++)
        for (int b = 0; b < cells; b++) {
            float *r = &f[((size_t)a * cells + b) * 4];
            r[0] = log2_lo + 0.5f * a;
            r[1] = log2_lo + 0.5f * b;
            r[2] = 0.5f;   // a dense input: the density of a call is not known up front
            r[3] = 1.0f;   // full rank assumed for the same reason
        }
    const size_t cells_max = (size_t)GF2_LEARNED_MAX_CELLS * GF2_LEARNED_MAX_CELLS;
    float *fd = (float *)ws;
    gf2_sched *od = (gf2_sched *)((char *)ws + align_up(cells_max * 4 * sizeof(float)));
    hipStream_t st = (hipStream_t)stream;
    std::vector<gf2_sched> out((size_t)N);
    GF2_TRY(hipMemcpyAsync(fd, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, st));
    GF2_TRY(launch_costmodel_predict(net.params, net.S, fd, N, table, od, st));
    GF2_TRY(hipMemcpyAsync(out.data(), od, out.size() * sizeof(gf2_sched), hipMemcpyDeviceToHost, st));
    GF2_TRY(hipStreamSynchronize(st));
    for (const gf2_sched &c : out)
        if (!sched_ok(&c)) return GF2_E_ARG;   // a table row that is not a schedule
    ctx->learned = std::move(out);
    ctx->l_lo = log2_lo;
    ctx->l_hi = log2_lo + 0.5f * (cells - 1);
    ctx->l_mn_hi = log2_mn_hi;
    ctx->l_cells = cells;
    return GF2_OK;
}

int gf2_ctx_learned_sched(gf2_ctx *ctx, int64_t m, int64_t n, gf2_sched *out) {
    if (!ctx || !out) return GF2_E_ARG;
    bool learned = false;
    *out = choose_sched(ctx, m, n, &learned);
    return learned ? 1 : 0;
}

int gf2_pls_unpack(gf2_ctx *ctx, gf2_mat A_pls, const int32_t *Q, const int32_t *rank,
                   gf2_mat L_out, gf2_mat S_out, void *stream) {
    if (!ctx || !Q || !rank) return GF2_E_ARG;
    int rc = check_mat(A_pls);
    if (rc != GF2_OK) return rc;
    const int64_t rmax = std::min(A_pls.m, A_pls.n);
    if (L_out.m != A_pls.m || L_out.n != rmax || S_out.m != rmax || S_out.n != A_pls.n)
        return GF2_E_ARG;
    if ((rc = check_mat(L_out)) != GF2_OK || (rc = check_mat(S_out)) != GF2_OK) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return GF2_E_HIP;
    const int lwords = (int)((rmax + 63) / 64), swords = (int)((A_pls.n + 63) / 64);
    const int64_t maxw = A_pls.m * lwords + rmax * swords;
    hipError_t e = launch_unpack(A_pls.words, A_pls.stride, (int)A_pls.m, (int)A_pls.n, Q, rank,
                                 L_out.words, L_out.stride, lwords, S_out.words, S_out.stride, swords,
                                 maxw, (hipStream_t)stream);
    return e == hipSuccess ? GF2_OK : GF2_E_HIP;
}

size_t gf2_pls_batched_workspace_bytes(int64_t count) {
    if (count < 0) return 0;
    return align_up(batch_ws_bytes(count));
}

int gf2_pls_batched(gf2_ctx *ctx, const gf2_batch_item *items, int64_t count, int32_t *ranks,
                    const gf2_sched *per_item, const gf2_sched *s, void *ws, size_t ws_bytes,
                    void *stream) {
    if (!ctx || count < 0 || count > (int64_t)1 << 30) return GF2_E_ARG;
    if (count == 0) return GF2_OK;
    if (!items || !ranks) return GF2_E_ARG;
    gf2_sched ss = s ? *s : default_sched();
    if (!sched_ok(&ss)) return GF2_E_ARG;
    if (!ws || ws_bytes < gf2_pls_batched_workspace_bytes(count)) return GF2_E_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0 || ((uintptr_t)items & 7) != 0 || ((uintptr_t)ranks & 3) != 0)
        return GF2_E_ALIGN;
    if (hipSetDevice(ctx->device) != hipSuccess) return GF2_E_HIP;
    const int64_t grid = std::min<int64_t>(count, (int64_t)ctx->cus * ctx->batch_bpc);
    hipError_t e = launch_pls_batched(items, (int)count, ranks, per_item, ss, (int32_t *)ws,
                                      (int)grid, (hipStream_t)stream);
    return e == hipSuccess ? GF2_OK : GF2_E_HIP;
}

}  // extern "C"

namespace {
// Workspace of gf2_rref.  Every extent of the solve depends on the rank, which
// only the device knows: `rr` holds {0, r, ceil((n - r) / 64)} (written by the
// first kernel), and every later launch is sized for the largest possible rank
// rmax = min(m, n) and clipped to rr on the device.
struct RrefLayout {
    size_t rr, pm, nm, pp, pn, uc, xc, bt, total;
    int64_t su, sx;
    int rmax, nw;
};

RrefLayout rref_layout(int64_t m, int64_t n) {
    RrefLayout L;
    const int64_t nw = std::max<int64_t>((n + 63) / 64, 1);
    L.nw = (int)nw;
    L.rmax = (int)std::min(m, n);
    L.su = std::max<int64_t>((L.rmax + 63) / 64, 1);
    L.sx = nw;
    size_t off = 0;
    L.rr = off; off = align_up(off + 16);
    L.pm = off; off = align_up(off + nw * 8);
    L.nm = off; off = align_up(off + nw * 8);
    L.pp = off; off = align_up(off + (nw + 1) * 4);
    L.pn = off; off = align_up(off + (nw + 1) * 4);
    L.uc = off; off = align_up(off + (size_t)std::max(L.rmax, 1) * L.su * 8);
    L.xc = off; off = align_up(off + (size_t)std::max(L.rmax, 1) * L.sx * 8);
    L.bt = off;
    off = align_up(off + gemm_bt_words((int)nw, std::max(64, (L.rmax / 64 / 2 + 1) * 64)) * 8);
    L.total = off;
    return L;
}

// X <- U^{-1} X for the unit upper triangular U (r x r, rows of Uc) on the
// compact non-pivot block X (r rows, rr[2] words): recursive on row halves,
// the lower half first, the coupling block by one product (Section 5 reduces
// the triangular solve to products), blocks of up to 1024 rows by the blocked
// table solve.  Launched for rmax rows and nwmax words; the kernels clip both
// to rr on the device.
struct UpperSolve {
    gf2_ctx *ctx;
    uint64_t *X;
    int64_t sx;
    const uint64_t *U;
    int64_t su;
    int rmax, nwmax, schur;
    const int32_t *rr;
    uint64_t *Bt;
    hipStream_t st;
    hipError_t err = hipSuccess;
    void chk(hipError_t e) {
        if (err == hipSuccess && e != hipSuccess) err = e;
    }
    // rows [a, min(r, a + sz)) <- U^{-1} rows, solving the last rows first
    void solve(int a, int sz) {
        if (a >= rmax || sz <= 0) return;
        if (sz <= trsm_block_max_rows()) {
            chk(launch_trsm_block(X, sx, U, su, rmax, row_range(-1, 1, a, sz), a / 64, 0, nwmax, rr,
                                  0, (sz + 63) / 64, nullptr, nullptr, 0, 0, st, rr + 2));
            return;
        }
        const int h = (sz / 64 / 2) * 64;
        solve(a + h, sz - h);
        chk(enqueue_gemm(ctx, X, sx, U, su, X, sx, rmax, rmax, row_range(-1, 1, a, h), (a + h) / 64,
                         0, nwmax, row_range(-1, 1, a + h, sz - h), sz - h, schur, rr, Bt, st,
                         false, rr + 2));
        solve(a, h);
    }
};
}  // namespace

namespace {
// Y <- L^{-1} Y for the unit lower triangle L of rows [0, r) of an in-place PLS
// (strictly lower bits stored in columns [0, r)), nw words of right-hand sides:
// recursive on row halves, the coupling block by one product, blocks of up to
// 1024 rows by the blocked table solve.  Launched for rmax rows; the kernels
// clip to ext[1] = r on the device.
struct LowerSolve {
    gf2_ctx *ctx;
    uint64_t *Y;
    int64_t sy;
    const uint64_t *L;
    int64_t sl;
    int rmax, nw, schur;
    const int32_t *ext;
    uint64_t *Bt;
    hipStream_t st;
    hipError_t err = hipSuccess;
    void chk(hipError_t e) {
        if (err == hipSuccess && e != hipSuccess) err = e;
    }
    void solve(int a, int sz) {
        if (a >= rmax || sz <= 0) return;
        if (sz <= trsm_block_max_rows()) {
            chk(launch_trsm_block(Y, sy, L, sl, rmax, row_range(-1, 1, a, sz), a / 64, 0, nw, ext, 1,
                                  (sz + 63) / 64, nullptr, nullptr, 0, 0, st));
            return;
        }
        const int h = (sz / 64 / 2) * 64;
        solve(a, h);
        chk(enqueue_gemm(ctx, Y, sy, L, sl, Y, sy, rmax, rmax, row_range(-1, 1, a + h, sz - h), a / 64,
                         0, nw, row_range(-1, 1, a, h), h, schur, ext, Bt, st));
        solve(a + h, sz - h);
    }
};

// Workspace of gf2_solve.
struct SolveLayout {
    size_t ext, rr, perm, cnt, off, fill, list, y, pm, nm, pp, pn, uc, bt, total;
    int64_t su, sy;
    int rmax, nw, nrw;
};

SolveLayout solve_layout(int64_t m, int64_t n, int64_t nrhs) {
    SolveLayout L;
    L.nw = (int)std::max<int64_t>((n + 63) / 64, 1);
    L.nrw = (int)std::max<int64_t>((nrhs + 63) / 64, 1);
    L.rmax = (int)std::min(m, n);
    L.su = std::max<int64_t>((L.rmax + 63) / 64, 1);
    L.sy = L.nrw;
    const size_t mm = (size_t)std::max<int64_t>(m, 1);
    size_t off = 0;
    L.ext = off; off = align_up(off + 16);
    L.rr = off; off = align_up(off + 16);
    L.perm = off; off = align_up(off + mm * 4);
    L.cnt = off; off = align_up(off + mm * 4);
    L.off = off; off = align_up(off + (mm + 1) * 4);
    L.fill = off; off = align_up(off + mm * 4);
    L.list = off; off = align_up(off + (size_t)std::max(L.rmax, 1) * 4);
    L.y = off; off = align_up(off + mm * L.sy * 8);
    L.pm = off; off = align_up(off + (size_t)L.nw * 8);
    L.nm = off; off = align_up(off + (size_t)L.nw * 8);
    L.pp = off; off = align_up(off + (size_t)(L.nw + 1) * 4);
    L.pn = off; off = align_up(off + (size_t)(L.nw + 1) * 4);
    L.uc = off; off = align_up(off + (size_t)std::max(L.rmax, 1) * L.su * 8);
    L.bt = off; off = align_up(off + gemm_bt_words(L.nrw, std::max(L.rmax, 64)) * 8);
    L.total = off;
    return L;
}

// Workspace of gf2_kernel_basis.
struct KernelLayout {
    size_t rr, pm, nm, pp, pn, uc, xc, bt, xt, total;
    int64_t su, sx, sxt;
    int rmax, nw;
};

KernelLayout kernel_layout(int64_t m, int64_t n) {
    KernelLayout L;
    L.nw = (int)std::max<int64_t>((n + 63) / 64, 1);
    L.rmax = (int)std::min(m, n);
    L.su = std::max<int64_t>((L.rmax + 63) / 64, 1);
    L.sx = L.nw;
    L.sxt = L.su;
    size_t off = 0;
    L.rr = off; off = align_up(off + 16);
    L.pm = off; off = align_up(off + (size_t)L.nw * 8);
    L.nm = off; off = align_up(off + (size_t)L.nw * 8);
    L.pp = off; off = align_up(off + (size_t)(L.nw + 1) * 4);
    L.pn = off; off = align_up(off + (size_t)(L.nw + 1) * 4);
    L.uc = off; off = align_up(off + (size_t)std::max(L.rmax, 1) * L.su * 8);
    L.xc = off; off = align_up(off + (size_t)std::max(L.rmax, 1) * L.sx * 8);
    L.bt = off;
    off = align_up(off + gemm_bt_words(L.nw, std::max(64, (L.rmax / 64 / 2 + 1) * 64)) * 8);
    L.xt = off; off = align_up(off + (size_t)64 * L.nw * L.sxt * 8);
    L.total = off;
    return L;
}
}  // namespace

extern "C" size_t gf2_solve_workspace_bytes(int64_t m, int64_t n, int64_t nrhs) {
    if (m < 0 || n < 0 || nrhs < 0 || m > kMaxDim || n > kMaxDim || nrhs > kMaxDim) return 0;
    return solve_layout(m, n, nrhs).total;
}

extern "C" int gf2_solve(gf2_ctx *ctx, gf2_mat A_pls, const int32_t *P, const int32_t *Q,
                         const int32_t *rank, gf2_mat B, gf2_mat X_out, uint64_t *bad,
                         const gf2_sched *s, void *ws, size_t ws_bytes, void *stream) {
    if (!ctx) return GF2_E_ARG;
    int rc;
    if ((rc = check_mat(A_pls)) != GF2_OK) return rc;
    if ((rc = check_mat(B)) != GF2_OK) return rc;
    if ((rc = check_mat(X_out)) != GF2_OK) return rc;
    if (B.m != A_pls.m || X_out.m != A_pls.n || X_out.n != B.n) return GF2_E_ARG;
    if (!rank || (A_pls.m > 0 && !P) || (A_pls.n > 0 && !Q) || (B.n > 0 && !bad)) return GF2_E_ARG;
    if (((uintptr_t)bad & 7) != 0) return GF2_E_ALIGN;
    const gf2_sched ss = s ? *s : default_sched();
    if (!sched_ok(&ss)) return GF2_E_ARG;
    SolveLayout L = solve_layout(A_pls.m, A_pls.n, B.n);
    if (!ws || ws_bytes < L.total) return GF2_E_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return GF2_E_ALIGN;
    if (B.n == 0 || A_pls.n == 0) return GF2_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return GF2_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    const int m = (int)A_pls.m, n = (int)A_pls.n, nrw = (int)((B.n + 63) / 64);
    int32_t *ext = (int32_t *)(base + L.ext), *rr = (int32_t *)(base + L.rr);
    int32_t *perm = (int32_t *)(base + L.perm);
    uint64_t *Y = (uint64_t *)(base + L.y);
    uint64_t *PM = (uint64_t *)(base + L.pm), *NM = (uint64_t *)(base + L.nm);
    int32_t *pp = (int32_t *)(base + L.pp), *pn = (int32_t *)(base + L.pn);
    uint64_t *Uc = (uint64_t *)(base + L.uc), *Bt = (uint64_t *)(base + L.bt);
    GF2_TRY(launch_solve_extents(rank, L.rmax, nrw, ext, st));
    if (m > 0) {
        // Y = P B
        GF2_TRY(launch_perm_from_swaps(P, rank, m, L.rmax, (int32_t *)(base + L.cnt),
                                       (int32_t *)(base + L.off), (int32_t *)(base + L.fill),
                                       (int32_t *)(base + L.list), perm, st));
        GF2_TRY(launch_gather_rows(Y, L.sy, B.words, B.stride, perm, m, nrw, st));
        // forward substitution with L's unit lower triangle on rows [0, r)
        LowerSolve fw{ctx, Y, L.sy, A_pls.words, A_pls.stride, L.rmax, nrw, ss.schur, ext, Bt, st};
        fw.solve(0, (L.rmax + 63) / 64 * 64);
        if (fw.err != hipSuccess) return GF2_E_HIP;
        // rows [r, m): Y_bottom + L_bottom Y_top must vanish
        GF2_TRY(enqueue_gemm(ctx, Y, L.sy, A_pls.words, A_pls.stride, Y, L.sy, m, m,
                             row_range(1, -1, 0, kINF), 0, 0, nrw, row_range(-1, 1, 0, kINF),
                             std::max(L.rmax, 1), ss.schur, ext, Bt, st));
        GF2_TRY(launch_consistency(Y, L.sy, m, nrw, ext, bad, st));
        // back substitution: U_Q = S[:, Q], Y_top <- U_Q^{-1} Y_top
        GF2_TRY(launch_rref_masks(PM, NM, pp, pn, Q, rank, n, L.rmax, rr, st));
        GF2_TRY(launch_rref_zero(Uc, L.su, nullptr, 0, L.rmax, ext, st));
        GF2_TRY(launch_rref_gather(A_pls.words, A_pls.stride, Q, L.rmax, n, PM, NM, pp, pn, Uc, L.su,
                                   nullptr, 0, ext, st));
        UpperSolve bw;
        bw.ctx = ctx;
        bw.X = Y; bw.sx = L.sy; bw.U = Uc; bw.su = L.su;
        bw.rmax = L.rmax; bw.nwmax = nrw; bw.schur = ss.schur;
        bw.rr = ext; bw.Bt = Bt; bw.st = st;
        bw.solve(0, (L.rmax + 63) / 64 * 64);
        if (bw.err != hipSuccess) return GF2_E_HIP;
    } else {
        GF2_TRY(launch_zero_rows(bad, nrw, 1, nrw, st));
        GF2_TRY(launch_zero_rows(PM, L.nw, 1, L.nw, st));
        GF2_TRY(launch_fill_i32(pp, 0, L.nw + 1, st));
    }
    // X[Q[i]] = Y[i], the other rows zero
    GF2_TRY(launch_solve_scatter(X_out.words, X_out.stride, n, nrw, Y, L.sy, PM, pp, st));
    if (X_out.stride > nrw)
        GF2_TRY(launch_zero_rows(X_out.words + nrw, X_out.stride, n, (int)(X_out.stride - nrw), st));
    return GF2_OK;
}

extern "C" size_t gf2_kernel_basis_workspace_bytes(int64_t m, int64_t n) {
    if (m < 0 || n < 0 || m > kMaxDim || n > kMaxDim) return 0;
    return kernel_layout(m, n).total;
}

extern "C" int gf2_kernel_basis(gf2_ctx *ctx, gf2_mat A_pls, const int32_t *Q, const int32_t *rank,
                                gf2_mat K_out, const gf2_sched *s, void *ws, size_t ws_bytes,
                                void *stream) {
    if (!ctx) return GF2_E_ARG;
    int rc;
    if ((rc = check_mat(A_pls)) != GF2_OK) return rc;
    if ((rc = check_mat(K_out)) != GF2_OK) return rc;
    if (K_out.m != A_pls.n || K_out.n != A_pls.n) return GF2_E_ARG;
    if (!rank || (A_pls.n > 0 && !Q)) return GF2_E_ARG;
    if (K_out.words == A_pls.words && A_pls.n > 0) return GF2_E_ARG;
    const gf2_sched ss = s ? *s : default_sched();
    if (!sched_ok(&ss)) return GF2_E_ARG;
    KernelLayout L = kernel_layout(A_pls.m, A_pls.n);
    if (!ws || ws_bytes < L.total) return GF2_E_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return GF2_E_ALIGN;
    if (A_pls.n == 0) return GF2_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return GF2_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    const int n = (int)A_pls.n;
    int32_t *rr = (int32_t *)(base + L.rr);
    uint64_t *PM = (uint64_t *)(base + L.pm), *NM = (uint64_t *)(base + L.nm);
    int32_t *pp = (int32_t *)(base + L.pp), *pn = (int32_t *)(base + L.pn);
    uint64_t *Uc = (uint64_t *)(base + L.uc), *Xc = (uint64_t *)(base + L.xc);
    uint64_t *XT = (uint64_t *)(base + L.xt);
    // rank 0 with no rows (m == 0) still has every column free
    GF2_TRY(launch_rref_masks(PM, NM, pp, pn, Q, rank, n, L.rmax, rr, st));
    if (L.rmax > 0) {
        // Xc = U_Q^{-1} S[:, N], the non-pivot columns of the RREF (as in gf2_rref)
        GF2_TRY(launch_rref_zero(Uc, L.su, Xc, L.sx, L.rmax, rr, st));
        GF2_TRY(launch_rref_gather(A_pls.words, A_pls.stride, Q, L.rmax, n, PM, NM, pp, pn, Uc, L.su,
                                   Xc, L.sx, rr, st));
        UpperSolve us;
        us.ctx = ctx;
        us.X = Xc; us.sx = L.sx; us.U = Uc; us.su = L.su;
        us.rmax = L.rmax; us.nwmax = L.nw; us.schur = ss.schur;
        us.rr = rr; us.Bt = (uint64_t *)(base + L.bt); us.st = st;
        us.solve(0, (L.rmax + 63) / 64 * 64);
        if (us.err != hipSuccess) return GF2_E_HIP;
        // XT row j = column j of Xc over rows [0, r) (bits past r zero)
        GF2_TRY(launch_transpose(Xc, L.sx, L.rmax, row_range(-1, 1, 0, kINF), 0, L.nw, L.rmax, XT,
                                 L.sxt, rr, st, rr + 2));
    }
    GF2_TRY(launch_kernel_scatter(K_out.words, K_out.stride, n, XT, L.sxt, PM, NM, pp, pn, rr, st));
    const int nw = (n + 63) / 64;
    if (K_out.stride > nw)
        GF2_TRY(launch_zero_rows(K_out.words + nw, K_out.stride, n, (int)(K_out.stride - nw), st));
    return GF2_OK;
}

extern "C" size_t gf2_rref_workspace_bytes(int64_t m, int64_t n) {
    if (m < 0 || n < 0 || m > kMaxDim || n > kMaxDim) return 0;
    return rref_layout(m, n).total;
}

namespace {
// The RREF sequence on validated arguments.  R_out may be A_pls itself (the
// hybrid works in place): A_pls is last read by the gather, before the scatter
// writes R.  zero_pad: clear R_out's words past ceil(n / 64) up to its stride.
int rref_run(gf2_ctx *ctx, const gf2_mat &A_pls, const int32_t *Q, const int32_t *rank,
             const gf2_mat &R_out, const gf2_sched &ss, const RrefLayout &L, char *base,
             hipStream_t st, bool zero_pad) {
    if (A_pls.m == 0 || A_pls.n == 0) return GF2_OK;
    const int m = (int)A_pls.m, n = (int)A_pls.n;
    int32_t *rr = (int32_t *)(base + L.rr);
    uint64_t *PM = (uint64_t *)(base + L.pm), *NM = (uint64_t *)(base + L.nm);
    int32_t *pp = (int32_t *)(base + L.pp), *pn = (int32_t *)(base + L.pn);
    uint64_t *Uc = (uint64_t *)(base + L.uc), *Xc = (uint64_t *)(base + L.xc);
    GF2_TRY(launch_rref_masks(PM, NM, pp, pn, Q, rank, n, L.rmax, rr, st));
    // with no non-pivot column (r == n) every kernel below returns at once: R is
    // the pivot pattern alone
    GF2_TRY(launch_rref_zero(Uc, L.su, Xc, L.sx, L.rmax, rr, st));
    GF2_TRY(launch_rref_gather(A_pls.words, A_pls.stride, Q, L.rmax, n, PM, NM, pp, pn, Uc, L.su, Xc,
                               L.sx, rr, st));
    UpperSolve us;
    us.ctx = ctx;
    us.X = Xc; us.sx = L.sx; us.U = Uc; us.su = L.su;
    us.rmax = L.rmax; us.nwmax = L.nw; us.schur = ss.schur;
    us.rr = rr; us.Bt = (uint64_t *)(base + L.bt); us.st = st;
    us.solve(0, (L.rmax + 63) / 64 * 64);
    if (us.err != hipSuccess) return GF2_E_HIP;
    GF2_TRY(launch_rref_scatter(R_out.words, R_out.stride, m, n, Q, rr, NM, pn, Xc, L.sx, st));
    const int nw = (n + 63) / 64;
    if (zero_pad && R_out.stride > nw)
        GF2_TRY(launch_zero_rows(R_out.words + nw, R_out.stride, m, (int)(R_out.stride - nw), st));
    return GF2_OK;
}
}  // namespace

extern "C" int gf2_rref(gf2_ctx *ctx, gf2_mat A_pls, const int32_t *Q, const int32_t *rank,
                        gf2_mat R_out, const gf2_sched *s, void *ws, size_t ws_bytes,
                        void *stream) {
    if (!ctx) return GF2_E_ARG;
    int rc;
    if ((rc = check_mat(A_pls)) != GF2_OK) return rc;
    if ((rc = check_mat(R_out)) != GF2_OK) return rc;
    if (R_out.m != A_pls.m || R_out.n != A_pls.n) return GF2_E_ARG;
    if (!rank || (A_pls.n > 0 && !Q)) return GF2_E_ARG;
    if (R_out.words == A_pls.words && A_pls.m > 0) return GF2_E_ARG;
    const gf2_sched ss = s ? *s : default_sched();
    if (!sched_ok(&ss)) return GF2_E_ARG;
    RrefLayout L = rref_layout(A_pls.m, A_pls.n);
    if (!ws || ws_bytes < L.total) return GF2_E_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return GF2_E_ALIGN;
    if (A_pls.m == 0 || A_pls.n == 0) return GF2_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return GF2_E_HIP;
    return rref_run(ctx, A_pls, Q, rank, R_out, ss, L, (char *)ws, (hipStream_t)stream, true);
}

// ------------------------------------------------------------------ M4RI
namespace {
struct M4riLayout {
    size_t rk, info, rec, bbuf, p, dens, cbuf, total;
    int64_t bstride;
    int nb;
};

M4riLayout m4ri_layout(int64_t m, int64_t n) {
    M4riLayout L;
    L.nb = (int)((n + 63) / 64);
    L.bstride = std::max(L.nb, 1);
    size_t off = 0;
    L.rk = off; off = align_up(off + (size_t)(L.nb + 2) * 4);
    L.info = off; off = align_up(off + panel_info_bytes());
    L.rec = off; off = align_up(off + m4ri_rec_bytes());
    L.bbuf = off; off = align_up(off + (size_t)64 * L.bstride * 8);
    L.p = off; off = align_up(off + (size_t)std::max<int64_t>(m, 1) * 4);
    L.dens = off; off = align_up(off + 16);
    L.cbuf = off; off = align_up(off + (size_t)std::max<int64_t>(m, 1) * 8);
    L.total = off;
    return L;
}

// One M4RI strip (Section 3.1) on the 64-column panel p: the panel search and
// its final pass (GaussSubmatrix's pivots, rows moved into place), the change
// of basis to the reduced pivot rows, and the table-driven reduction of every
// other row (MakeTable / AddRowsFromTable above and below).
hipError_t m4ri_step(gf2_ctx *ctx, const gf2_mat &A, const M4riLayout &L, char *base,
                     int32_t *Q, const gf2_sched &ss, int p, hipStream_t st) {
    int32_t *rk = (int32_t *)(base + L.rk);
    int32_t *info = (int32_t *)(base + L.info);
    uint64_t *Bbuf = (uint64_t *)(base + L.bbuf);
    const int m = (int)A.m, n = (int)A.n, nw = L.nb;
    hipError_t e = launch_leaf(A.words, A.stride, A.words, A.stride, 0, (int)A.stride, m, n, p, rk, p,
                               (int32_t *)(base + L.p), Q, info, Bbuf, L.bstride, p + 1, nw,
                               nullptr, st);
    if (e != hipSuccess) return e;
    if ((e = launch_m4ri_prep(info, rk, p, base + L.rec, st)) != hipSuccess) return e;
    return launch_m4ri_update(A.words, A.stride, m, p, rk, p, p + 1, nw, ss.k, ss.tables,
                              (const uint64_t *)(base + L.info + panel_info_linv_offset()),
                              base + L.rec, (uint64_t *)(base + L.cbuf), Bbuf, L.bstride, ctx->cus,
                              st);
}

// Workspace of the hybrid: the M4RI part, then (for the switch to PLS on the
// remaining block) a PLS workspace, an RREF workspace, P2, Q2, rank2, the
// pivot masks of the block, the gathered pivot columns of the rows above, the
// extents and the product's transposed operand.
struct MpLayout {
    M4riLayout m4;
    size_t pls, rref, p2, q2, r2, pm, nm, pp, pn, rr, cbuf, ext, bt, total;
    size_t pls_bytes, rref_bytes;
    int64_t sc;
};

MpLayout mp_layout(int64_t m, int64_t n, const gf2_sched &s) {
    MpLayout L;
    L.m4 = m4ri_layout(m, n);
    const int nb = L.m4.nb;
    // the block left for PLS is at most m x (n - 64 p) for the panel p it starts
    // at; every workspace term grows with both sizes
    size_t pb = 0;
    for (int p = 0; p < nb; p++) pb = std::max(pb, pls_layout(m, n - 64 * (int64_t)p, s).total);
    L.pls_bytes = pb;
    L.rref_bytes = rref_layout(m, n).total;
    const int64_t rmax = std::min(m, n);
    L.sc = std::max<int64_t>((rmax + 63) / 64, 1);
    const size_t nwp = (size_t)std::max(nb, 1);
    size_t off = L.m4.total;
    L.pls = off; off = align_up(off + pb);
    L.rref = off; off = align_up(off + L.rref_bytes);
    L.p2 = off; off = align_up(off + (size_t)std::max<int64_t>(m, 1) * 4);
    L.q2 = off; off = align_up(off + (size_t)std::max<int64_t>(n, 1) * 4);
    L.r2 = off; off = align_up(off + 16);
    L.pm = off; off = align_up(off + nwp * 8);
    L.nm = off; off = align_up(off + nwp * 8);
    L.pp = off; off = align_up(off + (nwp + 1) * 4);
    L.pn = off; off = align_up(off + (nwp + 1) * 4);
    L.rr = off; off = align_up(off + 16);
    L.cbuf = off; off = align_up(off + (size_t)std::max<int64_t>(m, 1) * L.sc * 8);
    L.ext = off; off = align_up(off + 16);
    L.bt = off; off = align_up(off + gemm_bt_words((int)nwp, (int)std::max<int64_t>(rmax, 64)) * 8);
    L.total = off;
    return L;
}

int check_m4ri_args(gf2_ctx *ctx, const gf2_mat &A, const int32_t *Q, const int32_t *rank,
                    const gf2_sched *s, gf2_sched *ss) {
    if (!ctx) return GF2_E_ARG;
    int rc = check_mat(A);
    if (rc != GF2_OK) return rc;
    *ss = s ? *s : default_sched();
    if (!sched_ok(ss)) return GF2_E_ARG;
    if (!rank || (A.n > 0 && !Q)) return GF2_E_ARG;
    return GF2_OK;
}
}  // namespace

extern "C" size_t gf2_m4ri_workspace_bytes(int64_t m, int64_t n) {
    if (m < 0 || n < 0 || m > kMaxDim || n > kMaxDim) return 0;
    return m4ri_layout(m, n).total;
}

extern "C" int gf2_m4ri(gf2_ctx *ctx, gf2_mat A, int32_t *Q, int32_t *rank, const gf2_sched *s,
                        void *ws, size_t ws_bytes, void *stream) {
    gf2_sched ss;
    int rc = check_m4ri_args(ctx, A, Q, rank, s, &ss);
    if (rc != GF2_OK) return rc;
    M4riLayout L = m4ri_layout(A.m, A.n);
    if (!ws || ws_bytes < L.total) return GF2_E_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return GF2_E_ALIGN;
    if (hipSetDevice(ctx->device) != hipSuccess) return GF2_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    int32_t *rk = (int32_t *)(base + L.rk);
    GF2_TRY(launch_fill_i32(rk, 0, L.nb + 1, st));
    if (A.m > 0)
        for (int p = 0; p < L.nb; p++) GF2_TRY(m4ri_step(ctx, A, L, base, Q, ss, p, st));
    GF2_TRY(launch_finalize((int32_t *)(base + L.p), Q, rank, rk, L.nb, (int)A.m, (int)A.n, st));
    return GF2_OK;
}

extern "C" size_t gf2_rref_mp_workspace_bytes(int64_t m, int64_t n, const gf2_sched *s) {
    if (m < 0 || n < 0 || m > kMaxDim || n > kMaxDim) return 0;
    const gf2_sched ss = s ? *s : default_sched();
    if (!sched_ok(&ss)) return 0;
    return mp_layout(m, n, ss).total;
}

extern "C" int gf2_rref_mp(gf2_ctx *ctx, gf2_mat A, int32_t *Q, int32_t *rank, float threshold,
                           int32_t *switch_panel, const gf2_sched *s, void *ws, size_t ws_bytes,
                           void *stream) {
    gf2_sched ss;
    int rc = check_m4ri_args(ctx, A, Q, rank, s, &ss);
    if (rc != GF2_OK) return rc;
    if (!(threshold >= 0.f)) return GF2_E_ARG;
    MpLayout L = mp_layout(A.m, A.n, ss);
    if (!ws || ws_bytes < L.total) return GF2_E_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return GF2_E_ALIGN;
    if (hipSetDevice(ctx->device) != hipSuccess) return GF2_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    const M4riLayout &M = L.m4;
    int32_t *rk = (int32_t *)(base + M.rk);
    int32_t *dens = (int32_t *)(base + M.dens);
    const int m = (int)A.m, n = (int)A.n;
    GF2_TRY(launch_fill_i32(rk, 0, M.nb + 1, st));
    int sw = -1, R = 0;
    for (int p = 0; p < M.nb && m > 0; p++) {
        // approximated density of what is left (Section 6), read back here: the
        // switch decides which kernels follow
        GF2_TRY(launch_m4ri_density(A.words, A.stride, m, n, p, rk, p, dens, st));
        int32_t h[2];
        GF2_TRY(hipMemcpyAsync(h, dens, sizeof h, hipMemcpyDeviceToHost, st));
        GF2_TRY(hipStreamSynchronize(st));
        float d;
        std::memcpy(&d, &h[0], sizeof d);
        R = h[1];
        if (R >= m) {
            // every row has its pivot: the remaining strips find none
            GF2_TRY(launch_fill_i32(rk + p + 1, R, M.nb - p, st));
            break;
        }
        if (d >= threshold) {
            sw = p;
            break;
        }
        GF2_TRY(m4ri_step(ctx, A, M, base, Q, ss, p, st));
    }
    if (switch_panel) *switch_panel = sw;
    if (sw < 0) {
        GF2_TRY(launch_finalize((int32_t *)(base + M.p), Q, rank, rk, M.nb, m, n, st));
        return GF2_OK;
    }
    // PLS and its RREF on the remaining block: rows [R, m), columns [64 sw, n)
    gf2_mat sub;
    sub.words = A.words + (int64_t)R * A.stride + sw;
    sub.m = m - R;
    sub.n = n - 64 * (int64_t)sw;
    sub.stride = A.stride;
    int32_t *P2 = (int32_t *)(base + L.p2), *Q2 = (int32_t *)(base + L.q2);
    int32_t *r2 = (int32_t *)(base + L.r2);
    PlsLayout PL = pls_layout(sub.m, sub.n, ss);
    if (PL.total > L.pls_bytes) return GF2_E_WORKSPACE;
    if ((rc = pls_run(ctx, sub, P2, Q2, r2, ss, PL, base + L.pls, st)) != GF2_OK) return rc;
    RrefLayout RL = rref_layout(sub.m, sub.n);
    if (RL.total > L.rref_bytes) return GF2_E_WORKSPACE;
    if ((rc = rref_run(ctx, sub, Q2, r2, sub, ss, RL, base + L.rref, st, false)) != GF2_OK) return rc;
    int32_t *ext = (int32_t *)(base + L.ext);
    GF2_TRY(launch_mp_finish(Q, rank, ext, Q2, r2, R, 64 * sw, n, st));
    if (R > 0) {
        // rows above: clear the block's pivot columns with the block's RREF rows,
        // X_top += X_top[:, Q2] R2 (R2[:, Q2] = I)
        const int nws = (int)((sub.n + 63) / 64);
        const int rmax2 = (int)std::min(sub.m, sub.n);
        uint64_t *PM = (uint64_t *)(base + L.pm), *NM = (uint64_t *)(base + L.nm);
        int32_t *pp = (int32_t *)(base + L.pp), *pn = (int32_t *)(base + L.pn);
        uint64_t *C = (uint64_t *)(base + L.cbuf);
        GF2_TRY(launch_rref_masks(PM, NM, pp, pn, Q2, r2, (int)sub.n, rmax2, (int32_t *)(base + L.rr),
                                  st));
        GF2_TRY(launch_zero_rows(C, L.sc, R, (int)L.sc, st));
        GF2_TRY(launch_gather_cols(A.words + sw, A.stride, R, nws, PM, pp, C, L.sc, st));
        GF2_TRY(enqueue_gemm(ctx, A.words, A.stride, C, L.sc, A.words, A.stride, R, m,
                             row_range(-1, -1, 0, kINF), 0, sw, nws, row_range(0, 1, 0, kINF),
                             std::max(rmax2, 1), ss.schur, ext, (uint64_t *)(base + L.bt), st));
    }
    return GF2_OK;
}

extern "C" {

size_t gf2_addmul_workspace_bytes(int64_t m, int64_t k, int64_t n) {
    if (m < 0 || k < 0 || n < 0 || m > kMaxDim || k > kMaxDim || n > kMaxDim) return 0;
    int64_t kc = std::min<int64_t>(k, kMfmaMaxK);
    size_t bt = (size_t)((n + 63) / 64) * 64 * ((kc + 63) / 64);
    return align_up(256) + align_up(bt * 8);
}

int gf2_addmul(gf2_ctx *ctx, gf2_mat C, gf2_mat A, gf2_mat B, int variant, void *ws,
               size_t ws_bytes, void *stream) {
    if (!ctx) return GF2_E_ARG;
    int rc;
    if ((rc = check_mat(C)) != GF2_OK) return rc;
    if ((rc = check_mat(A)) != GF2_OK) return rc;
    if ((rc = check_mat(B)) != GF2_OK) return rc;
    if (A.m != C.m || B.n != C.n || A.n != B.m) return GF2_E_ARG;
    if (variant != GF2_SCHUR_XOR && variant != GF2_SCHUR_MFMA && variant != GF2_SCHUR_FP4)
        return GF2_E_ARG;
    size_t need = gf2_addmul_workspace_bytes(C.m, A.n, C.n);
    if (!ws || ws_bytes < need) return GF2_E_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return GF2_E_ALIGN;
    if (C.m == 0 || C.n == 0 || A.n == 0) return GF2_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return GF2_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    int32_t *rk = (int32_t *)ws;
    uint64_t *Bt = (uint64_t *)((char *)ws + align_up(256));
    const int m = (int)C.m, K = (int)A.n, nw = (int)((C.n + 63) / 64);
    // rk[0] = 0, rk[1] = K: rows of B are [rk[0], rk[1])
    GF2_TRY(launch_fill_i32(rk, 0, 1, st));
    GF2_TRY(launch_fill_i32(rk + 1, K, 1, st));
    for (int k0 = 0; k0 < K; k0 += kMfmaMaxK) {
        const int kc = std::min(kMfmaMaxK, K - k0);
        RowRange br = row_range(0, 1, k0, kc);
        const int64_t sbt = (kc + 63) / 64;
        GF2_TRY(launch_transpose(B.words, B.stride, K, br, 0, nw, kc, Bt, sbt, rk, st));
        RowRange cr = row_range(-1, -1, 0, kINF);
        if (variant == GF2_SCHUR_MFMA || variant == GF2_SCHUR_FP4)
            GF2_TRY(launch_gemm_mfma(C.words, C.stride, A.words, A.stride, m, cr, k0 / 64, 0, nw, Bt,
                                     sbt, kc, br, K, rk, nullptr, variant == GF2_SCHUR_FP4, st));
        else
            GF2_TRY(launch_gemm_xor(C.words, C.stride, A.words, A.stride, m, cr, k0 / 64, 0, nw, Bt,
                                    sbt, kc, br, K, rk, nullptr, st));
    }
    return GF2_OK;
}

}  // extern "C"

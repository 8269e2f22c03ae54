/*
 * gf2pls -- PLS decomposition and reduced row echelon form of dense GF(2)
 * matrices on AMD Instinct MI355X (gfx950).
 *
 * Method: Albrecht & Pernet, "Efficient Decomposition of Dense Matrices over
 * GF(2)".  The decomposition follows the problem statement of Section 2
 * (Proposition "PLS decomposition": any m x n matrix A of rank r can be written
 * A = P L S, P an m x m permutation, L m x r unit lower triangular, S r x n upper
 * triangular up to a column permutation, here chosen in row echelon form), computed
 * in place as in Sections 4-5 (L below the main diagonal, S on and above it).
 *
 * Conventions shared by every call
 *  - Matrices are bit-packed row-major in 64-bit words: column j of row i is bit
 *    (j mod 64) of words[i * stride + j / 64].  Bits past column n must be zero
 *    on input and stay zero.  `words` is a DEVICE pointer, 8-byte aligned.
 *  - Permutations use the transposition ("swap sequence") form of the paper's
 *    algorithms: step i exchanged rows i and P[i] (i < r, P[i] >= i); pivot i lies
 *    in column Q[i].  P[i] = i for i >= r and Q[i] = i for r <= i < n.  Indices
 *    are 0-based int32 in DEVICE memory.
 *  - The caller owns every buffer.  No call allocates device memory; scratch
 *    space comes from a caller-provided workspace of the size the matching
 *    *_workspace_bytes call reports.  The library keeps no pointer after a call.
 *  - Calls are asynchronous on the given stream (a hipStream_t passed as void*;
 *    NULL is the default stream).  Arguments are validated on the host before
 *    anything is enqueued, so on error nothing is written.
 *  - Return value: GF2_OK (0) or a negative gf2_status.
 *  - A gf2_ctx is not thread-safe; use one per host thread.
 */
#ifndef GF2PLS_H
#define GF2PLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gf2_status {
    GF2_OK = 0,
    GF2_E_ARG = -1,         /* bad size, null pointer or out-of-range schedule     */
    GF2_E_ALIGN = -2,       /* stride < ceil(n/64) or misaligned pointer          */
    GF2_E_WORKSPACE = -3,   /* workspace missing or smaller than required         */
    GF2_E_HIP = -4,         /* a HIP runtime call failed                          */
    GF2_E_UNSUPPORTED = -5  /* size outside the supported range                   */
} gf2_status;

typedef struct gf2_ctx gf2_ctx;

/* A dense packed GF(2) matrix (device memory). */
typedef struct gf2_mat {
    uint64_t *words;
    int64_t m, n;
    int64_t stride; /* words per row, >= ceil(n / 64) */
} gf2_mat;

/* Schur-update variants for the recursive PLS (Section 5: A_SE <- A_SE + A_SW A_NE). */
enum { GF2_SCHUR_XOR = 0,   /* AND / XOR-popcount on the vector ALUs              */
       GF2_SCHUR_MFMA = 1,  /* int8 MFMA, int32 accumulation, reduced mod 2       */
       GF2_SCHUR_FP4 = 2    /* fp4 (e2m1) MFMA, fp32 accumulation of exact 0/1
                               products, reduced mod 2                            */ };

/*
 * Schedule.  Changes timing only, never a result bit.
 *  k       Gray-table width in bits for the table-driven updates (MakeTable1 /
 *          AddRowsFromTable, Section 4.1), 4..8.
 *  tables  tables applied per pass over the rows, 1, 2, 4 or 8.
 *  cutoff  recursion cutoff in columns (Section 6): column blocks of at most
 *          `cutoff` columns are factored by the MMPF base case.  Multiple of 64,
 *          64..2^30.  cutoff >= n runs MMPF alone.
 *  schur   GF2_SCHUR_XOR, GF2_SCHUR_MFMA or GF2_SCHUR_FP4.
 */
typedef struct gf2_sched {
    int32_t k;
    int32_t tables;
    int32_t cutoff;
    int32_t schur;
} gf2_sched;

/* Create a context on HIP device `device` (0-based).  *out is set on success. */
int gf2_ctx_create(gf2_ctx **out, int device);
void gf2_ctx_destroy(gf2_ctx *ctx);

/* Human-readable name of a status code (static storage). */
const char *gf2_status_str(int status);

/* The fixed default schedule (k 8, tables 8, cutoff 2048, GF2_SCHUR_FP4), the
 * fallback of any tuned or learned choice. */
void gf2_default_sched(gf2_sched *out);

/* Non-zero if `s` is a valid schedule. */
int gf2_sched_valid(const gf2_sched *s);

/* Workspace bytes gf2_pls needs for an m x n matrix under schedule s.  s == NULL:
 * enough for any schedule a call without one may run (the default or a learned
 * choice, see gf2_ctx_set_learned). */
size_t gf2_pls_workspace_bytes(int64_t m, int64_t n, const gf2_sched *s);

/*
 * PLS decomposition in place (Sections 4-5).
 * A is overwritten with the compressed in-place form: for i < r, columns < i of
 * row i hold L[i][.], column i holds 1, columns (i, Q[i]] hold 0 and columns
 * > Q[i] hold S[i][.]; for i >= r, columns < r hold L[i][.] and the rest 0.
 * P (m entries), Q (n entries) and *rank (one int32) are device pointers.
 * The result is identical to Gaussian PLS (Appendix A) for every schedule.
 * s == NULL: the context's learned choice for (m, n) when one is installed and
 * covers the shape (gf2_ctx_set_learned), else the default schedule.
 */
int gf2_pls(gf2_ctx *ctx, gf2_mat A, int32_t *P, int32_t *Q, int32_t *rank,
            const gf2_sched *s, void *ws, size_t ws_bytes, void *stream);

/*
 * gf2_pls without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, result and asynchrony as gf2_pls; the
 * scratch space is a fixed array of GF2_NOALLOC_SCRATCH_BYTES bytes that the
 * library holds on each device it runs on until the process ends.  Problems
 * whose gf2_pls_workspace_bytes exceeds that size return GF2_E_UNSUPPORTED
 * (nothing enqueued; 16 MiB covers 16384 x 16384 under the default schedule).
 * No HIP allocation is made by this call.  Every call on one device shares that
 * device's array: calls that overlap in time on one device (two streams, or two
 * host threads) race and give undefined results; calls ordered on one stream are
 * safe.  Everything the call needs zeroed is cleared by its own kernels.
 */
#define GF2_NOALLOC_SCRATCH_BYTES (16u << 20)
int gf2_pls_noalloc(gf2_ctx *ctx, gf2_mat A, int32_t *P, int32_t *Q, int32_t *rank,
                    const gf2_sched *s, void *stream);
size_t gf2_pls_noalloc_max_bytes(void);

/*
 * Explicit factors from a gf2_pls result (Section 2's A = P L S; in-place layout
 * of Sections 4-5).  A_pls, Q, rank are gf2_pls outputs (device); A_pls is only
 * read.  With rmax = min(m, n):
 *  L_out  m x rmax (device): row i has the stored L bits of columns < min(i, r),
 *         a one at column i when i < r, zeros elsewhere (columns >= r are zero).
 *  S_out  rmax x n (device): row i < r has a one at Q[i], zeros left of it and the
 *         stored S bits right of it; rows >= r are not written.
 * Then A = P L S with L truncated to r columns and S to r rows.
 */
int gf2_pls_unpack(gf2_ctx *ctx, gf2_mat A_pls, const int32_t *Q, const int32_t *rank,
                   gf2_mat L_out, gf2_mat S_out, void *stream);

/* Workspace bytes gf2_rref needs. */
size_t gf2_rref_workspace_bytes(int64_t m, int64_t n);

/*
 * Reduced row echelon form from a PLS (timed with the decomposition in the
 * paper's Table 1; Definition "Reduced Row Echelon Form", Section 2).
 * A_pls, Q and rank are gf2_pls outputs (device); A_pls is only read.
 * R_out (m x n, same shape as A_pls, its own buffer) receives the RREF of the
 * original A: rows < r in reduced echelon form with leading ones at Q[0..r),
 * rows >= r zero.  With U = S[:, Q] (unit upper triangular), R = U^{-1} S: only
 * the non-pivot columns need the triangular solve, which Section 5's reduction
 * turns into products; they use the schedule's Schur variant (s == NULL: the
 * default schedule; only the schur field is read).  Every extent depends on the
 * rank, which is read on the device: the call enqueues a fixed kernel sequence
 * sized for rank min(m, n), waits for nothing, and can be captured in a graph.
 */
int gf2_rref(gf2_ctx *ctx, gf2_mat A_pls, const int32_t *Q, const int32_t *rank,
             gf2_mat R_out, const gf2_sched *s, void *ws, size_t ws_bytes, void *stream);

/*
 * M4RI (Section 3.1, algorithm "M4RI"; GaussSubmatrix, MakeTable and
 * AddRowsFromTable of Appendix A): the reduced row echelon form directly, strip
 * by strip, every row above and below a strip's pivot rows reduced through
 * Gray-code tables of those rows.  Strips are 64-column panels; the schedule's
 * k and tables set the table width and the tables per pass (cutoff and schur
 * are not used).
 *  A      m x n (device), overwritten with its RREF: rows < r in reduced echelon
 *         form with leading ones at Q[0, r), rows >= r zero.
 *  Q      DEVICE int32[n]: the pivot columns Q[0, r), then Q[i] = i.
 *  rank   DEVICE int32: r.
 * Asynchronous; graph-capturable.  The result equals gf2_rref of gf2_pls of A
 * (the reduced row echelon form is unique).
 */
size_t gf2_m4ri_workspace_bytes(int64_t m, int64_t n);
int gf2_m4ri(gf2_ctx *ctx, gf2_mat A, int32_t *Q, int32_t *rank, const gf2_sched *s, void *ws,
             size_t ws_bytes, void *stream);

/*
 * The "M+P" hybrid of Section 6: M4RI strips while the approximated density of
 * the part left to eliminate (rows without a pivot, columns from the next strip
 * on) stays below `threshold` (the paper uses 0.15 and 0.20), then PLS
 * (Sections 4-5, the schedule's cutoff and Schur product) and the RREF from it
 * on that part, and finally the rows above it reduced by the part's RREF rows
 * (one product).  The density is estimated from up to 256 rows spread evenly
 * over the remaining rows, before every strip.
 *  A, Q, rank   as gf2_m4ri (A receives its RREF).
 *  switch_panel HOST int32 (nullable): the strip at which PLS took over, or -1
 *               when M4RI finished alone.
 * Threshold 0 runs PLS + RREF only; a threshold above 1 runs M4RI only.
 * Synchronous: the call reads each density estimate back to choose the kernels
 * that follow, so it waits on `stream` and cannot be captured in a graph.
 */
size_t gf2_rref_mp_workspace_bytes(int64_t m, int64_t n, const gf2_sched *s);
int gf2_rref_mp(gf2_ctx *ctx, gf2_mat A, int32_t *Q, int32_t *rank, float threshold,
                int32_t *switch_panel, const gf2_sched *s, void *ws, size_t ws_bytes,
                void *stream);

/*
 * Linear systems from a PLS (the decomposition as the building block for
 * solving systems of linear equations: abstract and Section 1).  With P A = L S,
 * A X = B becomes L S X = P B: Y = P B, forward substitution with L's unit lower
 * r x r triangle on Y's first r rows, a consistency test on the remaining rows
 * (Y_bottom = L_bottom Y_top), and back substitution with U_Q = S[:, Q].
 *  A_pls, P, Q, rank  gf2_pls outputs (device; only read).
 *  B      m x nrhs (device): column t is right-hand side t, so row i of B holds
 *         equation i's entries of every right-hand side.  Only read.
 *  X_out  n x nrhs (device): column t is a solution of A x = B[:, t] whose
 *         non-pivot entries (columns not in Q[0, r)) are zero, when one exists.
 *  bad    DEVICE uint64[ceil(nrhs / 64)]: bit t set when system t has no
 *         solution (X_out's column t is then not a solution).
 *  s      only the schur field is read (the substitutions' products).
 * Asynchronous, rank read on the device; graph-capturable.  The transposition
 * vector is turned into a row map on the device each call.
 */
size_t gf2_solve_workspace_bytes(int64_t m, int64_t n, int64_t nrhs);
int gf2_solve(gf2_ctx *ctx, gf2_mat A_pls, const int32_t *P, const int32_t *Q,
              const int32_t *rank, gf2_mat B, gf2_mat X_out, uint64_t *bad,
              const gf2_sched *s, void *ws, size_t ws_bytes, void *stream);

/*
 * Basis of the null space {x : A x = 0} from a PLS (A x = 0 exactly when
 * S x = 0, since P and L are injective on the rows that matter).  One basis
 * vector per non-pivot column f, in increasing order of f: x[f] = 1, the other
 * non-pivot entries 0, x[Q] = U_Q^{-1} S[:, f] -- the non-pivot columns of the
 * reduced row echelon form, transposed.
 *  A_pls, Q, rank  gf2_pls outputs (device; only read).
 *  K_out  n x n (device, its own buffer): rows [0, n - r) receive the basis
 *         vectors as packed rows, rows [n - r, n) are zeroed.
 *  s      only the schur field is read.
 * Asynchronous, rank read on the device; graph-capturable.
 */
size_t gf2_kernel_basis_workspace_bytes(int64_t m, int64_t n);
int gf2_kernel_basis(gf2_ctx *ctx, gf2_mat A_pls, const int32_t *Q, const int32_t *rank,
                     gf2_mat K_out, const gf2_sched *s, void *ws, size_t ws_bytes, void *stream);

/*
 * Batched PLS: `count` independent matrices of any shapes up to
 * GF2_BATCH_MAX_M x GF2_BATCH_MAX_N, each decomposed in place exactly as
 * gf2_pls does (the result of Gaussian PLS, Appendix A).  One persistent launch
 * serves them all: a block of the device takes one matrix at a time, largest
 * estimated cost first, and runs the MMPF base case of Section 4.1 over all of
 * its columns (so a schedule's cutoff and schur fields are ignored here).
 *  items     DEVICE array of count descriptors; every words/P/Q pointer is device
 *            memory; matrices must not overlap each other or any P/Q array.
 *  ranks     DEVICE int32[count]: the rank of item j, or GF2_E_ARG (negative) if
 *            item j is invalid (size out of range, stride too small, null or
 *            misaligned pointer); an invalid item's buffers are not touched.
 *  per_item  DEVICE gf2_sched[count] or NULL: k and tables of item j; an entry
 *            with k or tables out of range falls back to `s`.
 *  s         HOST schedule for every item without its own (NULL: default).
 * The call enqueues a fixed sequence of kernels and allocates nothing, so it can
 * be captured into a HIP graph and replayed (inputs restored between replays).
 */
#define GF2_BATCH_MAX_N 4096
#define GF2_BATCH_MAX_M (1 << 24)

typedef struct gf2_batch_item {
    uint64_t *words;
    int64_t m, n;
    int64_t stride;
    int32_t *P;
    int32_t *Q;
} gf2_batch_item;

size_t gf2_pls_batched_workspace_bytes(int64_t count);
int gf2_pls_batched(gf2_ctx *ctx, const gf2_batch_item *items, int64_t count, int32_t *ranks,
                    const gf2_sched *per_item, const gf2_sched *s, void *ws, size_t ws_bytes,
                    void *stream);

/*
 * Autotuner (schedules only; a schedule never changes a result bit).
 * gf2_sched_candidates: the deduplicated candidate schedules for an m x n
 *   problem: k in 4..8 x tables in {1,2,4,8} x cutoff in {256,512,1024,2048,4096}
 *   x schur in {XOR, MFMA, FP4}, where all cutoffs at or above the padded width
 *   collapse into one MMPF-only candidate (no Schur product is formed); with
 *   batched != 0, k x tables only (the batched call ignores cutoff and schur).
 *   Writes up to max entries (host array) and returns the total count, or a
 *   negative status.
 * gf2_autotune: runs gf2_pls once per repetition for every candidate on
 *   A_work after copying the pristine A_trial into it (same m, n; A_trial is only
 *   read), times each run with HIP events on `stream` and waits for them.
 *   ms_out[i] (host) receives candidate i's fastest time and *best the fastest
 *   candidate (the default schedule when ncand == 0).  The workspace must hold
 *   gf2_autotune_workspace_bytes(m, n, cands, ncand) bytes (256-byte aligned).
 * gf2_autotune_batched: the same for gf2_pls_batched on a batch of trial items
 *   (device descriptors `trial`, copied into the same-shaped `work` items before
 *   each run; ranks is a device int32[count]); workspace as gf2_pls_batched.
 * Not graph-capturable (the calls wait for their events).
 */
int gf2_sched_candidates(int64_t m, int64_t n, int batched, gf2_sched *out, int max);
size_t gf2_autotune_workspace_bytes(int64_t m, int64_t n, const gf2_sched *cands, int ncand);
int gf2_autotune(gf2_ctx *ctx, gf2_mat A_trial, gf2_mat A_work, const gf2_sched *cands, int ncand,
                 int reps, float *ms_out, gf2_sched *best, void *ws, size_t ws_bytes, void *stream);
int gf2_autotune_batched(gf2_ctx *ctx, const gf2_batch_item *trial, const gf2_batch_item *work,
                         int64_t count, int32_t *ranks, const gf2_sched *cands, int ncand, int reps,
                         float *ms_out, gf2_sched *best, void *ws, size_t ws_bytes, void *stream);

/*
 * Learned cost model: an fp32 network 4 -> 64 -> 64 -> S (ReLU) predicting the
 * log run time of each of S candidate schedules from a problem's features; the
 * predicted schedule is the argmin (the field-operation count alone mispredicts
 * run time, Section 1).  It only chooses schedules and never touches the
 * arithmetic.
 *  params  DEVICE fp32[gf2_mlp_param_count(S)]: W1[4][64] b1[64] W2[64][64]
 *          b2[64] W3[64][S] b3[S], W[a][j] from input a to output j.
 *  feats   DEVICE fp32[N][4] raw features: log2 m, log2 n, density, rank
 *          estimate / min(m, n); the network scales them to (f0/16, f1/16, f2, f3).
 * gf2_mlp_init: uniform(-sqrt(6/fan_in), +sqrt(6/fan_in)) weights from SplitMix64
 *   draws at the parameter index, zero biases.
 * gf2_mlp_forward: out (DEVICE fp32[N][S]) = predicted log times.
 * gf2_mlp_grad: loss = inv_count * sum of mask[i][s] (out[i][s] - target[i][s])^2
 *   over DEVICE fp32[N][S] target and mask; grad (DEVICE fp32[P + 1]) receives
 *   d loss / d params, then the loss.  Sums run in a fixed order (deterministic).
 *   Workspace: gf2_mlp_grad_workspace_bytes(S, N).
 * gf2_mlp_adam: one Adam step (Kingma & Ba) on params with first/second moment
 *   arrays m1, m2 (DEVICE fp32[P], zero before step 1), step >= 1.
 * gf2_costmodel_predict: out[i] (DEVICE gf2_sched[N]) = table[argmin_s out_s]
 *   with table a DEVICE gf2_sched[S] (the schedules the S outputs stand for).
 */
#define GF2_MLP_MAX_S 256

typedef struct gf2_mlp {
    float *params;
    int32_t S;
} gf2_mlp;

int64_t gf2_mlp_param_count(int S);
int gf2_mlp_init(gf2_ctx *ctx, gf2_mlp net, uint64_t seed, void *stream);
int gf2_mlp_forward(gf2_ctx *ctx, gf2_mlp net, const float *feats, int64_t N, float *out,
                    void *stream);
size_t gf2_mlp_grad_workspace_bytes(int S, int64_t N);
int gf2_mlp_grad(gf2_ctx *ctx, gf2_mlp net, const float *feats, const float *target,
                 const float *mask, int64_t N, float inv_count, float *grad, void *ws,
                 size_t ws_bytes, void *stream);
int gf2_mlp_adam(gf2_ctx *ctx, gf2_mlp net, const float *grad, float *m1, float *m2, float lr,
                 float beta1, float beta2, float eps, int step, void *stream);
int gf2_costmodel_predict(gf2_ctx *ctx, gf2_mlp net, const float *feats, int64_t N,
                          const gf2_sched *table, gf2_sched *out, void *stream);

/*
 * Features for the cost model computed on the device from the matrices
 * themselves: feats[i] = (log2 m, log2 n, density, r_est / min(m, n)) of item i
 * (DEVICE descriptors as for gf2_pls_batched; P and Q are not used).  The
 * density counts the ones of up to 256 rows spread evenly over the matrix; the
 * rank estimate r_est is r_hint[i] when r_hint (DEVICE int32[count], nullable)
 * holds a positive value, else min(m, n).  An invalid item gets zeros.
 */
int gf2_features(gf2_ctx *ctx, const gf2_batch_item *items, int64_t count,
                 const int32_t *r_hint, float *feats, void *stream);

/*
 * The learned schedule choice for gf2_pls / gf2_pls_noalloc calls with s == NULL.
 * The network (parameters and its DEVICE schedule table, as for
 * gf2_costmodel_predict) is evaluated once, now, on the device, for every cell
 * of a grid of shapes with log2 m and log2 n in [log2_lo, log2_hi] in steps of
 * 1/2 (at most GF2_LEARNED_MAX_CELLS per side), taking the features of a dense
 * full-rank input (density 1/2, rank estimate min(m, n)), since a call's
 * density is not known before it runs.  The argmins are kept in the context;
 * a call without a schedule takes the cell nearest to its (log2 m, log2 n), and
 * the default schedule for shapes more than a quarter step outside the grid or
 * with log2 m + log2 n above log2_mn_hi (outside the training range: the shapes
 * the network was trained on).  net.params == NULL removes the choice.
 * Waits on `stream` (the choice is read back).  The workspace holds
 * gf2_ctx_set_learned_workspace_bytes() bytes.
 * gf2_ctx_learned_sched: the schedule a call without one would use for m x n;
 * returns 1 when it is the learned choice, 0 for the default.
 */
#define GF2_LEARNED_MAX_CELLS 64
size_t gf2_ctx_set_learned_workspace_bytes(void);
int gf2_ctx_set_learned(gf2_ctx *ctx, gf2_mlp net, const gf2_sched *table, float log2_lo,
                        float log2_hi, float log2_mn_hi, void *ws, size_t ws_bytes,
                        void *stream);
int gf2_ctx_learned_sched(gf2_ctx *ctx, int64_t m, int64_t n, gf2_sched *out);

/* Workspace bytes gf2_addmul needs for C (m x n) += A (m x k) * B (k x n). */
size_t gf2_addmul_workspace_bytes(int64_t m, int64_t k, int64_t n);

/*
 * GF(2) matrix product accumulate C <- C + A * B, the Schur-complement update
 * of Section 5 (A_SE <- A_SE + A_SW * A_NE), exposed for direct use and tests.
 * A is m x k, B is k x n, C is m x n, all device matrices with their own
 * strides; C must not overlap A or B.  `variant` is GF2_SCHUR_XOR,
 * GF2_SCHUR_MFMA or GF2_SCHUR_FP4; all give identical bits; any other value
 * returns GF2_E_ARG.
 */
int gf2_addmul(gf2_ctx *ctx, gf2_mat C, gf2_mat A, gf2_mat B, int variant,
               void *ws, size_t ws_bytes, void *stream);

/*
 * Launch timing of the Schur-product kernels (diagnostics for roofline reports).
 * gf2_prof_enable: dev_log is a caller-owned DEVICE array of 3 * log_slots int32
 * (NULL disables).  While enabled, each product launch of gf2_pls / gf2_rref is
 * bracketed by HIP events on its stream and writes its row count M, inner
 * dimension K and column count N to the log (up to log_slots launches).
 * gf2_prof_read: waits for the recorded events, returns the launch count, the
 * summed event time and the summed algorithmic operations 2*M*N*K (one AND and
 * one XOR per bit product), then clears the record.
 */
typedef struct gf2_prof_stats {
    int64_t launches;
    double total_ms;
    double total_ops;
} gf2_prof_stats;

typedef struct gf2_prof_launch {
    double ms;
    int64_t m, n, k;
} gf2_prof_launch;

int gf2_prof_enable(gf2_ctx *ctx, int32_t *dev_log, int64_t log_slots);
int gf2_prof_read(gf2_ctx *ctx, gf2_prof_stats *out);
/* The recorded launches one by one (up to max, in launch order) without clearing
 * them; *count receives the number written.  Call before gf2_prof_read. */
int gf2_prof_read_launches(gf2_ctx *ctx, gf2_prof_launch *out, int64_t max, int64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* GF2PLS_H */

/*
 * pod.h -- C ABI of the MI355X (gfx950) implementation of the iterative
 * sample-and-merge POD (ISMA) of Charumathi, Ramakrishna & Vasudevan,
 * arXiv 1905.05107.
 *
 * Conventions for every entry point
 *  - The snapshot matrix A is m x n, column-major (snapshot j is contiguous),
 *    leading dimension lda >= m, stored as FP64 or FP32 in device memory.
 *  - Device pointers are plain HIP device addresses; "host" buffers are
 *    ordinary CPU memory.  The library never takes ownership of a caller
 *    buffer.  The caller keeps A alive and unmodified (except through
 *    center_rows) until pod_destroy.
 *  - All work is enqueued on the stream given to pod_init (a hipStream_t
 *    passed as void*, NULL = the default stream) in call order.  Entry
 *    points that return data to host memory synchronise that stream; they
 *    are marked "syncs".
 *  - Every entry point returns a pod_status; nothing throws across the ABI.
 *    After POD_EHIP the context must be destroyed.
 */
#ifndef POD_H
#define POD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pod_ctx pod_ctx;

typedef enum {
    POD_OK = 0,
    POD_EINVAL = 1,     /* bad argument or parameter combination            */
    POD_ENOMEM = 2,     /* device or host allocation failed                 */
    POD_EHIP = 3,       /* a HIP runtime call failed                        */
    POD_ENOTPD = 4,     /* Cholesky breakdown even after the shifted retry  */
    POD_ESTATE = 5,     /* call out of order (e.g. merge before sample)     */
    POD_EXHAUSTED = 6,  /* no column of S left to draw: normal stop         */
    POD_ENONFINITE = 7, /* NaN/Inf met in A or in a computed quantity       */
    POD_ENOCONV = 8     /* a Jacobi SVD did not converge in its sweep limit */
} pod_status;

/* Arithmetic of the merge / projection GEMMs.  The Cholesky factors and the
 * small SVDs are FP64 in every path.
 *   POD_F64          FP64 matrix cores, FP64 basis.
 *   POD_F32          FP32 matrix cores, FP32 basis (A stored FP32).
 *   POD_BF16_REFINE  the merge's m-pass products (both CholeskyQR Grams,
 *                    Q1 = X0 T1, U_new = Q1 Z2) on BF16 matrix cores with a
 *                    three-term split of every FP32 operand and FP32
 *                    accumulation (FP32-accurate: the span of the merge is not
 *                    moved by BF16 rounding); the final projection and
 *                    Rayleigh-Ritz rotation in FP32.  A stored FP32; single
 *                    runs and Alg. 3 only (the batch rejects it). */
typedef enum { POD_F64 = 0, POD_F32 = 1, POD_BF16_REFINE = 2 } pod_precision;

/* Column sampling from the second iteration on (first iteration: always
 * column-norm probabilities, Eq. LTSVD_prob):
 *   POD_COL_L2N  squared column norms over S;
 *   POD_COL_UNF  uniform over S;
 *   POD_COL_ORT  squared residuals |a_j - U U^T a_j|^2 of the columns of S
 *                against the current merged basis (Sec. "Column sampling"
 *                (c)), formed as nu_j - |U^T a_j|^2 from one pass over A per
 *                iteration (FP64 sums); residuals at or below 1e-12 nu_j
 *                (FP64 basis) or 16 u_32 nu_j (FP32 basis) count as zero.
 *                Single runs and Alg. 3 (the batch rejects it). */
typedef enum { POD_COL_L2N = 0, POD_COL_UNF = 1, POD_COL_ORT = 2 } pod_col_strategy;

/* Row sampling when w > 0: squared row norms of the sampled columns
 * (Eq. CTSVD_prob) or leverage scores of the current modes (second
 * iteration on). */
typedef enum { POD_ROW_L2 = 0, POD_ROW_LS = 1 } pod_row_strategy;

/* Convergence test of Alg. 1: principal angles between the subspaces of
 * successive estimates, or angles between corresponding modes. */
typedef enum { POD_CRIT_SUBSPACE = 0, POD_CRIT_MODE = 1 } pod_criterion;

/* Inputs of ISMA(A, p, k, c, w, r, tau, rows) (Alg. 1). */
typedef struct {
    int64_t m, n, lda;     /* A is m x n column-major, lda >= m                 */
    int32_t a_dtype;       /* storage of A: POD_F64 or POD_F32                  */
    int32_t precision;     /* pod_precision                                     */
    int32_t k;             /* modes reported                                    */
    int32_t r;             /* rank kept after each merge (0 -> k), r >= k       */
    int32_t c;             /* column draws per iteration (with replacement)     */
    int32_t w;             /* row draws per iteration, 0..1024; 0 = columns    */
                           /* only (ICS).  w > 0 (ICRS): the merge takes        */
                           /* C = D V~(:, 0:r_u), V~ the right singular vectors */
                           /* of the scaled row sample W, r_u = min(r, g, h,    */
                           /* rank W)                                           */
    int32_t r_update;      /* w = 0 only: >0 keeps the top r_update right      */
                           /* singular directions of each new block D before    */
                           /* the merge (C = D V(:, 0:r_update)); 0 merges D    */
    int32_t col_strategy;  /* pod_col_strategy                                  */
    int32_t row_strategy;  /* pod_row_strategy                                  */
    int32_t criterion;     /* pod_criterion                                     */
    int32_t center_rows;   /* 1: subtract row means of A in place at init       */
    int32_t max_iter;      /* merges allowed (>= 1)                             */
    double theta_tol;      /* stop when the largest angle < theta_tol (radians) */
    uint64_t seed;         /* Philox key word 0                                 */
    uint64_t block;        /* Philox counter word 2 (column block of Alg. 3)    */
} pod_params;

/* Why a run of Alg. 1 stops (pod_info.stop_reason): the stop rule of
 * pod_converged evaluated on the current state, in this priority order. */
typedef enum {
    POD_STOP_NONE = 0,       /* no rule holds: more merges can follow          */
    POD_STOP_NONFINITE = 1,  /* a NaN/Inf was met (POD_ENONFINITE)             */
    POD_STOP_CONVERGED = 2,  /* from the second merge on, the largest angle     */
                             /* between successive estimates is below theta_tol */
    POD_STOP_EXHAUSTED = 3,  /* S has no drawable column left                   */
    POD_STOP_MAX_ITER = 4,   /* max_iter merges were done                       */
    POD_STOP_BREAKDOWN = 5   /* a Cholesky of the merge broke down even after   */
                             /* the shifted retry (POD_ENOTPD); ranked after     */
                             /* POD_STOP_NONFINITE                               */
} pod_stop_reason;

/* Host-readable progress of a context (pod_get_info, syncs). */
typedef struct {
    int32_t iter;          /* merges done                                       */
    int32_t rank;          /* columns of the current basis U                    */
    int32_t g;             /* distinct columns of the last draw                 */
    int32_t h;             /* distinct rows of the last draw                    */
    int32_t exhausted;     /* S had no drawable column at the last pod_sample   */
    int32_t flags;         /* bit 0: shifted Cholesky used; bit 1: non-finite;  */
                           /* bit 2: sweep limit hit; bit 3: all row weights    */
                           /* zero; bit 4: Cholesky breakdown after the shift   */
    int32_t max_sweeps;    /* most Jacobi sweeps of any merge so far            */
    int32_t total_sweeps;  /* Jacobi sweeps summed over the merges              */
    double sin_theta;      /* sine of the last convergence angle (NaN first)    */
    int32_t stop_reason;   /* pod_stop_reason of the current state              */
    int32_t reserved;      /* 0                                                 */
} pod_info;

/* Create a context for A (device, borrowed) and run the set-up pass:
 * optional row centring (two passes over A), the column squared norms
 * (Eq. LTSVD_prob, one pass, FP64 in a fixed summation order) and their
 * integer sampling weights.  Errors: POD_EINVAL for bad sizes or options,
 * POD_ENOMEM, POD_EHIP. */
pod_status pod_init(pod_ctx **ctx, const pod_params *prm, void *A_dev, void *stream);

/* GET UPDATE of Alg. 1: draw c columns from S with the current probabilities
 * (Philox-4x64-10, key (seed, 0), counter (iter, d/4, block, 0)), keep the
 * distinct ones in ascending order, remove them from S, and, when w > 0,
 * SAMPLE AND SCALE UNIQUE ROWS (key (seed, 1)) followed by the small SVD of
 * W^T W.  g_out / h_out (host, nullable) receive the numbers of distinct
 * columns / rows: passing them syncs.  POD_EXHAUSTED (syncs) when S has no
 * drawable column; the context then stays valid for pod_project. */
pod_status pod_sample(pod_ctx *ctx, int32_t *g_out, int32_t *h_out);

/* BLOCK MERGE of Alg. 2 on [U_r Sigma_r | C]: CholeskyQR2 of the tall
 * block, FP64 SVD of the (r+g) x (r+g) factor, rank guard, truncation to r.
 * POD_ESTATE if no sample is pending. */
pod_status pod_merge(pod_ctx *ctx);

/* Convergence test of Alg. 1 (syncs): *done = 1 when the largest angle
 * between the first k modes of the last two estimates is below theta_tol,
 * S is exhausted, max_iter merges were done, or the run failed.
 * *sin_theta_max (nullable) gets the sine of that angle (NaN after the first
 * merge).  Returns POD_ENONFINITE after a NaN/Inf in A or a computed
 * quantity, POD_ENOTPD after a Cholesky breakdown that the shifted retry did
 * not cure (e.g. a merge block whose Gram is zero); *done is 1 then. */
pod_status pod_converged(pod_ctx *ctx, int32_t *done, double *sin_theta_max);

/* The loop of Alg. 1 driven from the device: enqueue iterations (pod_sample
 * + pod_merge + the stop test of pod_converged, evaluated by a kernel that
 * sets a stop flag on which every later kernel of the loop returns at once)
 * `chunk` at a time (<= 0: 8) and sync once per chunk, until the run stops
 * or max_merges merges were done.  stop_on_converged = 0 ignores the angle
 * test (a fixed number of merges; S exhaustion and max_iter still stop).
 * Results are those of the host loop sample / merge / converged.
 * sin_out (host, nullable, >= max_merges doubles) receives the convergence
 * sine of each merge of this call (NaN for the first merge of the run);
 * *merges_out (nullable) the number of merges done; *done_out (nullable) 1
 * when the run stopped (converged, S exhausted, max_iter reached, or a
 * failure: the status is then that of pod_converged).  No sample may be
 * pending (POD_ESTATE); the context is left ready for pod_sample /
 * pod_project.  Syncs. */
pod_status pod_run(pod_ctx *ctx, int32_t max_merges, int32_t stop_on_converged, int32_t chunk, double *sin_out,
                   int32_t *merges_out, int32_t *done_out);

/* Final step of Alg. 1 (syncs): B = U_r^T A (one pass over A), SVD of B,
 * U <- U U_B, Sigma <- Sigma_B, V = B^T U_B Sigma_B^-1.  Writes the first
 * k modes: U_out (device, m x k column-major, FP64 for POD_F64 else FP32),
 * sigma_out (device, k FP64), V_out (device, n x k like U_out, nullable).
 * Each u_i is signed so that its largest-magnitude entry is positive. */
pod_status pod_project(pod_ctx *ctx, void *U_out, double *sigma_out, void *V_out);

/* Quality measure of the converged modes (Sec. "Quality of converged
 * solution", Eq. ang_meas): with the k pairs (U_k, Sigma_k, V_k) that the last
 * pod_project wrote (U_k device m x k, V_k device n x k, both column-major in
 * the compute type: FP64 for POD_F64 else FP32; Sigma_k and sigma_{k+1} are
 * the Rayleigh-Ritz values the context keeps),
 *   R = A V_k - U_k Sigma_k,  S = A^T U_k - V_k Sigma_k,
 *   out[0] = ||R||_F, out[1] = ||S||_F,
 *   out[2] = omega^ = min(|sigma_k - sigma_{k+1}|, sigma_k),
 *   out[3] = sqrt(out[0]^2 + out[1]^2) / omega^ (+inf when omega^ = 0),
 * Wedin's bound on the sines of the principal angles between the exact and
 * the computed dominant subspaces (out: host, 4 doubles).  Two passes over A,
 * FP64 accumulation, fixed summation order.  The first call allocates a
 * workspace (m k + k n doubles and partials) that the context keeps.
 * POD_ESTATE unless pod_project ran after the last merge; POD_EINVAL when the
 * rank r is not above k (sigma_{k+1} is needed) or k > 64.  Syncs. */
pod_status pod_wedin_bound(pod_ctx *ctx, const void *U_k, const void *V_k, double *out);

/* Copy the current merged basis (before the final step) to caller device
 * buffers: U_out m x rank (ld = m, precision as in pod_project) and
 * sigma_out (device, rank FP64); *rank_out (host) gets the rank.  Syncs. */
pod_status pod_get_basis(pod_ctx *ctx, void *U_out, double *sigma_out, int32_t *rank_out);

/* Progress counters (syncs). */
pod_status pod_get_info(pod_ctx *ctx, pod_info *info);

/* Indices drawn at merge `iter` (0-based), copied to host buffers of at
 * least c (cols, col_counts) and w (rows, row_counts) entries; any pointer
 * may be NULL.  *g / *h (host, nullable) get their numbers.  Syncs. */
pod_status pod_get_indices(pod_ctx *ctx, int32_t iter, int32_t *cols, int32_t *col_counts, int32_t *g,
                           int32_t *rows, int32_t *row_counts, int32_t *h);

/* Replay of a draw (parity checks against a reference run, finite
 * differences with frozen indices): the next pod_sample (or the first draw of
 * the next pod_run), which is the draw of merge `iter` (iter must equal the
 * merges done), takes these indices instead of drawing from the Philox
 * stream.  GET UPDATE of Alg. 1 then continues as after a draw: the columns
 * leave S, the column log records them, and with w > 0 SAMPLE AND SCALE
 * UNIQUE ROWS scales the given rows by sqrt(t^_i / (w q_i)), q_i from the
 * current row weights (Eq. CTSVD_prob, or leverage scores), followed by the
 * small SVD of W^T W.
 *   cols (host): g >= 1 distinct columns of S in ascending order, g <= c;
 *   col_counts (host, nullable = all 1): their multiplicities (>= 1, logged);
 *   rows, row_counts (host; required when w > 0, ignored otherwise): h >= 1
 *   distinct rows in ascending order, h <= w, multiplicities >= 1 summing to w.
 * A row whose current weight is zero makes the scale infinite: the merge then
 * reports POD_ENONFINITE.  POD_EINVAL for indices out of range, unsorted,
 * repeated or (columns) no longer in S; POD_ESTATE while a draw is pending or
 * when iter is not the next merge.  Syncs. */
pod_status pod_set_indices(pod_ctx *ctx, int32_t iter, const int32_t *cols, const int32_t *col_counts, int32_t g,
                           const int32_t *rows, const int32_t *row_counts, int32_t h);

/* ---------------------------------------------------------------------------
 * Reverse mode through the merge chain of Alg. 1 (ICS with merge widths up to
 * 160 and p + r <= 208; ICRS with rows, w > 0, merge width <= 64; r_update =
 * 0).  Outputs differentiated: the first
 * k merged modes and singular values (U_k, Sigma_k) as pod_get_basis returns
 * them (before the final step); the sampled columns and rows and the row
 * scales are constants (draws and quantised weights are piecewise constant in
 * A).  A row-sampled merge runs on [U Sigma | D V_u], V_u the leading r_u
 * eigenvectors of W^T W, W = diag(s) D(rows, :) (Alg. 1, GET UPDATE with
 * rows); its adjoint adds the eigenvector term
 * dA(rows, cols) += 2 diag(s)^2 A(rows, cols) G-bar, G-bar = sym(V K V^T),
 * K_ij = v_i^T Vbar_j d / (d^2 + eta^2 lambda_1^2), d = lambda_j - lambda_i
 * (j < r_u, i != j) over the full eigenbasis of W^T W.  Each merge's truncated thin SVD is differentiated with the
 * coupling F_ij = d / (d^2 + eta^2 s_1^4), d = s_j^2 - s_i^2 (eta = 1e-12 for
 * POD_F64, 1e-6 otherwise; F_ij = 1/(s_j^2 - s_i^2) when |d| >> eta s_1^2)
 * (Townsend 2016; Ionescu, Vantzos & Sminchisescu 2015).
 * ------------------------------------------------------------------------- */

/* Keep what the reverse pass needs: per merge the starting basis (m x r) and
 * Sigma, and the p x p merge factor.  Call after pod_init, before the first
 * pod_sample; with rows also V_u, the rows and the row scales of each merge.
 * POD_EINVAL for truncated blocks (r_update > 0), for row draws with a merge
 * width above 64, or when the merge width plus r exceeds 208 (the Gram of
 * [U | A(:, I) | Ubar] of a reverse step); POD_ESTATE after a draw. */
pod_status pod_enable_adjoint(pod_ctx *ctx);

/* dA (device, m x n, ld m, compute type) += d<dU, U_k> + <dsigma, Sigma_k> / dA
 * for dU (device, m x k, ld m, compute type; nullable) and dsigma (device, k
 * FP64; nullable).  POD_ESTATE without pod_enable_adjoint or before a merge.
 * Syncs. */
pod_status pod_backward(pod_ctx *ctx, const void *dU, const double *dsigma, void *dA);

/* Loss L = |A - U_k U_k^T A|_F^2 of the merged modes and its gradient:
 * dA (device, m x n, ld m, compute type) is overwritten with dL/dA and
 * *loss (host, nullable) gets L.  Two passes over A plus two per merge.
 * POD_EINVAL when k exceeds 64.  Syncs. */
pod_status pod_loss_grad(pod_ctx *ctx, void *dA, double *loss);

/* ---------------------------------------------------------------------------
 * Alg. 3, incremental POD: ISMA on each column block (with its final step),
 * then BLOCK MERGE of the block's leading pairs [U_b Sigma_b] into the
 * running (U, Sigma), truncated to r.  One pass over the matrix.
 * ------------------------------------------------------------------------- */
typedef struct pod_inc pod_inc;

typedef struct {
    int32_t blocks;        /* blocks merged                                     */
    int64_t columns;       /* columns seen                                      */
    double host_bytes;     /* bytes copied from host blocks                     */
    double copy_ms;        /* summed host-to-device copy time of those blocks   */
    double wall_ms;        /* wall time of pod_inc_add_host_blocks calls        */
} pod_inc_info;

/* prm holds the ISMA parameters of every block; prm->n is the largest block
 * width, prm->lda and prm->block are ignored (block b, counted from 0 in the
 * order added, is the Philox counter word 2 of its draws) and center_rows
 * must be 0 (rows are centred over the whole matrix beforehand).  The merged
 * state keeps r = prm->r (or k) columns; r + r must be <= 160.  Errors:
 * POD_EINVAL, POD_ENOMEM, POD_EHIP. */
pod_status pod_inc_init(pod_inc **inc, const pod_params *prm, void *stream);

/* One block B (device, m x nb column-major, leading dimension ldb >= m,
 * borrowed for the duration of the call), nb <= prm->n.  Syncs. */
pod_status pod_inc_add_block(pod_inc *inc, const void *B_dev, int64_t nb, int64_t ldb);

/* `count` blocks in host memory (B_host[i]: m x nb[i], ld m, storage as
 * prm->a_dtype; pinned memory for the copies to run asynchronously).  The
 * library copies them through two device buffers on a side stream, the copy
 * of block i+1 overlapping the ISMA of block i.  Syncs. */
pod_status pod_inc_add_host_blocks(pod_inc *inc, const void *const *B_host, const int64_t *nb, int32_t count);

/* First k (<= rank) modes of the merged state: U_out (device, m x k, compute
 * type, signed as in pod_project; nullable), sigma_out (device, k FP64;
 * nullable), *k_out (host, nullable).  POD_ESTATE before any block.  Syncs. */
pod_status pod_inc_result(pod_inc *inc, void *U_out, double *sigma_out, int32_t *k_out);

/* Counters of the streamed blocks (host). */
pod_status pod_inc_get_info(pod_inc *inc, pod_inc_info *info);

void pod_inc_destroy(pod_inc *inc);

/* ---------------------------------------------------------------------------
 * Batched ISMA: `count` independent runs of Alg. 1 on matrices of uneven m, n
 * and k (for the callers that need many small decompositions at once).
 * Every iteration launches each kernel once for the whole batch; from the
 * second iteration the launch sequence is replayed from a captured HIP graph.
 * ------------------------------------------------------------------------- */
typedef struct pod_batch pod_batch;

/* prm[i], A[i] (device, borrowed) as for pod_init, for i < count.  Rows are
 * not sampled (w = 0, r_update = 0), the precision is the same for all, and
 * every merge width r + min(c, n) must round up to <= 64.  The set-up pass
 * (norms, weights) runs here.  The batch owns an internal stream.  Errors:
 * POD_EINVAL, POD_ENOMEM, POD_EHIP. */
pod_status pod_batch_init(pod_batch **b, int32_t count, const pod_params *prm, void *const *A);

/* Measure, per (merge-width bucket of 16, floor(log2 m), compute type) present
 * in the batch, the row-block count of the Gram passes (256 to 4096 rows per
 * workgroup) on the batch's own buffers and use the fastest.  Call before
 * pod_batch_run; *table_entries (nullable) gets the number of buckets. */
pod_status pod_batch_autotune(pod_batch *b, int32_t *table_entries);

/* Iterate until every matrix has stopped (the stop rule of pod_converged) or
 * max_rounds iterations; use_graph = 1 replays a captured HIP graph.
 * *rounds_out (nullable) gets the iterations run.  POD_ESTATE if some matrix
 * is still running after max_rounds.  Syncs. */
pod_status pod_batch_run(pod_batch *b, int32_t use_graph, int32_t max_rounds, int32_t *rounds_out);

/* Keep the reverse-pass checkpoints of every matrix (pod_enable_adjoint for
 * each; same restrictions); call before pod_batch_run. */
pod_status pod_batch_enable_adjoint(pod_batch *b);

/* pod_loss_grad for matrix i (dA device, m_i x n_i, ld m_i, compute type).
 * Syncs. */
pod_status pod_batch_loss_grad(pod_batch *b, int32_t i, void *dA, double *loss);

/* pod_batch_loss_grad for every matrix at once: dA[i] (device, m_i x n_i,
 * ld m_i, compute type; accumulated, so zero it first) receives dL_i/dA_i and
 * loss[i] (host, nullable) L_i.  The reverse steps of all matrices run
 * together (reverse step s takes the (T_i - s)-th merge of each matrix that
 * has one, in one launch per kernel); the gradients equal those of
 * pod_batch_loss_grad bit for bit.  Wider reverse steps (p + r > 64) fall
 * back to one matrix after another.  Same errors as pod_batch_loss_grad.
 * Syncs. */
pod_status pod_batch_loss_grad_all(pod_batch *b, void *const *dA, double *loss);

/* Final step of Alg. 1 for matrix i, as pod_project.  Syncs. */
pod_status pod_batch_project(pod_batch *b, int32_t i, void *U_out, double *sigma_out, void *V_out);

/* Progress of matrix i as pod_get_info; *gram_blocks (nullable) gets its
 * row-block count from the tile table.  Syncs. */
pod_status pod_batch_get_info(pod_batch *b, int32_t i, pod_info *info, int32_t *gram_blocks);

void pod_batch_destroy(pod_batch *b);

/* Column squared norms computed at init (device -> host, n FP64).  Syncs. */
pod_status pod_get_col_sqnorms(pod_ctx *ctx, double *nu_host);

/* Stand-alone column squared norms of an m x n device matrix in the
 * library's fixed summation order: nu_dev (device, n FP64).  Stream-ordered
 * on `stream`, no sync. */
pod_status pod_col_sqnorms(const void *A_dev, int32_t a_dtype, int64_t m, int64_t n, int64_t lda,
                           double *nu_dev, void *stream);

/* Row centring of an m x n device matrix in place (the snapshots are
 * mean-subtracted before the POD, Sec. 1): mean_i = (1/n) sum_j a_ij summed in
 * FP64 (rows along threads; the columns split into s = min(8, max(1,
 * ceil(2048 / ceil(m / 256)))) ranges whose sums are added in order), then
 * a_ij <- a_ij - mean_i rounded to the storage type.  What
 * pod_init does with center_rows = 1; Alg. 3 needs it over the whole matrix
 * before the blocks are streamed.  Allocates a scratch of s m doubles for the
 * call.  Syncs `stream`.  POD_EINVAL for bad sizes or types. */
pod_status pod_center_rows(void *A_dev, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, void *stream);

/* pod_center_rows for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and result bit for bit, with the scratch in a device
 * array of the library (2^23 doubles = 64 MiB per device, kept until the
 * process ends), so s m <= 2^23 (s as in pod_center_rows; m <= 4,194,304
 * rows), else POD_EINVAL.  Runs on the current device, which must own A and
 * `stream`.  Stream-ordered, no sync, no allocation.  The array is shared by
 * every call on a device: calls that overlap on one device (other streams or
 * threads) race. */
pod_status pod_center_rows_noalloc(void *A_dev, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, void *stream);

/* One-shot sampled SVDs of Appendix A, the methods the iteration builds on
 * (device, stream-ordered on `stream`, syncs):
 *   Alg. 4 (LTSVD, prm->w = 0): c draws over the columns of A with the norm
 *   probabilities of Eq. (LTSVD_prob) (Philox key (seed, 0), counter
 *   (0, d/4, block, 0): the first draw of pod_sample), folded into the g
 *   distinct columns, each scaled by sqrt(t_j / (c p_j)) (t_j draws, p_j its
 *   probability): C (m x g); V Sigma^2 V^T = eig(C^T C);
 *   l = min(k, #{lambda_i > g u lambda_1}); u_i = C v_i / sigma_i.
 *   Alg. 5 (CTSVD, prm->w > 0): as Alg. 4 for C, then w draws over the rows
 *   with q_i = |c^i|^2 / |C|_F^2 (Eq. CTSVD_prob_col; key (seed, 1)), folded
 *   into the h distinct rows, each scaled by sqrt(t_i / (w q_i)): W (h x g);
 *   V Sigma^2 V^T = eig(W^T W); gamma = eps / (100 k);
 *   l = min(k, max{r : sigma_r^2 >= gamma |W|_F^2}); u_i = C v_i / sigma_i
 *   (not orthonormal in general).
 * prm as for pod_init (m, n, lda, a_dtype, precision, k, c, w, seed, block,
 * center_rows; the merge width k + min(c, n) must be <= 160).  U_out (device,
 * m x k column-major, FP64 for POD_F64 else FP32; columns past l are zero,
 * each u_i signed as in pod_project), sigma_out (device, k FP64, zero past l),
 * *l_out (host, nullable).  POD_EXHAUSTED when no column (or, for Alg. 5, no
 * row) has a non-zero weight; POD_EINVAL for bad parameters or eps <= 0 with
 * w > 0. */
pod_status pod_oneshot(const pod_params *prm, const void *A_dev, double eps, void *U_out, double *sigma_out,
                       int32_t *l_out, void *stream);

/* Sample sizes of Eqs. (c_LTSVD) and (c_w_CTSVD), rounded up:
 * kind 0: c = 4k (1 + sqrt(8 ln(1/delta)))^2 / eps^2;
 * kind 1: c = w = k^2 (1 + sqrt(ln(2/delta)))^2 / eps^4.
 * Returns -1 for invalid arguments. */
int64_t pod_sample_size(int32_t kind, int32_t k, double eps, double delta);

/* Kernel classes for measurement (pod_profile_enable). */
typedef enum {
    POD_K_COLNORMS = 0,   /* column squared norms (one pass over A)          */
    POD_K_DRAW = 1,       /* weights + Philox draw + dedupe                  */
    POD_K_GRAM = 2,       /* partial Grams of the tall block (CholeskyQR)    */
    POD_K_GRAM_REDUCE = 3,/* fixed-order sum of the Gram partials            */
    POD_K_CHOL = 4,       /* FP64 Cholesky + triangular inverse (pass 1)     */
    POD_K_TALL = 5,       /* tall transform Y = X T                          */
    POD_K_SVD = 6,        /* pass-2 Cholesky + FP64 SVD of the merge factor  */
    POD_K_PROJECT = 7,    /* B = U^T A (one pass over A)                     */
    POD_K_RR = 8,         /* Rayleigh-Ritz small kernels                     */
    POD_K_SIGN = 9,       /* sign convention of the outputs                  */
    POD_K_COUNT = 10
} pod_kernel_class;

/* Measurement hook for benchmarks (process-wide, not thread-safe): while a
 * class is enabled, every launch of that class is bracketed by HIP events on
 * its launch stream.  pod_profile_read (syncs those events) returns the
 * number of launches and their summed event time in ms, then clears the
 * record.  kclass = -1 disables.  POD_EINVAL for an unknown class. */
pod_status pod_profile_enable(int32_t kclass);
pod_status pod_profile_read(int64_t *launches, double *total_ms);

/* Release everything the context owns (not A).  Syncs its stream. */
void pod_destroy(pod_ctx *ctx);

/* Static description of a status code. */
const char *pod_status_str(pod_status s);

#ifdef __cplusplus
}
#endif

#endif /* POD_H */

// pod_ctx.h -- the context behind the opaque pod_ctx handle of the C ABI and
// the library-internal calls shared by pod_api.hip and pod_incremental.hip.
#pragma once

#include "../../include/pod.h"
#include "pod_internal.h"

struct pod_ctx {
    int64_t n_cap = 0;       // columns the buffers were sized for
    pod_params prm;
    int32_t r = 0, pmax = 0;
    hipStream_t st = nullptr;
    void *A = nullptr;
    size_t esz = 8;          // bytes per element of the compute type
    pod::DevState *ds = nullptr;  // device
    pod::DevState hs{};           // host copy after the last sync
    double *nu = nullptr;
    uint64_t *wq = nullptr;
    uint8_t *inS = nullptr;
    int32_t *cols = nullptr, *ccnt = nullptr, *col_log = nullptr, *ccnt_log = nullptr, *col_log_off = nullptr;
    int32_t *forced = nullptr;
    double *rho = nullptr, *Vt = nullptr;  // row weights (m), right factor of the new block (pmax x pmax)
    double *rho_ort = nullptr;             // ORT column residuals (n)
    uint64_t *wort = nullptr;              // their integer weights (n)
    uint64_t *wr = nullptr;
    int32_t *rows = nullptr, *rcnt = nullptr, *row_log = nullptr, *rcnt_log = nullptr;
    void *U[2] = {nullptr, nullptr};
    double *sig[2] = {nullptr, nullptr};
    int cur = 0;
    double *part = nullptr, *G = nullptr, *R1 = nullptr, *R2 = nullptr, *work = nullptr;
    double *ws = nullptr;    // small-kernel matrices when pmax > 64
    void *Tc = nullptr, *Y = nullptr;
    void *tsplit = nullptr;   // POD_BF16_REFINE: split right factor of the tall transform
    int32_t nblk = 0;
    double *Bpart = nullptr, *B = nullptr, *GB = nullptr, *UB = nullptr, *sigB = nullptr;
    void *Zc = nullptr;
    double *signv = nullptr;
    int64_t *signi = nullptr;
    int32_t nsplit = 0;
    int pending = 0;         // a draw waits for its merge
    int32_t merges = 0;      // merges launched
    int exhausted = 0;       // known on the host
    int failed = 0;          // a HIP error happened: only destroy is allowed
    int32_t forced_g = -1;   // replay of the next draw: distinct columns (-1: draw)
    int32_t forced_h = 0;    // and distinct rows (w > 0); forced = [cols | counts | rows | counts], 1024 each
    double *sin_log = nullptr;   // device-driven runs: convergence sine of each merge
    int32_t log_cap = 0;
    // reverse pass (pod_enable_adjoint): per-merge checkpoints and buffers
    int32_t ck_cap = 0, pb = 0;
    int32_t ck_max = 0;      // merges a run can do: min(max_iter, n) + 1
    int ck_lost = 0;         // a checkpoint could not be grown: no reverse pass
    void *ckU = nullptr;     // basis before each merge (cap x m x r, compute type)
    double *ckS = nullptr;   // Sigma before each merge (cap x r)
    double *ckR = nullptr;   // merge factor R of each merge (cap x pmax^2)
    int32_t *ckMeta = nullptr;  // per merge: rs, g, rank after, valid
    // row-sampled merges (w > 0): the right factor V_u of the block (cap x pmax^2),
    // the row scales and the distinct rows (cap x w each) and (r_u, h) per merge (cap x 2)
    double *ckV = nullptr, *ckSc = nullptr;
    int32_t *ckRH = nullptr, *ckRows = nullptr;
    double *rscale = nullptr;    // scales of the last row draw (w), written by the block eigensolver
    double *adj_rows = nullptr;  // reverse pass of a row-sampled merge: full eigenbasis, eigenvalues, G-bar
    pod::DevState *dsb = nullptr;
    double *partb = nullptr, *Gext = nullptr, *adj_ws = nullptr, *sbar[2] = {nullptr, nullptr}, *lossp = nullptr;
    void *Wt = nullptr, *Ubar[2] = {nullptr, nullptr};
    // the last pod_project (merge count, pairs written, Rayleigh-Ritz rank)
    // and the workspace of pod_wedin_bound (allocated at its first call)
    int32_t proj_it = -1, proj_k = 0, proj_rank = 0;
    double *qws = nullptr;
    size_t qws_n = 0;
};

namespace pod {

// Validate `prm` (prm->n = the largest number of columns the context will
// see) and allocate every buffer; no access to A.
pod_status ctx_create(pod_ctx **out, const pod_params *prm, void *stream);
// Start a fresh ISMA run on A (m x n, n <= n_cap, leading dimension lda):
// reset the sampling state, optionally centre the rows, and compute the
// column norms and weights.  `block` is the Philox counter word 2.
pod_status ctx_bind(pod_ctx *ctx, void *A, int64_t n, int64_t lda, uint64_t block);
// Final step of Alg. 1 writing kout <= rank Rayleigh-Ritz pairs.
pod_status ctx_project(pod_ctx *ctx, void *U_out, double *sigma_out, void *V_out, int32_t kout);
// BLOCK MERGE of the context's state with an external basis:
// [U Sigma | Ub diag(sb)] (Ub m x rb in the compute type, ld m; sb device FP64),
// truncated to r.  The first call on an empty state takes (Ub, sb) as is.
pod_status ctx_merge_basis(pod_ctx *ctx, const void *Ub, const double *sb, int32_t rb);

// Checkpoints of the reverse pass around a merge (no-ops when the pending
// draw found S exhausted).
hipError_t launch_ckpt_pre(pod_ctx *ctx, hipStream_t st);
// Grow the per-merge checkpoints to at least `need` merges (capped at
// ck_max), keeping what they hold.  Syncs the context's stream when it grows.
// POD_ENOMEM leaves the context usable (the old checkpoints stay).
pod_status ckpt_reserve(pod_ctx *ctx, int32_t need);
hipError_t launch_ckpt_post(pod_ctx *ctx, hipStream_t st);
// row-sampled merges: V_u, the row scales, the rows and (r_u, h) of the merge about to run
hipError_t launch_ckpt_rows(pod_ctx *ctx, hipStream_t st);

// Batched checkpoints (per-matrix entries in device memory).
struct CkptArgs {
    const pod::DevState *ds;
    const void *U0, *U1;
    const double *s0, *s1;
    int64_t m;
    int32_t r, cap, pm2;
    void *ckU;
    double *ckS, *ckR;
    const double *R;
    int32_t *meta;
};
CkptArgs ctx_ckpt_args(pod_ctx *ctx);
hipError_t launch_ckpt_pre_b(const CkptArgs *arr, int32_t count, int64_t max_mr, int32_t prec, hipStream_t st);
hipError_t launch_ckpt_post_b(const CkptArgs *arr, int32_t count, hipStream_t st);

// Argument blocks of one context's launches (shared with the batched path).
DrawArgs ctx_draw_args(pod_ctx *ctx);
SmallArgs ctx_small_args(pod_ctx *ctx);
GemmDesc ctx_gather_desc(pod_ctx *ctx);
GemmDesc ctx_plain_desc(pod_ctx *ctx, const void *Y);

}  // namespace pod

// pod_api.hip -- the C ABI of include/pod.h: context ownership, argument
// checks and the order of kernel launches for one ISMA run (Alg. 1) on a
// single gfx950 GPU.  Every step of the method runs in the kernels of
// pod_sample.hip, pod_gemm.hip and pod_small.hip; this file only allocates,
// launches and copies results.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "pod_ctx.h"

using namespace pod;


namespace {

template <typename T> hipError_t dalloc(T **p, size_t count)
{
    return hipMalloc((void **)p, count * sizeof(T) + 16);
}

double unit_roundoff(int32_t prec) { return prec == POD_F64 ? 1.1102230246251565e-16 : 5.9604644775390625e-08; }

// ORT residuals nu_j - |U^T a_j|^2 at or below this fraction of nu_j count as
// zero: the column lies in the current subspace to the accuracy of the basis
// (FP64: the oracle's 1e-12; FP32 bases: 16 u_32, the size of the cancellation)
double ort_floor(int32_t prec) { return prec == POD_F64 ? 1e-12 : 16.0 * 5.9604644775390625e-08; }

#define POD_HIP(call)                                                                                                 \
    do {                                                                                                              \
        hipError_t e_ = (call);                                                                                       \
        if (e_ != hipSuccess) {                                                                                       \
            if (ctx) ctx->failed = 1;                                                                                 \
            return (e_ == hipErrorOutOfMemory) ? POD_ENOMEM : POD_EHIP;                                               \
        }                                                                                                             \
    } while (0)

pod_status sync_state(pod_ctx *ctx)
{
    POD_HIP(hipMemcpyAsync(&ctx->hs, ctx->ds, sizeof(DevState), hipMemcpyDeviceToHost, ctx->st));
    POD_HIP(hipStreamSynchronize(ctx->st));
    // the current basis is U[it & 1]; a merge launched on an exhausted draw
    // is a no-op on the device
    ctx->cur = ctx->hs.it & 1;
    if (ctx->hs.it < ctx->merges) ctx->merges = ctx->hs.it;
    if (ctx->hs.exhausted || (ctx->hs.s_empty && !ctx->pending)) ctx->exhausted = 1;
    return POD_OK;
}

// Status of the error flags a run raised on the device.
pod_status flag_status(int32_t flags)
{
    if (flags & FLAG_NONFINITE) return POD_ENONFINITE;
    if (flags & FLAG_NOTPD) return POD_ENOTPD;
    if (flags & FLAG_NOCONV) return POD_ENOCONV;
    return POD_OK;
}

// The stop rule of pod_converged on the state of the last sync.
int32_t stop_reason(const pod_ctx *ctx)
{
    const DevState &h = ctx->hs;
    const double tol = ctx->prm.theta_tol < 1.5707963267948966 ? sin(ctx->prm.theta_tol) : 1.0;
    if (h.flags & FLAG_NONFINITE) return POD_STOP_NONFINITE;
    if (h.flags & FLAG_NOTPD) return POD_STOP_BREAKDOWN;
    if (h.it >= 2 && h.sin_theta < tol) return POD_STOP_CONVERGED;
    if (h.exhausted || h.s_empty || ctx->exhausted) return POD_STOP_EXHAUSTED;
    if (h.it >= ctx->prm.max_iter) return POD_STOP_MAX_ITER;
    return POD_STOP_NONE;
}

void free_all(pod_ctx *ctx)
{
    void *ptrs[] = {ctx->ds,   ctx->nu,   ctx->wq,    ctx->inS,  ctx->cols, ctx->ccnt, ctx->col_log, ctx->ccnt_log,
                    ctx->col_log_off, ctx->forced, ctx->U[0], ctx->U[1], ctx->sig[0], ctx->sig[1], ctx->part,
                    ctx->G,    ctx->R1,   ctx->R2,    ctx->work, ctx->Tc,   ctx->Y,    ctx->Bpart,
                    ctx->B,    ctx->GB,   ctx->UB,    ctx->sigB, ctx->Zc, ctx->signv, ctx->signi,
                    ctx->rho,  ctx->Vt,   ctx->wr,    ctx->rows, ctx->rcnt, ctx->row_log, ctx->rcnt_log,
                    ctx->ws,   ctx->ckU,  ctx->ckS,   ctx->ckR,  ctx->ckMeta, ctx->dsb, ctx->partb, ctx->Gext,
                    ctx->adj_ws, ctx->sbar[0], ctx->sbar[1], ctx->lossp, ctx->Wt, ctx->Ubar[0], ctx->Ubar[1],
                    ctx->sin_log, ctx->tsplit, ctx->qws, ctx->rho_ort, ctx->wort,
                    ctx->ckV,  ctx->ckSc, ctx->ckRH,  ctx->rscale, ctx->adj_rows, ctx->ckRows};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
}

GemmDesc gather_desc(pod_ctx *ctx)
{
    GemmDesc d;
    d.prec = ctx->prm.precision;
    d.a_dtype = ctx->prm.a_dtype;
    d.m = ctx->prm.m;
    d.U = ctx->U[0];
    d.U1 = ctx->U[1];
    d.A = ctx->A;
    d.lda = ctx->prm.lda;
    d.cols = ctx->cols;
    d.Y = nullptr;
    d.gather = 1;
    d.guard = 1;
    d.Z = nullptr;
    d.tsplit = ctx->tsplit;
    return d;
}

BlockEigArgs block_eig_args(pod_ctx *ctx, int32_t mode)
{
    BlockEigArgs b;
    b.mode = mode;
    b.a_dtype = ctx->prm.a_dtype;
    b.A = ctx->A;
    b.lda = ctx->prm.lda;
    b.m = ctx->prm.m;
    b.cols = ctx->cols;
    b.rows = ctx->rows;
    b.rcnt = ctx->rcnt;
    b.w = ctx->prm.w;
    b.wr = ctx->wr;
    b.G = ctx->G;
    b.pmax = ctx->pmax;
    b.r_lim = (mode == 0) ? ctx->r : ctx->prm.r_update;
    b.Vt = ctx->Vt;
    b.ws = ctx->ws;
    b.ds = ctx->ds;
    if (mode == 0) b.scales = ctx->rscale;
    return b;
}

GemmDesc plain_desc(pod_ctx *ctx, const void *Y)
{
    GemmDesc d = gather_desc(ctx);
    d.Y = Y;
    d.gather = 0;
    return d;
}

// The merge sequence of Alg. 2 on X0 = [U | source(:, cols)] (gd), the new
// block weighted by sigma2 (nullable: 1) or, with use_vt, by its right factor
// Vt (computed here from the pass-1 Gram when block_eig_mode1).
pod_status merge_launch(pod_ctx *ctx, const GemmDesc &gd, const double *sigma2, bool use_vt, bool block_eig_mode1)
{
    const int32_t pm = ctx->pmax;
    if (ctx->ckU) {
        // room for this merge's checkpoint (merge index <= merges launched)
        if (!ctx->ck_lost) {
            const pod_status s = ckpt_reserve(ctx, ctx->merges + 1);
            if (s == POD_ENOMEM) ctx->ck_lost = 1;   // the forward run goes on; the reverse pass is refused
            else if (s != POD_OK) return s;
        }
        POD_HIP(launch_ckpt_pre(ctx, ctx->st));
        if (ctx->prm.w > 0) POD_HIP(launch_ckpt_rows(ctx, ctx->st));
    }
    // pass 1: G0 = X0^T X0, X0 = [U | A(:, I_c)] gathered on the fly
    POD_HIP(launch_gram_partial(gd, ctx->ds, -1, pm, ctx->part, ctx->nblk, ctx->st));
    POD_HIP(launch_gram_reduce_sel(ctx->part, ctx->nblk, pm, ctx->ds, -1, ctx->G, ctx->st));
    SmallArgs sa = ctx_small_args(ctx);
    sa.use_vt = use_vt;
    sa.sigma2 = sigma2;
    if (block_eig_mode1) {
        // the new block truncated to its leading r_update directions
        BlockEigArgs ba = block_eig_args(ctx, 1);
        POD_HIP(launch_block_eig(ba, ctx->st));
    }
    POD_HIP(launch_chol_first(sa, ctx->st));
    // Q1 = X0 T1 (T1 = P R1^-1, upper triangular unless the new block has a right factor)
    POD_HIP(launch_gemm_tall(gd, ctx->ds, -1, -2, pm, pm, ctx->Tc, pm, ctx->Y, nullptr, ctx->st, use_vt ? 0 : 1));
    // pass 2: G2 = Q1^T Q1
    GemmDesc yd = plain_desc(ctx, ctx->Y);
    POD_HIP(launch_gram_partial(yd, ctx->ds, -2, pm, ctx->part, ctx->nblk, ctx->st));
    POD_HIP(launch_gram_reduce_sel(ctx->part, ctx->nblk, pm, ctx->ds, -2, ctx->G, ctx->st));
    POD_HIP(launch_svd_merge(sa, ctx->st));
    if (ctx->ckU) POD_HIP(launch_ckpt_post(ctx, ctx->st));
    // U_new = Q1 R2^-1 U_R(:, 0:r')
    // (svd_merge advanced the merge count: U[it & 1] is the new basis)
    POD_HIP(launch_gemm_tall(yd, ctx->ds, -2, -3, pm, ctx->r, ctx->Tc, pm, ctx->U[0], ctx->U[1], ctx->st));
    ctx->merges += 1;
    return POD_OK;
}

}  // namespace

extern "C" {

const char *pod_status_str(pod_status s)
{
    switch (s) {
    case POD_OK: return "ok";
    case POD_EINVAL: return "invalid argument";
    case POD_ENOMEM: return "out of memory";
    case POD_EHIP: return "HIP runtime error";
    case POD_ENOTPD: return "Cholesky breakdown after the shifted retry";
    case POD_ESTATE: return "call out of order";
    case POD_EXHAUSTED: return "no column left to sample";
    case POD_ENONFINITE: return "non-finite value";
    case POD_ENOCONV: return "Jacobi SVD did not converge";
    }
    return "unknown status";
}

int64_t pod_sample_size(int32_t kind, int32_t k, double eps, double delta)
{
    if (k < 1 || !(eps > 0.0) || !(delta > 0.0)) return -1;
    double c;
    if (kind == 0) {
        if (!(delta < 1.0)) return -1;
        c = 4.0 * k * pow(1.0 + sqrt(8.0 * log(1.0 / delta)), 2.0) / (eps * eps);
    } else if (kind == 1) {
        if (!(delta < 2.0)) return -1;
        c = (double)k * k * pow(1.0 + sqrt(log(2.0 / delta)), 2.0) / (eps * eps * eps * eps);
    } else {
        return -1;
    }
    if (!(c < 9.0e18)) return -1;
    return (int64_t)ceil(c);
}

pod_status pod_col_sqnorms(const void *A_dev, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, double *nu_dev,
                           void *stream)
{
    pod_ctx *ctx = nullptr;
    if (!A_dev || !nu_dev || m < 1 || n < 1 || lda < m || (a_dtype != POD_F64 && a_dtype != POD_F32))
        return POD_EINVAL;
    if (n > 0x7fffffff) return POD_EINVAL;
    POD_HIP(launch_col_sqnorms(A_dev, a_dtype, m, n, lda, nu_dev, (hipStream_t)stream));
    return POD_OK;
}

pod_status pod_init(pod_ctx **out, const pod_params *prm, void *A_dev, void *stream)
{
    if (!out || !prm || !A_dev) return POD_EINVAL;
    *out = nullptr;
    pod_ctx *ctx = nullptr;
    pod_status s = ctx_create(&ctx, prm, stream);
    if (s != POD_OK) return s;
    s = ctx_bind(ctx, A_dev, prm->n, prm->lda, prm->block);
    if (s != POD_OK) {
        pod_destroy(ctx);
        return s;
    }
    *out = ctx;
    return POD_OK;
}

}  // extern "C"

DrawArgs pod::ctx_draw_args(pod_ctx *ctx)
{
    DrawArgs a;
    a.wq = (ctx->prm.col_strategy == POD_COL_ORT) ? ctx->wort : ctx->wq;
    a.wq_left = ctx->wq;
    a.inS = ctx->inS;
    a.n = ctx->prm.n;
    a.c = ctx->prm.c;
    a.unf = (ctx->prm.col_strategy == POD_COL_UNF);
    a.seed = ctx->prm.seed;
    a.block = ctx->prm.block;
    a.cols = ctx->cols;
    a.ccnt = ctx->ccnt;
    a.col_log = ctx->col_log;
    a.ccnt_log = ctx->ccnt_log;
    a.col_log_off = ctx->col_log_off;
    a.max_iter = (int32_t)((ctx->prm.max_iter < ctx->prm.n) ? ctx->prm.max_iter : ctx->prm.n);
    a.forced = (ctx->forced_g >= 0) ? ctx->forced : nullptr;
    a.forced_g = ctx->forced_g;
    a.ds = ctx->ds;
    return a;
}

SmallArgs pod::ctx_small_args(pod_ctx *ctx)
{
    const pod_params &p = ctx->prm;
    SmallArgs sa;
    sa.ds = ctx->ds;
    sa.sig0 = ctx->sig[0];
    sa.sig1 = ctx->sig[1];
    sa.G = ctx->G;
    sa.R1 = ctx->R1;
    sa.R2 = ctx->R2;
    sa.Tc = ctx->Tc;
    sa.work = ctx->work;
    sa.pmax = ctx->pmax;
    sa.r = ctx->r;
    sa.k = p.k;
    sa.prec = p.precision;
    sa.criterion = p.criterion;
    sa.urnd = unit_roundoff(p.precision);
    sa.Vt = ctx->Vt;
    sa.use_vt = 0;
    sa.sigma2 = nullptr;
    sa.ws = ctx->ws;
    return sa;
}

GemmDesc pod::ctx_gather_desc(pod_ctx *ctx) { return gather_desc(ctx); }
GemmDesc pod::ctx_plain_desc(pod_ctx *ctx, const void *Y) { return plain_desc(ctx, Y); }

pod_status pod::ctx_create(pod_ctx **out, const pod_params *prm, void *stream)
{
    if (!out || !prm) return POD_EINVAL;
    *out = nullptr;
    const pod_params &p = *prm;
    if (p.m < 1 || p.n < 1 || p.lda < p.m || p.n > 0x7fffffff || p.m > ((int64_t)1 << 40)) return POD_EINVAL;
    if (p.a_dtype != POD_F64 && p.a_dtype != POD_F32) return POD_EINVAL;
    if (p.precision != POD_F64 && p.precision != POD_F32 && p.precision != POD_BF16_REFINE) return POD_EINVAL;
    if (p.precision != POD_F64 && p.a_dtype == POD_F64) return POD_EINVAL;
    const int32_t r = p.r ? p.r : p.k;
    if (p.k < 1 || r < p.k || p.c < 1 || p.c > 1024 || p.max_iter < 1) return POD_EINVAL;
    if (p.w < 0 || p.w > 1024 || p.r_update < 0) return POD_EINVAL;
    if (p.w > 0 && p.row_strategy != POD_ROW_L2 && p.row_strategy != POD_ROW_LS) return POD_EINVAL;
    if (p.w > 0 && p.m > 0x7fffffff) return POD_EINVAL;
    if (p.col_strategy != POD_COL_L2N && p.col_strategy != POD_COL_UNF && p.col_strategy != POD_COL_ORT)
        return POD_EINVAL;
    if (p.criterion != POD_CRIT_SUBSPACE && p.criterion != POD_CRIT_MODE) return POD_EINVAL;
    if (!(p.theta_tol >= 0.0)) return POD_EINVAL;
    const int64_t cmax = (p.c < p.n) ? p.c : p.n;
    const int32_t pmax = (int32_t)(((r + cmax) + 15) & ~15);
    if (pmax > 160) return POD_EINVAL;

    pod_ctx *ctx = new (std::nothrow) pod_ctx();
    if (!ctx) return POD_ENOMEM;
    ctx->prm = p;
    ctx->prm.r = r;
    ctx->r = r;
    ctx->pmax = pmax;
    ctx->st = (hipStream_t)stream;
    ctx->n_cap = p.n;
    ctx->esz = (p.precision == POD_F64) ? 8 : 4;
    const int64_t m = p.m, n = p.n;
    const int32_t cap_iter = (int32_t)((p.max_iter < n) ? p.max_iter : n) + 1;
    ctx->nblk = (int32_t)((m + 255) / 256 < 256 ? (m + 255) / 256 : 256);
    if (ctx->nblk < 1) ctx->nblk = 1;
    ctx->nsplit = 32;
    if (m < 4096) ctx->nsplit = 8;
    hipError_t e = hipSuccess;
#define ALLOC(ptr, T, count)                                                                                          \
    if (e == hipSuccess) e = dalloc((T **)&(ptr), (size_t)(count))
    ALLOC(ctx->ds, DevState, 1);
    ALLOC(ctx->nu, double, n);
    ALLOC(ctx->wq, uint64_t, n);
    ALLOC(ctx->inS, uint8_t, n);
    ALLOC(ctx->cols, int32_t, 1024);
    ALLOC(ctx->ccnt, int32_t, 1024);
    ALLOC(ctx->forced, int32_t, 4096);
    ALLOC(ctx->col_log, int32_t, n);
    ALLOC(ctx->ccnt_log, int32_t, n);
    ALLOC(ctx->col_log_off, int32_t, cap_iter + 1);
    ALLOC(ctx->sin_log, double, cap_iter + 1);
    ctx->log_cap = cap_iter;
    for (int b = 0; b < 2; ++b) {
        ALLOC(ctx->U[b], unsigned char, (size_t)m * r * ctx->esz);
        ALLOC(ctx->sig[b], double, r);
    }
    ALLOC(ctx->part, double, (size_t)ctx->nblk * pmax * pmax);
    ALLOC(ctx->G, double, pmax * pmax);
    ALLOC(ctx->R1, double, pmax * pmax);
    ALLOC(ctx->R2, double, pmax * pmax);
    ALLOC(ctx->work, double, pmax * pmax);
    ALLOC(ctx->Tc, unsigned char, (size_t)pmax * pmax * ctx->esz);
    if (p.precision == POD_BF16_REFINE) ALLOC(ctx->tsplit, unsigned char, TSPLIT_BYTES);
    ALLOC(ctx->Y, unsigned char, (size_t)m * pmax * ctx->esz);
    ALLOC(ctx->Bpart, double, (size_t)ctx->nsplit * r * n);
    ALLOC(ctx->B, double, (size_t)r * n);
    ALLOC(ctx->GB, double, (size_t)r * r);
    ALLOC(ctx->UB, double, (size_t)r * r);
    ALLOC(ctx->sigB, double, r);
    ALLOC(ctx->Zc, unsigned char, (size_t)r * r * ctx->esz);
    ALLOC(ctx->signv, double, (size_t)64 * r);
    ALLOC(ctx->signi, int64_t, (size_t)64 * r);
    if (p.w > 0 || p.r_update > 0) ALLOC(ctx->Vt, double, (size_t)pmax * pmax);
    if (p.col_strategy == POD_COL_ORT) {
        ALLOC(ctx->rho_ort, double, n);
        ALLOC(ctx->wort, uint64_t, n);
    }
    if (pmax > 64) ALLOC(ctx->ws, double, big_dinv_offset(pmax) + BIG_DINV_DOUBLES);
    if (p.w > 0) {
        ALLOC(ctx->rho, double, m);
        ALLOC(ctx->wr, uint64_t, m);
        ALLOC(ctx->rows, int32_t, p.w);
        ALLOC(ctx->rcnt, int32_t, p.w);
        ALLOC(ctx->row_log, int32_t, (size_t)cap_iter * p.w);
        ALLOC(ctx->rscale, double, (size_t)p.w);
        ALLOC(ctx->rcnt_log, int32_t, (size_t)cap_iter * p.w);
    }
#undef ALLOC
    if (e != hipSuccess) {
        free_all(ctx);
        delete ctx;
        return e == hipErrorOutOfMemory ? POD_ENOMEM : POD_EHIP;
    }
    DevState h{};
    h.sin_theta = __builtin_nan("");
    ctx->hs = h;
    e = hipMemcpyAsync(ctx->ds, &h, sizeof(DevState), hipMemcpyHostToDevice, ctx->st);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->sig[0], 0, sizeof(double) * r, ctx->st);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->sig[1], 0, sizeof(double) * r, ctx->st);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
    if (e != hipSuccess) {
        free_all(ctx);
        delete ctx;
        return POD_EHIP;
    }
    *out = ctx;
    return POD_OK;
}

pod_status pod::ctx_bind(pod_ctx *ctx, void *A_dev, int64_t n, int64_t lda, uint64_t block)
{
    if (!ctx || !A_dev || n < 1 || n > ctx->n_cap || lda < ctx->prm.m) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    ctx->proj_it = -1;   // a fresh run: no Rayleigh-Ritz values yet
    ctx->prm.n = n;
    ctx->prm.lda = lda;
    ctx->prm.block = block;
    ctx->A = A_dev;
    ctx->cur = 0;
    ctx->pending = 0;
    ctx->merges = 0;
    ctx->exhausted = 0;
    ctx->forced_g = -1;
    ctx->forced_h = 0;
    const pod_params &p = ctx->prm;
    const int64_t m = p.m;
    const int32_t r = ctx->r;
    const int32_t cap_iter = (int32_t)((p.max_iter < n) ? p.max_iter : n) + 1;
    DevState h{};
    h.sin_theta = __builtin_nan("");
    ctx->hs = h;   // the copy reads ctx->hs, which outlives the call
    POD_HIP(hipMemcpyAsync(ctx->ds, &ctx->hs, sizeof(DevState), hipMemcpyHostToDevice, ctx->st));
    POD_HIP(hipMemsetAsync(ctx->inS, 1, (size_t)n, ctx->st));
    POD_HIP(hipMemsetAsync(ctx->col_log_off, 0, sizeof(int32_t) * (cap_iter + 1), ctx->st));
    POD_HIP(hipMemsetAsync(ctx->sig[0], 0, sizeof(double) * r, ctx->st));
    POD_HIP(hipMemsetAsync(ctx->sig[1], 0, sizeof(double) * r, ctx->st));
    if (p.w > 0) POD_HIP(hipMemsetAsync(ctx->rcnt_log, 0, sizeof(int32_t) * (size_t)cap_iter * p.w, ctx->st));
    if (p.center_rows) {
        // row means (FP64), then a_ij <- a_ij - mean_i
        const pod_status sc = pod_center_rows(A_dev, p.a_dtype, m, n, p.lda, ctx->st);
        if (sc != POD_OK) {
            if (sc == POD_EHIP) ctx->failed = 1;
            return sc;
        }
    }
    POD_HIP(launch_col_sqnorms(A_dev, p.a_dtype, m, n, p.lda, ctx->nu, ctx->st));
    POD_HIP(launch_quantize(ctx->nu, n, ctx->wq, ctx->ds, 0, ctx->st));
    return POD_OK;
}

// The draw of one iteration of Alg. 1 (columns; rows and the right factor of
// the new block when rows are sampled), enqueued without waiting.
static pod_status enqueue_sample(pod_ctx *ctx)
{
    if (ctx->prm.col_strategy == POD_COL_ORT) {
        // ORT weights from the second iteration: B = U^T A over every column
        // (the live rank and the current basis are picked on the device),
        // residuals nu_j - |B(:, j)|^2 over S, integer weights
        const pod_params &p = ctx->prm;
        ProjArgs pa;
        pa.prec = p.precision;
        pa.a_dtype = p.a_dtype;
        pa.m = p.m;
        pa.n = p.n;
        pa.lda = p.lda;
        pa.U = ctx->U[0];
        pa.U1 = ctx->U[1];
        pa.ds = ctx->ds;
        pa.A = ctx->A;
        pa.r = ctx->r;
        pa.Bpart = ctx->Bpart;
        pa.nsplit = ctx->nsplit;
        pa.B = ctx->B;
        POD_HIP(launch_project_partial(pa, ctx->st));
        POD_HIP(launch_project_reduce(pa, ctx->st));
        POD_HIP(launch_ort_resid(ctx->nu, ctx->B, ctx->r, p.n, ctx->inS, ort_floor(p.precision), ctx->ds, ctx->rho_ort,
                                 ctx->st));
        POD_HIP(launch_quantize(ctx->rho_ort, p.n, ctx->wort, ctx->ds, 0, ctx->st));
    }
    DrawArgs a = ctx_draw_args(ctx);
    POD_HIP(launch_draw_cols(a, ctx->st));
    const pod_params &p = ctx->prm;
    if (p.w > 0) {
        // SAMPLE AND SCALE UNIQUE ROWS, then the right factor of the new block
        const bool ls = (p.row_strategy == POD_ROW_LS);
        POD_HIP(launch_row_sqnorms(ctx->A, p.a_dtype, p.m, p.lda, ctx->cols, ls ? ctx->U[0] : nullptr,
                                   ls ? ctx->U[1] : nullptr, p.precision, p.k, ctx->ds, ctx->rho, ctx->st));
        POD_HIP(launch_quantize(ctx->rho, p.m, ctx->wr, ctx->ds, 1, ctx->st));
        RowDrawArgs ra;
        ra.wr = ctx->wr;
        ra.m = p.m;
        ra.w = p.w;
        ra.seed = p.seed;
        ra.block = p.block;
        ra.rows = ctx->rows;
        ra.rcnt = ctx->rcnt;
        ra.row_log = ctx->row_log;
        ra.rcnt_log = ctx->rcnt_log;
        ra.max_iter = a.max_iter;
        ra.forced = (ctx->forced_g >= 0) ? ctx->forced : nullptr;
        ra.forced_h = ctx->forced_h;
        ra.ds = ctx->ds;
        POD_HIP(launch_draw_rows(ra, ctx->st));
        BlockEigArgs ba = block_eig_args(ctx, 0);
        POD_HIP(launch_block_eig(ba, ctx->st));
    }
    ctx->forced_g = -1;
    ctx->forced_h = 0;
    return POD_OK;
}


extern "C" {

pod_status pod_sample(pod_ctx *ctx, int32_t *g_out, int32_t *h_out)
{
    if (!ctx) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    if (ctx->pending) return POD_ESTATE;
    if (ctx->exhausted) return POD_EXHAUSTED;
    if (ctx->merges >= ctx->prm.max_iter) return POD_ESTATE;
    pod_status s0 = enqueue_sample(ctx);
    if (s0 != POD_OK) return s0;
    ctx->pending = 1;
    if (g_out || h_out) {
        pod_status s = sync_state(ctx);
        if (s != POD_OK) return s;
        if (g_out) *g_out = ctx->hs.g;
        if (h_out) *h_out = ctx->hs.h;
        if (ctx->hs.exhausted) {
            ctx->pending = 0;
            return POD_EXHAUSTED;
        }
    }
    return POD_OK;
}

pod_status pod_merge(pod_ctx *ctx)
{
    if (!ctx) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    if (!ctx->pending) return POD_ESTATE;
    const pod_params &p = ctx->prm;
    pod_status s = merge_launch(ctx, gather_desc(ctx), nullptr, p.w > 0 || p.r_update > 0, p.w == 0 && p.r_update > 0);
    if (s != POD_OK) return s;
    ctx->pending = 0;
    return POD_OK;
}

pod_status pod_run(pod_ctx *ctx, int32_t max_merges, int32_t stop_on_converged, int32_t chunk, double *sin_out,
                   int32_t *merges_out, int32_t *done_out)
{
    if (!ctx || max_merges < 0) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    if (ctx->pending) return POD_ESTATE;
    if (chunk < 1) chunk = 8;
    pod_status s = sync_state(ctx);
    if (s != POD_OK) return s;
    const pod_params &p = ctx->prm;
    const int32_t it0 = ctx->hs.it;
    const int32_t limit = (int32_t)((int64_t)it0 + max_merges < (int64_t)p.max_iter ? it0 + max_merges : p.max_iter);
    const double tol = p.theta_tol < 1.5707963267948966 ? sin(p.theta_tol) : 1.0;
    const bool rows_eig = p.w > 0 || p.r_update > 0, block_mode1 = p.w == 0 && p.r_update > 0;
    int32_t enqueued = 0;
    while (!ctx->exhausted && ctx->hs.it < limit && !ctx->hs.done) {
        // up to `chunk` iterations without waiting; the stop test on the device
        // turns the rest of the chunk into no-ops
        const int32_t todo = (limit - ctx->hs.it < chunk) ? limit - ctx->hs.it : chunk;
        for (int32_t q = 0; q < todo; ++q) {
            s = enqueue_sample(ctx);
            if (s != POD_OK) return s;
            s = merge_launch(ctx, gather_desc(ctx), nullptr, rows_eig, block_mode1);
            if (s != POD_OK) return s;
            POD_HIP(launch_run_done(ctx->ds, limit, tol, stop_on_converged ? 1 : 0, ctx->sin_log, ctx->log_cap,
                                    ctx->st));
            ++enqueued;
        }
        s = sync_state(ctx);
        if (s != POD_OK) return s;
    }
    const int32_t merged = ctx->hs.it - it0;
    if (done_out) *done_out = ctx->hs.done || ctx->exhausted || ctx->hs.it >= p.max_iter;
    if (merges_out) *merges_out = merged;
    if (sin_out && merged > 0)
        POD_HIP(hipMemcpyAsync(sin_out, ctx->sin_log + it0, sizeof(double) * merged, hipMemcpyDeviceToHost, ctx->st));
    // hand the context back to step-by-step use
    ctx->merges = ctx->hs.it;
    if (ctx->hs.done) {
        ctx->hs.done = 0;
        POD_HIP(hipMemcpyAsync(ctx->ds, &ctx->hs, sizeof(DevState), hipMemcpyHostToDevice, ctx->st));
    }
    POD_HIP(hipStreamSynchronize(ctx->st));
    (void)enqueued;
    return flag_status(ctx->hs.flags);
}

pod_status pod_converged(pod_ctx *ctx, int32_t *done, double *sin_theta_max)
{
    if (!ctx || !done) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    if (ctx->pending) return POD_ESTATE;
    pod_status s = sync_state(ctx);
    if (s != POD_OK) return s;
    const DevState &h = ctx->hs;
    if (sin_theta_max) *sin_theta_max = h.sin_theta;
    const double tol = ctx->prm.theta_tol < 1.5707963267948966 ? sin(ctx->prm.theta_tol) : 1.0;
    *done = h.exhausted || h.s_empty || h.it >= ctx->prm.max_iter || (h.it >= 2 && h.sin_theta < tol) ||
            (h.flags & FLAG_FATAL) != 0;
    return flag_status(h.flags);
}

pod_status pod_project(pod_ctx *ctx, void *U_out, double *sigma_out, void *V_out)
{
    return ctx_project(ctx, U_out, sigma_out, V_out, 0);
}

}  // extern "C"

pod_status pod::ctx_project(pod_ctx *ctx, void *U_out, double *sigma_out, void *V_out, int32_t kout)
{
    if (!ctx || !U_out || !sigma_out) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    if (ctx->pending) return POD_ESTATE;
    pod_status s = sync_state(ctx);
    if (s != POD_OK) return s;
    const int32_t rs = ctx->hs.rs;
    if (rs < 1) return POD_ESTATE;
    int32_t k = (ctx->prm.k < rs) ? ctx->prm.k : rs;
    if (kout > 0) k = (kout < rs) ? kout : rs;
    const pod_params &p = ctx->prm;
    ProjArgs pa;
    pa.prec = p.precision;
    pa.a_dtype = p.a_dtype;
    pa.m = p.m;
    pa.n = p.n;
    pa.lda = p.lda;
    pa.U = ctx->U[ctx->cur];
    pa.A = ctx->A;
    pa.r = rs;
    pa.Bpart = ctx->Bpart;
    pa.nsplit = ctx->nsplit;
    pa.B = ctx->B;
    POD_HIP(launch_project_partial(pa, ctx->st));
    POD_HIP(launch_project_reduce(pa, ctx->st));
    RRArgs ra;
    ra.B = ctx->B;
    ra.n = p.n;
    ra.r = rs;
    ra.k = k;
    ra.part = ctx->Bpart;   // free once B is reduced
    ra.GB = ctx->GB;
    ra.UB = ctx->UB;
    ra.sig = ctx->sigB;
    ra.Zc = ctx->Zc;
    ra.ws = ctx->ws;
    ra.prec = p.precision;
    ra.ds = ctx->ds;
    POD_HIP(launch_rr_small(ra, ctx->st));
    GemmDesc ud = plain_desc(ctx, ctx->U[ctx->cur]);
    ud.prec = (p.precision == POD_F64) ? POD_F64 : POD_F32;   // the Rayleigh-Ritz rotation in FP32
    ud.guard = 0;
    POD_HIP(launch_gemm_tall(ud, ctx->ds, rs, k, rs, k, ctx->Zc, rs, U_out, nullptr, ctx->st));
    POD_HIP(hipMemcpyAsync(sigma_out, ctx->sigB, sizeof(double) * k, hipMemcpyDeviceToDevice, ctx->st));
    if (V_out) POD_HIP(launch_rr_v(ctx->B, p.n, rs, k, ctx->UB, ctx->sigB, p.precision, V_out, ctx->st));
    POD_HIP(launch_sign_fix(p.precision, U_out, p.m, k, V_out, p.n, ctx->signv, ctx->signi, ctx->st));
    s = sync_state(ctx);
    if (s != POD_OK) return s;
    s = flag_status(ctx->hs.flags);
    if (s != POD_OK) return s;
    ctx->proj_it = ctx->hs.it;
    ctx->proj_k = k;
    ctx->proj_rank = rs;
    return POD_OK;
}

pod_status pod::ctx_merge_basis(pod_ctx *ctx, const void *Ub, const double *sb, int32_t rb)
{
    if (!ctx || !Ub || !sb || rb < 1 || rb > ctx->n_cap || rb > ctx->prm.c) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    if (ctx->pending) return POD_ESTATE;
    const pod_params &p = ctx->prm;
    const int32_t first = (ctx->merges == 0);
    POD_HIP(launch_basis_state(ctx->ds, rb, ctx->r, first, ctx->cols, ctx->st));
    if (first) {
        // the first block is the state (Alg. 3)
        // (the merge count becomes 1: the current basis is U[1])
        const int32_t rr = (rb < ctx->r) ? rb : ctx->r;
        POD_HIP(hipMemcpyAsync(ctx->U[1], Ub, (size_t)p.m * rr * ctx->esz, hipMemcpyDeviceToDevice, ctx->st));
        POD_HIP(hipMemcpyAsync(ctx->sig[1], sb, sizeof(double) * rr, hipMemcpyDeviceToDevice, ctx->st));
        ctx->merges = 1;
        return POD_OK;
    }
    GemmDesc gd = gather_desc(ctx);
    gd.A = Ub;
    gd.a_dtype = p.precision == POD_F64 ? POD_F64 : POD_F32;
    gd.lda = p.m;
    return merge_launch(ctx, gd, sb, false, false);
}

extern "C" {

pod_status pod_get_basis(pod_ctx *ctx, void *U_out, double *sigma_out, int32_t *rank_out)
{
    if (!ctx) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    pod_status s = sync_state(ctx);
    if (s != POD_OK) return s;
    const int32_t rs = ctx->hs.rs;
    if (rank_out) *rank_out = rs;
    if (U_out && rs > 0)
        POD_HIP(hipMemcpyAsync(U_out, ctx->U[ctx->cur], (size_t)ctx->prm.m * rs * ctx->esz, hipMemcpyDeviceToDevice,
                               ctx->st));
    if (sigma_out && rs > 0)
        POD_HIP(hipMemcpyAsync(sigma_out, ctx->sig[ctx->cur], sizeof(double) * rs, hipMemcpyDeviceToDevice, ctx->st));
    POD_HIP(hipStreamSynchronize(ctx->st));
    return POD_OK;
}

pod_status pod_get_info(pod_ctx *ctx, pod_info *info)
{
    if (!ctx || !info) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    pod_status s = sync_state(ctx);
    if (s != POD_OK) return s;
    info->iter = ctx->hs.it;
    info->rank = ctx->hs.rs;
    info->g = ctx->hs.g;
    info->h = ctx->hs.h;
    info->exhausted = ctx->hs.exhausted || ctx->hs.s_empty;
    info->flags = ctx->hs.flags;
    info->max_sweeps = ctx->hs.sweeps;
    info->total_sweeps = ctx->hs.sweeps_total;
    info->sin_theta = ctx->hs.sin_theta;
    info->stop_reason = stop_reason(ctx);
    info->reserved = 0;
    return POD_OK;
}

pod_status pod_set_indices(pod_ctx *ctx, int32_t iter, const int32_t *cols, const int32_t *col_counts, int32_t g,
                           const int32_t *rows, const int32_t *row_counts, int32_t h)
{
    if (!ctx || !cols || g < 1) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    if (ctx->pending) return POD_ESTATE;
    pod_status s = sync_state(ctx);
    if (s != POD_OK) return s;
    const pod_params &p = ctx->prm;
    if (iter != ctx->hs.it || ctx->exhausted || ctx->hs.it >= p.max_iter) return POD_ESTATE;
    if (g > p.c || g > 1024) return POD_EINVAL;
    for (int32_t d = 0; d < g; ++d) {
        if (cols[d] < 0 || cols[d] >= p.n || (d > 0 && cols[d] <= cols[d - 1])) return POD_EINVAL;
        if (col_counts && col_counts[d] < 1) return POD_EINVAL;
    }
    if (p.w > 0) {
        if (!rows || !row_counts || h < 1 || h > p.w) return POD_EINVAL;
        int64_t tot = 0;
        for (int32_t d = 0; d < h; ++d) {
            if (rows[d] < 0 || rows[d] >= p.m || (d > 0 && rows[d] <= rows[d - 1]) || row_counts[d] < 1)
                return POD_EINVAL;
            tot += row_counts[d];
        }
        if (tot != p.w) return POD_EINVAL;
    }
    // the columns must still be in S
    uint8_t *in = (uint8_t *)malloc((size_t)p.n);
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * 4096);
    if (!in || !buf) {
        free(in);
        free(buf);
        return POD_ENOMEM;
    }
    hipError_t e = hipMemcpyAsync(in, ctx->inS, (size_t)p.n, hipMemcpyDeviceToHost, ctx->st);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
    bool ok = (e == hipSuccess);
    for (int32_t d = 0; ok && d < g; ++d) ok = in[cols[d]] != 0;
    free(in);
    if (e != hipSuccess) {
        free(buf);
        ctx->failed = 1;
        return POD_EHIP;
    }
    if (!ok) {
        free(buf);
        return POD_EINVAL;
    }
    memset(buf, 0, sizeof(int32_t) * 4096);
    for (int32_t d = 0; d < g; ++d) {
        buf[d] = cols[d];
        buf[1024 + d] = col_counts ? col_counts[d] : 1;
    }
    if (p.w > 0)
        for (int32_t d = 0; d < h; ++d) {
            buf[2048 + d] = rows[d];
            buf[3072 + d] = row_counts[d];
        }
    e = hipMemcpyAsync(ctx->forced, buf, sizeof(int32_t) * 4096, hipMemcpyHostToDevice, ctx->st);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
    free(buf);
    if (e != hipSuccess) {
        ctx->failed = 1;
        return POD_EHIP;
    }
    ctx->forced_g = g;
    ctx->forced_h = (p.w > 0) ? h : 0;
    return POD_OK;
}

pod_status pod_get_indices(pod_ctx *ctx, int32_t iter, int32_t *cols, int32_t *col_counts, int32_t *g, int32_t *rows,
                           int32_t *row_counts, int32_t *h)
{
    if (!ctx || iter < 0) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    pod_status s = sync_state(ctx);
    if (s != POD_OK) return s;
    const int32_t cap = (int32_t)((ctx->prm.max_iter < ctx->prm.n) ? ctx->prm.max_iter : ctx->prm.n);
    const int32_t drawn = ctx->hs.it + (ctx->pending ? 1 : 0);
    if (iter >= drawn || iter >= cap) return POD_EINVAL;
    int32_t off[2];
    POD_HIP(hipMemcpy(off, ctx->col_log_off + iter, sizeof(off), hipMemcpyDeviceToHost));
    const int32_t cnt = off[1] - off[0];
    if (g) *g = cnt;
    if (cols && cnt > 0)
        POD_HIP(hipMemcpy(cols, ctx->col_log + off[0], sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
    if (col_counts && cnt > 0)
        POD_HIP(hipMemcpy(col_counts, ctx->ccnt_log + off[0], sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
    int32_t hh = 0;
    if (ctx->prm.w > 0) {
        const int32_t w = ctx->prm.w;
        int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)w);
        if (!buf) return POD_ENOMEM;
        hipError_t e = hipMemcpy(buf, ctx->row_log + (size_t)iter * w, sizeof(int32_t) * w, hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMemcpy(buf + w, ctx->rcnt_log + (size_t)iter * w, sizeof(int32_t) * w, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            free(buf);
            ctx->failed = 1;
            return POD_EHIP;
        }
        while (hh < w && buf[w + hh] > 0) ++hh;
        if (rows) memcpy(rows, buf, sizeof(int32_t) * hh);
        if (row_counts) memcpy(row_counts, buf + w, sizeof(int32_t) * hh);
        free(buf);
    }
    if (h) *h = hh;
    return POD_OK;
}

pod_status pod_get_col_sqnorms(pod_ctx *ctx, double *nu_host)
{
    if (!ctx || !nu_host) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    POD_HIP(hipMemcpyAsync(nu_host, ctx->nu, sizeof(double) * ctx->prm.n, hipMemcpyDeviceToHost, ctx->st));
    POD_HIP(hipStreamSynchronize(ctx->st));
    return POD_OK;
}

void pod_destroy(pod_ctx *ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->st);
    free_all(ctx);
    delete ctx;
}

}  // extern "C"

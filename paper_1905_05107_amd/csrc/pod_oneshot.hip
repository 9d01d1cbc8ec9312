// pod_oneshot.hip -- the one-shot sampled SVDs of Appendix A on the kernels of
// the iterative path: Alg. 4 (LTSVD: columns drawn with the norm
// probabilities, scaled, the SVD of the sample from the eigen-decomposition of
// C^T C) and Alg. 5 (CTSVD: rows of the scaled sample drawn and scaled in
// turn, the eigen-decomposition of W^T W, the eps filter).
#include <math.h>

#include "pod_ctx.h"

using namespace pod;

namespace {

#define OS_HIP(call)                                                                                                  \
    do {                                                                                                              \
        hipError_t e_ = (call);                                                                                       \
        if (e_ != hipSuccess) {                                                                                       \
            pod_destroy(ctx);                                                                                         \
            return (e_ == hipErrorOutOfMemory) ? POD_ENOMEM : POD_EHIP;                                               \
        }                                                                                                             \
    } while (0)

// Column scales of the folded draws: distinct column d, drawn t_d times,
// enters once with s_d = sqrt((t_d W) / (c w_j)) (W the total integer weight,
// w_j the column's weight: p_j = w_j / W), which keeps C C^T the sum over the c
// draws of a_j a_j^T / (c p_j).
__global__ __launch_bounds__(256) void k_oneshot_scale(const int32_t *__restrict__ cols,
                                                       const int32_t *__restrict__ cnt,
                                                       const uint64_t *__restrict__ wq, const DevState *ds, int32_t c,
                                                       double *__restrict__ scale)
{
    const int g = ds->g;
    const double W = (double)ds->wtot;
    for (int d = threadIdx.x; d < g; d += 256)
        scale[d] = sqrt(((double)cnt[d] * W) / ((double)c * (double)wq[cols[d]]));
}

// T = S V(:, 0:l) Sigma^-1 (g x l in a zero-padded pm x pm, compute type):
// u_i = C v_i / sigma_i with C = D S; the l singular values; the device counts
// for the tall transform (input g columns of D, output l columns).
template <typename TC>
__global__ __launch_bounds__(256) void k_oneshot_t(const double *__restrict__ Vt, const double *__restrict__ evals,
                                                   const double *__restrict__ scale, int32_t pm, int32_t k,
                                                   DevState *ds, TC *__restrict__ T, double *__restrict__ sigma)
{
    const int g = ds->g, l = ds->ru;
    for (int idx = threadIdx.x; idx < pm * pm; idx += 256) {
        const int i = idx % pm, j = idx / pm;
        double v = 0.0;
        if (i < g && j < l) v = (scale[i] * Vt[i + j * pm]) / sqrt(evals[j]);
        T[idx] = (TC)v;
    }
    for (int j = threadIdx.x; j < k; j += 256) sigma[j] = (j < l) ? sqrt(evals[j]) : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        ds->rs = 0;
        ds->p0 = g;
        ds->rnew = l;
    }
}

}  // namespace

extern "C" {

pod_status pod_oneshot(const pod_params *prm, const void *A_dev, double eps, void *U_out, double *sigma_out,
                       int32_t *l_out, void *stream)
{
    if (!prm || !A_dev || !U_out || !sigma_out) return POD_EINVAL;
    if (prm->w > 0 && !(eps > 0.0)) return POD_EINVAL;
    pod_params p = *prm;
    p.r = p.k;
    p.r_update = 0;
    p.col_strategy = POD_COL_L2N;
    p.max_iter = 1;
    pod_ctx *ctx = nullptr;
    pod_status s = ctx_create(&ctx, &p, stream);
    if (s != POD_OK) return s;
    s = ctx_bind(ctx, const_cast<void *>(A_dev), p.n, p.lda, p.block);
    if (s != POD_OK) {
        pod_destroy(ctx);
        return s;
    }
    hipStream_t st = ctx->st;
    const int32_t pm = ctx->pmax;
    if (!ctx->Vt) OS_HIP(hipMalloc((void **)&ctx->Vt, sizeof(double) * (size_t)pm * pm));
    double *scale = ctx->work, *evals = ctx->work + pm;   // pm^2 >= 2 pm doubles
    // the first loop of Alg. 4 / Alg. 5: c draws over the columns (Philox key
    // (seed, 0), counter (0, d/4, block, 0)), folded into the distinct ones
    OS_HIP(launch_draw_cols(ctx_draw_args(ctx), st));
    hipLaunchKernelGGL(k_oneshot_scale, dim3(1), dim3(256), 0, st, ctx->cols, ctx->ccnt, ctx->wq, ctx->ds, p.c,
                       scale);
    OS_HIP(hipGetLastError());
    BlockEigArgs ba;
    ba.a_dtype = p.a_dtype;
    ba.A = A_dev;
    ba.lda = p.lda;
    ba.m = p.m;
    ba.cols = ctx->cols;
    ba.rows = ctx->rows;
    ba.rcnt = ctx->rcnt;
    ba.w = p.w;
    ba.wr = ctx->wr;
    ba.G = ctx->G;
    ba.pmax = pm;
    ba.r_lim = p.k;
    ba.Vt = ctx->Vt;
    ba.ws = ctx->ws;
    ba.ds = ctx->ds;
    ba.cscale = scale;
    ba.evals = evals;
    const GemmDesc gd = ctx_gather_desc(ctx);
    if (p.w == 0) {
        // Alg. 4: C^T C = S D^T D S from the Gram of the gathered columns;
        // l = min(k, rank C), rank C = #{lambda_i > g u lambda_1}
        OS_HIP(launch_gram_partial(gd, ctx->ds, -1, pm, ctx->part, ctx->nblk, st));
        OS_HIP(launch_gram_reduce_sel(ctx->part, ctx->nblk, pm, ctx->ds, -1, ctx->G, st));
        ba.mode = 1;
        ba.crit = 0;
    } else {
        // Alg. 5: rows drawn with q_i = |c^i|^2 / |C|_F^2 of the scaled sample
        // (key (seed, 1)), W = diag(sqrt(t_i / (w q_i))) C(I_r, :);
        // l = min(k, max{r : sigma_r^2 >= gamma |W|_F^2}), gamma = eps / (100 k)
        OS_HIP(launch_row_sqnorms(A_dev, p.a_dtype, p.m, p.lda, ctx->cols, nullptr, nullptr, p.precision, p.k,
                                  ctx->ds, ctx->rho, st, scale));
        OS_HIP(launch_quantize(ctx->rho, p.m, ctx->wr, ctx->ds, 1, st));
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
        ra.max_iter = 1;
        ra.forced = nullptr;
        ra.forced_h = 0;
        ra.ds = ctx->ds;
        OS_HIP(launch_draw_rows(ra, st));
        ba.mode = 0;
        ba.crit = 1;
        ba.gamma = eps / (100.0 * p.k);
    }
    OS_HIP(launch_block_eig(ba, st));
    const size_t esz = ctx->esz;
    if (p.precision == POD_F64)
        hipLaunchKernelGGL(k_oneshot_t<double>, dim3(1), dim3(256), 0, st, ctx->Vt, evals, scale, pm, p.k, ctx->ds,
                           (double *)ctx->Tc, sigma_out);
    else
        hipLaunchKernelGGL(k_oneshot_t<float>, dim3(1), dim3(256), 0, st, ctx->Vt, evals, scale, pm, p.k, ctx->ds,
                           (float *)ctx->Tc, sigma_out);
    OS_HIP(hipGetLastError());
    OS_HIP(hipMemsetAsync(U_out, 0, (size_t)p.m * p.k * esz, st));
    GemmDesc td = gd;
    td.prec = (p.precision == POD_F64) ? POD_F64 : POD_F32;   // FP32 product on the split-BF16 setting
    td.guard = 0;
    OS_HIP(launch_gemm_tall(td, ctx->ds, -1, -3, pm, p.k, ctx->Tc, pm, U_out, nullptr, st, 0));
    DevState h{};
    OS_HIP(hipMemcpyAsync(&h, ctx->ds, sizeof(DevState), hipMemcpyDeviceToHost, st));
    OS_HIP(hipStreamSynchronize(st));
    OS_HIP(launch_sign_fix(td.prec, U_out, p.m, h.ru, nullptr, 0, ctx->signv, ctx->signi, st));
    OS_HIP(hipStreamSynchronize(st));
    if (l_out) *l_out = h.ru;
    const int32_t flags = h.flags;
    pod_destroy(ctx);
    if (flags & FLAG_NONFINITE) return POD_ENONFINITE;
    if (h.exhausted || h.g == 0) return POD_EXHAUSTED;
    if (p.w > 0 && (flags & FLAG_ZERO_ROWS)) return POD_EXHAUSTED;
    return POD_OK;
}

}  // extern "C"

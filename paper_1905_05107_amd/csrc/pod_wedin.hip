// pod_wedin.hip -- quality measure of the converged modes (Sec. "Quality of
// converged solution", Eq. ang_meas).  With the top k Rayleigh-Ritz triplets
// (U_k, Sigma_k, V_k) of the final step,
//     R = A V_k - U_k Sigma_k,   S = A^T U_k - V_k Sigma_k,
// Wedin's theorem bounds the sines of the principal angles between the exact
// and the computed dominant subspaces by sqrt(||R||_F^2 + ||S||_F^2) / omega;
// omega is estimated from the (k+1)-th computed value:
// omega^ = min(|sigma_k - sigma_{k+1}|, sigma_k).
//
// Both residuals are differences of nearly equal quantities, so every
// product is accumulated in FP64 (A and the modes converted on load):
//   R: one pass over A by row stripes, one row per thread, V_k staged in LDS
//      64 columns of A at a time, the residual squared and summed per block;
//   S: A^T U_k by the FP64 projection kernels on an FP64 copy of U_k (a
//      second pass over A), then the residual against V_k Sigma_k.
// Every sum runs in a fixed order, so the result is reproducible.
#include <cmath>

#include "pod_ctx.h"

using namespace pod;

namespace {

constexpr int WT = 256;

__device__ __forceinline__ double wsum64(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of v over the workgroup (WT threads), waves in order; valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    v = wsum64(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

template <typename T> __device__ __forceinline__ double ld(const T *p, int64_t i) { return (double)p[i]; }

// Per block: sum over its rows i of sum_c (A(i, :) V(:, c) - U(i, c) s_c)^2.
// KC >= k accumulators per thread (columns c >= k have V = 0 in LDS).
template <int KC, typename TA, typename TV>
__global__ __launch_bounds__(WT) void k_wedin_r(const TA *__restrict__ A, int64_t m, int64_t n, int64_t lda,
                                                const TV *__restrict__ V, const TV *__restrict__ U,
                                                const double *__restrict__ sig, int k, double *__restrict__ part)
{
    constexpr int JC = 64;
    __shared__ double Vs[JC][KC];
    __shared__ double sh[WT / 64];
    const int64_t i = (int64_t)blockIdx.x * WT + threadIdx.x;
    const bool live = i < m;
    const TA *Ai = A + (live ? i : 0);
    double acc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += JC) {
        const int jn = (n - j0 < JC) ? (int)(n - j0) : JC;
        __syncthreads();   // the previous chunk is consumed
        for (int idx = threadIdx.x; idx < JC * KC; idx += WT) {
            const int jj = idx % JC, c = idx / JC;
            Vs[jj][c] = (jj < jn && c < k) ? ld(V, j0 + jj + (int64_t)c * n) : 0.0;
        }
        __syncthreads();
        if (live) {
            int jj = 0;
            for (; jj + 8 <= jn; jj += 8) {
                double a[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) a[q] = ld(Ai, (j0 + jj + q) * lda);
#pragma unroll
                for (int q = 0; q < 8; ++q)
#pragma unroll
                    for (int c = 0; c < KC; ++c) acc[c] = fma(a[q], Vs[jj + q][c], acc[c]);
            }
            for (; jj < jn; ++jj) {
                const double a = ld(Ai, (j0 + jj) * lda);
#pragma unroll
                for (int c = 0; c < KC; ++c) acc[c] = fma(a, Vs[jj][c], acc[c]);
            }
        }
    }
    double sq = 0.0;
    if (live) {
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            if (c < k) {
                const double r = acc[c] - ld(U, i + (int64_t)c * m) * sig[c];
                sq = fma(r, r, sq);
            }
        }
    }
    const double t = block_sum(sq, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Per block: sum over its columns j of sum_c (B(c, j) - V(j, c) s_c)^2 with
// B = U_k^T A (k x n, ld k, FP64).
template <typename TV>
__global__ __launch_bounds__(WT) void k_wedin_s(const double *__restrict__ B, const TV *__restrict__ V,
                                                const double *__restrict__ sig, int k, int64_t n,
                                                double *__restrict__ part)
{
    __shared__ double sh[WT / 64];
    const int64_t j = (int64_t)blockIdx.x * WT + threadIdx.x;
    double sq = 0.0;
    if (j < n) {
        for (int c = 0; c < k; ++c) {
            const double s = B[c + j * k] - ld(V, j + (int64_t)c * n) * sig[c];
            sq = fma(s, s, sq);
        }
    }
    const double t = block_sum(sq, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(WT) void k_to_f64(const float *__restrict__ x, int64_t cnt, double *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * WT + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * WT) y[i] = x[i];
}

// out = (||R||_F, ||S||_F, omega^, bound) from the block partials.
__global__ __launch_bounds__(WT) void k_wedin_final(const double *__restrict__ rp, int nr, const double *__restrict__ sp,
                                                    int ns, const double *__restrict__ sig, int k,
                                                    double *__restrict__ out)
{
    __shared__ double sh[WT / 64];
    double a = 0.0, b = 0.0;
    for (int q = threadIdx.x; q < nr; q += WT) a += rp[q];
    for (int q = threadIdx.x; q < ns; q += WT) b += sp[q];
    const double r2 = block_sum(a, sh);
    __syncthreads();
    const double s2 = block_sum(b, sh);
    if (threadIdx.x == 0) {
        const double sk = sig[k - 1], sk1 = sig[k];
        const double om = fmin(fabs(sk - sk1), sk);
        out[0] = sqrt(r2);
        out[1] = sqrt(s2);
        out[2] = om;
        out[3] = (om > 0.0) ? sqrt(r2 + s2) / om : INFINITY;
    }
}

template <int KC, typename TA, typename TV>
void launch_r(const pod_ctx *ctx, const void *V, const void *U, int k, double *part, unsigned nb)
{
    const pod_params &p = ctx->prm;
    hipLaunchKernelGGL((k_wedin_r<KC, TA, TV>), dim3(nb), dim3(WT), 0, ctx->st, (const TA *)ctx->A, p.m, p.n, p.lda,
                       (const TV *)V, (const TV *)U, (const double *)ctx->sigB, k, part);
}

template <typename TA, typename TV>
void launch_r_k(const pod_ctx *ctx, const void *V, const void *U, int k, double *part, unsigned nb)
{
    if (k <= 8) launch_r<8, TA, TV>(ctx, V, U, k, part, nb);
    else if (k <= 16) launch_r<16, TA, TV>(ctx, V, U, k, part, nb);
    else if (k <= 24) launch_r<24, TA, TV>(ctx, V, U, k, part, nb);
    else if (k <= 32) launch_r<32, TA, TV>(ctx, V, U, k, part, nb);
    else if (k <= 48) launch_r<48, TA, TV>(ctx, V, U, k, part, nb);
    else launch_r<64, TA, TV>(ctx, V, U, k, part, nb);
}

}  // namespace

#define WD_HIP(call)                                                                                                  \
    do {                                                                                                              \
        hipError_t e_ = (call);                                                                                       \
        if (e_ != hipSuccess) {                                                                                       \
            ctx->failed = 1;                                                                                          \
            return (e_ == hipErrorOutOfMemory) ? POD_ENOMEM : POD_EHIP;                                               \
        }                                                                                                             \
    } while (0)

extern "C" pod_status pod_wedin_bound(pod_ctx *ctx, const void *U_k, const void *V_k, double *out)
{
    if (!ctx || !U_k || !V_k || !out) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    if (ctx->pending) return POD_ESTATE;
    WD_HIP(hipMemcpyAsync(&ctx->hs, ctx->ds, sizeof(DevState), hipMemcpyDeviceToHost, ctx->st));
    WD_HIP(hipStreamSynchronize(ctx->st));
    // the Rayleigh-Ritz values of the last pod_project, taken after the last merge
    if (ctx->proj_k < 1 || ctx->proj_it != ctx->hs.it) return POD_ESTATE;
    const int k = ctx->proj_k;
    if (ctx->proj_rank <= k) return POD_EINVAL;   // omega^ needs sigma_{k+1}: r > k
    if (k > 64) return POD_EINVAL;
    const pod_params &p = ctx->prm;
    const bool f64 = p.precision == POD_F64;
    const unsigned nbr = (unsigned)((p.m + WT - 1) / WT), nbs = (unsigned)((p.n + WT - 1) / WT);
    const size_t need = (f64 ? 0 : (size_t)p.m * k) + (size_t)k * p.n + nbr + nbs + 4;
    if (need > ctx->qws_n) {
        if (ctx->qws) WD_HIP(hipFree(ctx->qws));
        ctx->qws = nullptr;
        ctx->qws_n = 0;
        WD_HIP(hipMalloc((void **)&ctx->qws, need * sizeof(double)));
        ctx->qws_n = need;
    }
    double *U64 = ctx->qws;
    double *Bk = U64 + (f64 ? 0 : (size_t)p.m * k);
    double *rpart = Bk + (size_t)k * p.n;
    double *spart = rpart + nbr;
    double *dout = spart + nbs;
    // R = A V_k - U_k Sigma_k
    if (f64) {
        if (p.a_dtype == POD_F64) launch_r_k<double, double>(ctx, V_k, U_k, k, rpart, nbr);
        else launch_r_k<float, double>(ctx, V_k, U_k, k, rpart, nbr);
    } else {
        launch_r_k<float, float>(ctx, V_k, U_k, k, rpart, nbr);
    }
    WD_HIP(hipGetLastError());
    // S = A^T U_k - V_k Sigma_k: B_k = U_k^T A in FP64
    const void *Uf = U_k;
    if (!f64) {
        const int64_t cnt = p.m * k;
        const unsigned nb = (unsigned)((cnt + WT - 1) / WT < 4096 ? (cnt + WT - 1) / WT : 4096);
        hipLaunchKernelGGL(k_to_f64, dim3(nb), dim3(WT), 0, ctx->st, (const float *)U_k, cnt, U64);
        WD_HIP(hipGetLastError());
        Uf = U64;
    }
    ProjArgs pa;
    pa.prec = POD_F64;
    pa.a_dtype = p.a_dtype;
    pa.m = p.m;
    pa.n = p.n;
    pa.lda = p.lda;
    pa.U = Uf;
    pa.A = ctx->A;
    pa.r = k;
    pa.Bpart = ctx->Bpart;   // nsplit x r x n >= nsplit x k x n
    pa.nsplit = ctx->nsplit;
    pa.B = Bk;
    WD_HIP(launch_project_partial(pa, ctx->st));
    WD_HIP(launch_project_reduce(pa, ctx->st));
    if (f64) {
        hipLaunchKernelGGL(k_wedin_s<double>, dim3(nbs), dim3(WT), 0, ctx->st, (const double *)Bk,
                           (const double *)V_k, (const double *)ctx->sigB, k, p.n, spart);
    } else {
        hipLaunchKernelGGL(k_wedin_s<float>, dim3(nbs), dim3(WT), 0, ctx->st, (const double *)Bk,
                           (const float *)V_k, (const double *)ctx->sigB, k, p.n, spart);
    }
    WD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_wedin_final, dim3(1), dim3(WT), 0, ctx->st, (const double *)rpart, (int)nbr,
                       (const double *)spart, (int)nbs, (const double *)ctx->sigB, k, dout);
    WD_HIP(hipGetLastError());
    WD_HIP(hipMemcpyAsync(out, dout, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->st));
    WD_HIP(hipStreamSynchronize(ctx->st));
    return POD_OK;
}

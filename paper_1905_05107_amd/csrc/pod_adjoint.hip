// pod_adjoint.hip -- reverse pass of the merge chain of Alg. 1 (ICS): the
// gradient with respect to A of a function of the merged modes (U_k, Sigma_k),
// the sampled columns held fixed.  The forward pass keeps, per merge, the
// basis and Sigma it started from and the merge factor R (small); the
// reverse pass recomputes the rest: per merge one Gram pass over
// [U_{t-1} | A(:, I_t) | Ubar_t], the small FP64 adjoint of the truncated thin
// SVD (k_adj_small; for merges wider than 64 columns k_adj_wide_eig and the
// k_adj_wide_step launches), and one pass writing Ubar_{t-1} and adding the adjoint of
// the sampled columns to dA(:, I_t).
#include <math.h>

#include <new>
#include <vector>

#include "pod_ctx.h"

using namespace pod;

namespace {

#define A_HIP(call)                                                                                                   \
    do {                                                                                                              \
        hipError_t e_ = (call);                                                                                       \
        if (e_ != hipSuccess) {                                                                                       \
            ctx->failed = 1;                                                                                          \
            return (e_ == hipErrorOutOfMemory) ? POD_ENOMEM : POD_EHIP;                                               \
        }                                                                                                             \
    } while (0)

template <typename TC>
__global__ __launch_bounds__(256) void k_ckpt_pre(const DevState *ds, const TC *U0, const TC *U1, const double *s0,
                                                  const double *s1, int64_t m, int32_t r, TC *ckU, double *ckS,
                                                  int32_t *meta, int32_t cap)
{
    if (merge_halted(ds)) return;
    const int32_t t = ds->it;
    if (t >= cap) return;
    const int32_t rs = ds->rs;
    const TC *U = (t & 1) ? U1 : U0;
    const double *sg = (t & 1) ? s1 : s0;
    TC *dst = ckU + (int64_t)t * m * r;
    const int64_t total = m * rs;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256)
        dst[idx] = U[idx];
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < rs; i += 256) ckS[(int64_t)t * r + i] = sg[i];
        if (threadIdx.x == 0) {
            meta[4 * t] = rs;
            meta[4 * t + 1] = ds->g;
            meta[4 * t + 3] = 0;
        }
    }
}

__global__ __launch_bounds__(256) void k_ckpt_post(const DevState *ds, const double *R, int32_t pm2, double *ckR,
                                                   int32_t *meta, int32_t cap)
{
    if (merge_halted(ds)) return;
    const int32_t t = ds->it - 1;
    if (t < 0 || t >= cap) return;
    for (int i = threadIdx.x; i < pm2; i += 256) ckR[(int64_t)t * pm2 + i] = R[i];
    if (threadIdx.x == 0) {
        meta[4 * t + 2] = ds->rnew;
        meta[4 * t + 3] = 1;
    }
}

// Row-sampled merge about to run (merge ds->it): its right factor V_u
// (g x r_u, ld pm), the scales and distinct rows of its row draw, and (r_u, h).
__global__ __launch_bounds__(256) void k_ckpt_rows(const DevState *ds, const double *Vt, const double *sc,
                                                   const int32_t *rows, int32_t pm, int32_t w, double *ckV,
                                                   double *ckSc, int32_t *ckRows, int32_t *ckRH, int32_t cap)
{
    if (merge_halted(ds)) return;
    const int32_t t = ds->it;
    if (t >= cap) return;
    const int32_t g = ds->g, ru = ds->ru, h = ds->h;
    double *v = ckV + (int64_t)t * pm * pm;
    for (int idx = threadIdx.x; idx < g * ru; idx += 256) {
        const int i = idx % g, j = idx / g;
        v[i + j * pm] = Vt[i + j * pm];
    }
    for (int q = threadIdx.x; q < h; q += 256) {
        ckSc[(int64_t)t * w + q] = sc[q];
        ckRows[(int64_t)t * w + q] = rows[q];
    }
    if (threadIdx.x == 0) {
        ckRH[2 * t] = ru;
        ckRH[2 * t + 1] = h;
    }
}

__global__ void k_adj_state(DevState *ds, int32_t rs, int32_t g)
{
    ds->rs = rs;
    ds->g = g;
    ds->it = 0;
    ds->exhausted = 0;
    ds->done = 0;
}

struct AdjStateArg {
    DevState *ds;
    int32_t rs, g;
};
// Batched: entry blockIdx.x.
__global__ void k_adj_state_b(const AdjStateArg *__restrict__ arr)
{
    const AdjStateArg a = arr[blockIdx.x];
    if (threadIdx.x == 0) {
        a.ds->rs = a.rs;
        a.ds->g = a.g;
        a.ds->it = 0;
        a.ds->exhausted = 0;
        a.ds->done = 0;
    }
}

// L = |A - U_k B|_F^2 (B = U_k^T A), dA = 2 (A - U_k B), Ubar = -2 (A - U_k B) B^T.
// One thread per row, columns in order; per-workgroup loss partials.
template <typename TC, typename TA, int KM>
__global__ __launch_bounds__(256) void k_loss_resid(const TA *__restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                    const TC *__restrict__ U, int32_t k, const double *__restrict__ B,
                                                    TC *__restrict__ dA, TC *__restrict__ Ubar,
                                                    double *__restrict__ lossp)
{
    __shared__ double sw[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double u[KM], acc[KM];
    // (loads without branches, from index 0 where out of range, so that they
    // are in flight together)
#pragma unroll
    for (int l = 0; l < KM; ++l) {
        const bool ok = i < m && l < k;
        const TC v = U[ok ? (int64_t)l * m + i : 0];
        u[l] = ok ? (double)v : 0.0;
        acc[l] = 0.0;
    }
    double L = 0.0;
    if (i < m) {
        // A(i, j) read four columns ahead of its use
        constexpr int AH = 4;
        double ah[AH];
#pragma unroll
        for (int q = 0; q < AH; ++q) ah[q] = (q < n) ? (double)A[(int64_t)q * lda + i] : 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double aij = ah[0];
#pragma unroll
            for (int q = 0; q + 1 < AH; ++q) ah[q] = ah[q + 1];
            const int64_t jn = (j + AH < n) ? j + AH : n - 1;
            ah[AH - 1] = (double)A[jn * lda + i];
            const double *b = B + j * k;
            double pr = 0.0;
#pragma unroll
            for (int l = 0; l < KM; ++l)
                if (l < k) pr += u[l] * b[l];
            const double R = aij - pr;
            dA[j * m + i] = (TC)(2.0 * R);
            L += R * R;
#pragma unroll
            for (int l = 0; l < KM; ++l)
                if (l < k) acc[l] += R * b[l];
        }
#pragma unroll
        for (int l = 0; l < KM; ++l)
            if (l < k) Ubar[(int64_t)l * m + i] = (TC)(-2.0 * acc[l]);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) L += __shfl_xor(L, o, 64);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = L;
    __syncthreads();
    if (threadIdx.x == 0) lossp[blockIdx.x] = ((sw[0] + sw[1]) + sw[2]) + sw[3];
}

// The same for k > 16 on the FP64 matrix cores: B U_k^T and R B^T are dense
// contractions (2 m n k flops each).  A workgroup of 8 waves takes 256 rows
// (the loss partial of k_loss_resid's layout); wave w its two 16-row tiles
// (two independent product chains), U_k of its rows held in the B-operand
// layout (lane l: row l % 16, k = 4 s + l / 16).  Per 16-column chunk c:
//   S = B(:, c)^T U_k(rows, :)^T   (16 x 16, k in steps of 4),
//   R^T = A(rows, c)^T - S, dA(rows, c) = 2 R, L += |R|^2,
//   Ubar(rows, :)^T += B(:, c) R(rows, c)^T (k in tiles of 16),
// where the FP64 accumulator layout of S (lane l: column l / 16 + 4 v of the
// chunk, row l % 16) is the B-operand layout of the second product; k is
// padded to 64 with zero operands.  B is
// staged in LDS 64 columns at a time (column-major, padded); loads of A,
// clamped into range, carry no branch.
constexpr int LM_NT = 512, LM_NC = 64, LM_LDB = 65;
template <typename TC, typename TA>
__global__ __launch_bounds__(LM_NT) void k_loss_mfma(const TA *__restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                     const TC *__restrict__ U, int32_t k,
                                                     const double *__restrict__ B, TC *__restrict__ dA,
                                                     TC *__restrict__ Ubar, double *__restrict__ lossp)
{
    __shared__ double Bs[LM_NC * LM_LDB];
    __shared__ double sw[LM_NT / 64];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = l & 15, lk = l >> 4;
    int64_t row[2];
    bool rin[2];
    double u[2][16];
    v4d ub[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        row[t] = (int64_t)blockIdx.x * 256 + w * 32 + t * 16 + li;
        rin[t] = row[t] < m;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int kk = 4 * s + lk;
            const bool ok = rin[t] && kk < k;
            const TC v = U[ok ? (int64_t)kk * m + row[t] : 0];
            u[t][s] = ok ? (double)v : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) ub[t][q] = v4d{0.0, 0.0, 0.0, 0.0};
    }
    const int64_t rc[2] = {rin[0] ? row[0] : 0, rin[1] ? row[1] : 0};
    double L = 0.0;
    for (int64_t c0 = 0; c0 < n; c0 += LM_NC) {
        __syncthreads();
        for (int e = threadIdx.x; e < LM_NC * 64; e += LM_NT) {
            const int cc = e >> 6, kk = e & 63;
            const bool ok = c0 + cc < n && kk < k;
            const double v = B[ok ? (c0 + cc) * k + kk : 0];
            Bs[cc * LM_LDB + kk] = ok ? v : 0.0;
        }
        __syncthreads();
        const int nch = (int)(((n - c0 < LM_NC) ? n - c0 : LM_NC) + 15) >> 4;
        for (int ch = 0; ch < nch; ++ch) {
            const int cb = ch * 16;
            // A of the four columns l / 16 + 4 v of the chunk, for both row tiles
            TA av[2][4];
            bool cin[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t col = c0 + cb + lk + 4 * v;
                cin[v] = col < n;
                const int64_t cl = cin[v] ? col : 0;
#pragma unroll
                for (int t = 0; t < 2; ++t) av[t][v] = A[cl * lda + rc[t]];
            }
            v4d S[2] = {v4d{0.0, 0.0, 0.0, 0.0}, v4d{0.0, 0.0, 0.0, 0.0}};
            const double *ba = Bs + (cb + li) * LM_LDB + lk;
#pragma unroll
            for (int s = 0; s < 16; ++s) {   // (zero operands past k)
                const double a = ba[4 * s];
#pragma unroll
                for (int t = 0; t < 2; ++t) S[t] = mfma16x16x4(a, u[t][s], S[t]);
            }
            v4d R[2];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double r = (rin[t] && cin[v]) ? (double)av[t][v] - S[t][v] : 0.0;
                    R[t][v] = r;
                    L += r * r;
                }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (rin[t] && cin[v]) dA[(c0 + cb + lk + 4 * v) * m + row[t]] = (TC)(2.0 * R[t][v]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double *bb = Bs + (cb + lk) * LM_LDB + 16 * q + li;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const double a = bb[4 * s * LM_LDB];
#pragma unroll
                    for (int t = 0; t < 2; ++t) ub[t][q] = mfma16x16x4(a, R[t][s], ub[t][q]);
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int kk = 16 * q + lk + 4 * v;
                if (rin[t] && kk < k) Ubar[(int64_t)kk * m + row[t]] = (TC)(-2.0 * ub[t][q][v]);
            }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) L += __shfl_xor(L, o, 64);
    if (l == 0) sw[w] = L;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < LM_NT / 64; ++q) t += sw[q];
        lossp[blockIdx.x] = t;
    }
}

template <typename TC, typename TA>
hipError_t loss_resid_launch(const void *A, int64_t lda, int64_t m, int64_t n, const void *U, int32_t k,
                             const double *B, void *dA, void *Ubar, double *lossp, hipStream_t st)
{
    const unsigned nb = (unsigned)((m + 255) / 256);
    if (k <= 16)
        hipLaunchKernelGGL((k_loss_resid<TC, TA, 16>), dim3(nb), dim3(256), 0, st, (const TA *)A, lda, m, n,
                           (const TC *)U, k, B, (TC *)dA, (TC *)Ubar, lossp);
    else if (k <= 64)
        hipLaunchKernelGGL((k_loss_mfma<TC, TA>), dim3(nb), dim3(LM_NT), 0, st, (const TA *)A, lda, m, n,
                           (const TC *)U, k, B, (TC *)dA, (TC *)Ubar, lossp);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// The reverse pass from (Ubar[0], sbar[0]) holding the adjoints of the final
// merged state (all of its columns); dA accumulates.
pod_status reverse_merges(pod_ctx *ctx, void *dA)
{
    const pod_params &p = ctx->prm;
    const int32_t T = ctx->hs.it;
    std::vector<int32_t> meta(4 * (size_t)(T > 0 ? T : 1)), off(T + 1);
    if (T < 1) return POD_OK;
    if (ctx->ck_lost || T > ctx->ck_cap) return POD_ENOMEM;   // merges without checkpoints
    A_HIP(hipMemcpy(meta.data(), ctx->ckMeta, sizeof(int32_t) * 4 * T, hipMemcpyDeviceToHost));
    A_HIP(hipMemcpy(off.data(), ctx->col_log_off, sizeof(int32_t) * (T + 1), hipMemcpyDeviceToHost));
    for (int32_t t = 0; t < T; ++t)
        if (meta[4 * t + 3] != 1) return POD_ESTATE;
    const bool rowm = p.w > 0;
    std::vector<int32_t> rh(rowm ? 2 * (size_t)T : 0);
    if (rowm) A_HIP(hipMemcpy(rh.data(), ctx->ckRH, sizeof(int32_t) * 2 * T, hipMemcpyDeviceToHost));
    const size_t esz = ctx->esz;
    const double eta = (p.precision == POD_F64) ? 1e-12 : 1e-6;
    int cur = 0;
    for (int32_t t = T - 1; t >= 0; --t) {
        const int32_t rs = meta[4 * t], g = meta[4 * t + 1], rz = meta[4 * t + 2];
        const int32_t P = rs + g, Pext = P + rz;
        hipLaunchKernelGGL(k_adj_state, dim3(1), dim3(1), 0, ctx->st, ctx->dsb, rs, g);
        A_HIP(hipGetLastError());
        GemmDesc gd;
        gd.prec = (p.precision == POD_F64) ? POD_F64 : POD_F32;
        gd.a_dtype = p.a_dtype;
        gd.m = p.m;
        gd.U = (const unsigned char *)ctx->ckU + (size_t)t * p.m * ctx->r * esz;
        gd.U1 = nullptr;
        gd.A = ctx->A;
        gd.lda = p.lda;
        gd.cols = ctx->col_log + off[t];
        gd.Y = nullptr;
        gd.gather = 1;
        gd.guard = 0;
        gd.Z = ctx->Ubar[cur];
        A_HIP(launch_gram_partial(gd, ctx->dsb, Pext, ctx->pb, ctx->partb, ctx->nblk, ctx->st));
        A_HIP(launch_gram_reduce_sel(ctx->partb, ctx->nblk, ctx->pb, ctx->dsb, Pext, ctx->Gext, ctx->st));
        AdjArgs aa;
        aa.Gext = ctx->Gext;
        aa.pb = ctx->pb;
        aa.R = ctx->ckR + (size_t)t * ctx->pmax * ctx->pmax;
        aa.pm = ctx->pmax;
        aa.sig = ctx->ckS + (size_t)t * ctx->r;
        aa.sbar_in = ctx->sbar[cur];
        aa.sbar_out = ctx->sbar[cur ^ 1];
        aa.Wt = ctx->Wt;
        aa.prec = p.precision;
        aa.ws = ctx->adj_ws;
        aa.rs = rs;
        aa.g = g;
        aa.rz = rz;
        aa.eta = eta;
        AdjRowsArgs ra;
        const int32_t pm = ctx->pmax;
        if (rowm) {
            // merge t ran on X0 P with P = blkdiag(Sigma, V_u): the eigenbasis of
            // G = W^T W first, for the adjoint of V_u
            const int32_t ru = rh[2 * t], h = rh[2 * t + 1];
            if (rs + ru > pm || h > p.w) return POD_ESTATE;
            ra.A = ctx->A;
            ra.a_dtype = p.a_dtype;
            ra.lda = p.lda;
            ra.cols = ctx->col_log + off[t];
            ra.rows = ctx->ckRows + (size_t)t * p.w;
            ra.scales = ctx->ckSc + (size_t)t * p.w;
            ra.vt = ctx->ckV + (size_t)t * pm * pm;
            ra.g = g;
            ra.h = h;
            ra.ru = ru;
            ra.pm = pm;
            ra.vfull = ctx->adj_rows;
            ra.gbar = ctx->adj_rows + (size_t)pm * pm;
            ra.lam = ctx->adj_rows + 2 * (size_t)pm * pm;
            ra.dA = dA;
            ra.ldd = p.m;
            ra.prec = p.precision;
            if (ru > 0) A_HIP(launch_adj_rows_eig(ra, ctx->st));
            aa.vt = ra.vt;
            aa.ru = ru;
            aa.vfull = ra.vfull;
            aa.lam = ra.lam;
            aa.gbar = ctx->adj_rows + (size_t)pm * pm;
        }
        if (ctx->pmax > SMALL_LDS_P) A_HIP(launch_adj_wide(aa, ctx->st));
        else A_HIP(launch_adj_small(aa, ctx->st));
        A_HIP(launch_gemm_tall_scatter(gd, ctx->dsb, Pext, P, Pext, P, ctx->Wt, ctx->pb, ctx->Ubar[cur ^ 1], rs,
                                       ctx->col_log + off[t], dA, p.m, ctx->st));
        // the part of dA(rows, cols) through G = W^T W
        if (rowm && ra.ru > 0) A_HIP(launch_adj_rows_update(ra, ctx->st));
        cur ^= 1;
    }
    A_HIP(hipStreamSynchronize(ctx->st));
    return POD_OK;
}

// Batched checkpoints: one entry per matrix (blockIdx.y), stopped matrices skipped.
template <typename TC>
__global__ __launch_bounds__(256) void k_ckpt_pre_b(const CkptArgs *__restrict__ arr)
{
    const CkptArgs &a = arr[blockIdx.y];
    if (a.ds->done) return;
    const DevState *ds = a.ds;
    if (merge_halted(ds)) return;
    const int32_t t = ds->it;
    if (t >= a.cap) return;
    const int32_t rs = ds->rs;
    const TC *U = reinterpret_cast<const TC *>((t & 1) ? a.U1 : a.U0);
    const double *sg = (t & 1) ? a.s1 : a.s0;
    TC *dst = reinterpret_cast<TC *>(a.ckU) + (int64_t)t * a.m * a.r;
    const int64_t total = a.m * rs;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256)
        dst[idx] = U[idx];
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < rs; i += 256) a.ckS[(int64_t)t * a.r + i] = sg[i];
        if (threadIdx.x == 0) {
            a.meta[4 * t] = rs;
            a.meta[4 * t + 1] = ds->g;
            a.meta[4 * t + 3] = 0;
        }
    }
}

__global__ __launch_bounds__(256) void k_ckpt_post_b(const CkptArgs *__restrict__ arr)
{
    const CkptArgs &a = arr[blockIdx.y];
    if (a.ds->done) return;
    const DevState *ds = a.ds;
    if (merge_halted(ds)) return;
    const int32_t t = ds->it - 1;
    if (t < 0 || t >= a.cap) return;
    for (int i = threadIdx.x; i < a.pm2; i += 256) a.ckR[(int64_t)t * a.pm2 + i] = a.R[i];
    if (threadIdx.x == 0) {
        a.meta[4 * t + 2] = ds->rnew;
        a.meta[4 * t + 3] = 1;
    }
}

}  // namespace

// The reverse passes of many runs together (a batch; every run with merge
// widths p + r <= 64 and one stream): reverse step s takes merge T_i - 1 - s of
// every run i that has one, and each of the five launches of a step covers all
// of those runs at once (blockIdx selects the run).  Per run the kernels, their
// arguments and their order are those of reverse_merges, so the gradients are
// the same bit for bit; only the runs' small stages now share the GPU.
pod_status pod::reverse_merges_batch(pod_ctx *const *ctxs, int32_t count, void *const *dA, hipStream_t st)
{
    struct Run {
        std::vector<int32_t> meta, off;
        int32_t T;
    };
    std::vector<Run> run(count);
    int32_t maxT = 0, pb_max = 0, max_nblk = 0, max_nb = 0, p_max = 0;
    const int32_t prec = ctxs[0]->prm.precision;
    for (int32_t i = 0; i < count; ++i) {
        pod_ctx *ctx = ctxs[i];
        Run &R = run[i];
        R.T = ctx->hs.it;
        if (ctx->prm.precision != prec || ctx->pb > 64 || ctx->pmax > 64 || ctx->prm.w != 0) return POD_EINVAL;
        if (R.T < 1) continue;
        if (ctx->ck_lost || R.T > ctx->ck_cap) return POD_ENOMEM;
        R.meta.resize(4 * (size_t)R.T);
        R.off.resize(R.T + 1);
        A_HIP(hipMemcpy(R.meta.data(), ctx->ckMeta, sizeof(int32_t) * 4 * R.T, hipMemcpyDeviceToHost));
        A_HIP(hipMemcpy(R.off.data(), ctx->col_log_off, sizeof(int32_t) * (R.T + 1), hipMemcpyDeviceToHost));
        for (int32_t t = 0; t < R.T; ++t)
            if (R.meta[4 * t + 3] != 1) return POD_ESTATE;
        maxT = (R.T > maxT) ? R.T : maxT;
        pb_max = (ctx->pb > pb_max) ? ctx->pb : pb_max;
        p_max = (ctx->pmax > p_max) ? ctx->pmax : p_max;
        max_nblk = (ctx->nblk > max_nblk) ? ctx->nblk : max_nblk;
        const int32_t nb = tall_blocks(ctx->prm.m);
        max_nb = (nb > max_nb) ? nb : max_nb;
    }
    if (maxT < 1) return POD_OK;
    // every step's arguments, built on the host and uploaded once
    std::vector<AdjStateArg> hs;
    std::vector<GramArgs> hg;
    std::vector<AdjArgs> ha;
    std::vector<ScatterArgs> hc;
    std::vector<int32_t> first(maxT + 1, 0);
    const double eta = (prec == POD_F64) ? 1e-12 : 1e-6;
    for (int32_t sidx = 0; sidx < maxT; ++sidx) {
        first[sidx] = (int32_t)hs.size();
        const int cur = sidx & 1;
        for (int32_t i = 0; i < count; ++i) {
            pod_ctx *ctx = ctxs[i];
            const Run &R = run[i];
            const int32_t t = R.T - 1 - sidx;
            if (t < 0) continue;
            const pod_params &p = ctx->prm;
            const int32_t rs = R.meta[4 * t], g = R.meta[4 * t + 1], rz = R.meta[4 * t + 2];
            const int32_t P = rs + g, Pext = P + rz;
            if (P > ctx->pmax) return POD_ESTATE;
            hs.push_back(AdjStateArg{ctx->dsb, rs, g});
            GemmDesc gd;
            gd.prec = (p.precision == POD_F64) ? POD_F64 : POD_F32;
            gd.a_dtype = p.a_dtype;
            gd.m = p.m;
            gd.U = (const unsigned char *)ctx->ckU + (size_t)t * p.m * ctx->r * ctx->esz;
            gd.U1 = nullptr;
            gd.A = ctx->A;
            gd.lda = p.lda;
            gd.cols = ctx->col_log + R.off[t];
            gd.Y = nullptr;
            gd.gather = 1;
            gd.guard = 0;
            gd.Z = ctx->Ubar[cur];
            GramArgs ga;
            ga.d = gd;
            ga.ds = ctx->dsb;
            ga.which_p = Pext;
            ga.pmax = ctx->pb;
            ga.nblk = ctx->nblk;
            ga.vec = gemm_vec_ok(gd);
            ga.part = ctx->partb;
            ga.G = ctx->Gext;
            hg.push_back(ga);
            AdjArgs aa;
            aa.Gext = ctx->Gext;
            aa.pb = ctx->pb;
            aa.R = ctx->ckR + (size_t)t * ctx->pmax * ctx->pmax;
            aa.pm = ctx->pmax;
            aa.sig = ctx->ckS + (size_t)t * ctx->r;
            aa.sbar_in = ctx->sbar[cur];
            aa.sbar_out = ctx->sbar[cur ^ 1];
            aa.Wt = ctx->Wt;
            aa.prec = p.precision;
            aa.ws = ctx->adj_ws;
            aa.rs = rs;
            aa.g = g;
            aa.rz = rz;
            aa.eta = eta;
            ha.push_back(aa);
            ScatterArgs sa;
            sa.d = gd;
            sa.ds = ctx->dsb;
            sa.which_in = Pext;
            sa.which_out = P;
            sa.T = ctx->Wt;
            sa.ldt = ctx->pb;
            sa.Yout = ctx->Ubar[cur ^ 1];
            sa.split = rs;
            sa.cmap = ctx->col_log + R.off[t];
            sa.D = dA[i];
            sa.ldd = p.m;
            sa.vec = gemm_vec_ok(gd);
            sa.nb = tall_blocks(p.m);
            hc.push_back(sa);
        }
    }
    first[maxT] = (int32_t)hs.size();
    const size_t ne = hs.size();
    AdjStateArg *ds_ = nullptr;
    GramArgs *dg = nullptr;
    AdjArgs *da = nullptr;
    ScatterArgs *dc = nullptr;
    hipError_t e = hipMalloc((void **)&ds_, sizeof(AdjStateArg) * ne);
    if (e == hipSuccess) e = hipMalloc((void **)&dg, sizeof(GramArgs) * ne);
    if (e == hipSuccess) e = hipMalloc((void **)&da, sizeof(AdjArgs) * ne);
    if (e == hipSuccess) e = hipMalloc((void **)&dc, sizeof(ScatterArgs) * ne);
    if (e == hipSuccess) e = hipMemcpy(ds_, hs.data(), sizeof(AdjStateArg) * ne, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dg, hg.data(), sizeof(GramArgs) * ne, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(da, ha.data(), sizeof(AdjArgs) * ne, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dc, hc.data(), sizeof(ScatterArgs) * ne, hipMemcpyHostToDevice);
    for (int32_t sidx = 0; sidx < maxT && e == hipSuccess; ++sidx) {
        const int32_t f = first[sidx], cnt = first[sidx + 1] - f;
        if (cnt < 1) continue;
        hipLaunchKernelGGL(k_adj_state_b, dim3((unsigned)cnt), dim3(64), 0, st, ds_ + f);
        e = hipGetLastError();
        if (e == hipSuccess) e = launch_gram_partial_b(dg + f, cnt, max_nblk, pb_max, prec, st);
        if (e == hipSuccess) e = launch_gram_reduce_b(dg + f, cnt, pb_max, st);
        if (e == hipSuccess) e = launch_adj_small_b(da + f, cnt, st);
        if (e == hipSuccess) e = launch_gemm_tall_scatter_b(dc + f, cnt, max_nb, pb_max, p_max, prec, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(ds_);
    (void)hipFree(dg);
    (void)hipFree(da);
    (void)hipFree(dc);
    return (e == hipSuccess) ? POD_OK : POD_EHIP;
}


hipError_t pod::launch_ckpt_pre(pod_ctx *ctx, hipStream_t st)
{
    const int64_t m = ctx->prm.m;
    const unsigned nb = (unsigned)(((m * ctx->r + 255) / 256 < 1024) ? (m * ctx->r + 255) / 256 : 1024);
    if (ctx->esz == 8)
        hipLaunchKernelGGL(k_ckpt_pre<double>, dim3(nb > 0 ? nb : 1), dim3(256), 0, st, ctx->ds,
                           (const double *)ctx->U[0], (const double *)ctx->U[1], ctx->sig[0], ctx->sig[1], m, ctx->r,
                           (double *)ctx->ckU, ctx->ckS, ctx->ckMeta, ctx->ck_cap);
    else
        hipLaunchKernelGGL(k_ckpt_pre<float>, dim3(nb > 0 ? nb : 1), dim3(256), 0, st, ctx->ds,
                           (const float *)ctx->U[0], (const float *)ctx->U[1], ctx->sig[0], ctx->sig[1], m, ctx->r,
                           (float *)ctx->ckU, ctx->ckS, ctx->ckMeta, ctx->ck_cap);
    return hipGetLastError();
}

hipError_t pod::launch_ckpt_rows(pod_ctx *ctx, hipStream_t st)
{
    hipLaunchKernelGGL(k_ckpt_rows, dim3(1), dim3(256), 0, st, ctx->ds, ctx->Vt, ctx->rscale, ctx->rows, ctx->pmax,
                       ctx->prm.w, ctx->ckV, ctx->ckSc, ctx->ckRows, ctx->ckRH, ctx->ck_cap);
    return hipGetLastError();
}

hipError_t pod::launch_ckpt_post(pod_ctx *ctx, hipStream_t st)
{
    hipLaunchKernelGGL(k_ckpt_post, dim3(1), dim3(256), 0, st, ctx->ds, ctx->R2, ctx->pmax * ctx->pmax, ctx->ckR,
                       ctx->ckMeta, ctx->ck_cap);
    return hipGetLastError();
}

CkptArgs pod::ctx_ckpt_args(pod_ctx *ctx)
{
    CkptArgs a;
    a.ds = ctx->ds;
    a.U0 = ctx->U[0];
    a.U1 = ctx->U[1];
    a.s0 = ctx->sig[0];
    a.s1 = ctx->sig[1];
    a.m = ctx->prm.m;
    a.r = ctx->r;
    a.ckU = ctx->ckU;
    a.ckS = ctx->ckS;
    a.ckR = ctx->ckR;
    a.R = ctx->R2;
    a.meta = ctx->ckMeta;
    a.cap = ctx->ck_cap;
    a.pm2 = ctx->pmax * ctx->pmax;
    return a;
}

hipError_t pod::launch_ckpt_pre_b(const CkptArgs *arr, int32_t count, int64_t max_mr, int32_t prec, hipStream_t st)
{
    const unsigned nb = (unsigned)(((max_mr + 255) / 256 < 1024) ? (max_mr + 255) / 256 : 1024);
    const dim3 grid(nb > 0 ? nb : 1, (unsigned)count);
    if (prec == POD_F64)
        hipLaunchKernelGGL(k_ckpt_pre_b<double>, grid, dim3(256), 0, st, arr);
    else
        hipLaunchKernelGGL(k_ckpt_pre_b<float>, grid, dim3(256), 0, st, arr);
    return hipGetLastError();
}

hipError_t pod::launch_ckpt_post_b(const CkptArgs *arr, int32_t count, hipStream_t st)
{
    hipLaunchKernelGGL(k_ckpt_post_b, dim3(1, (unsigned)count), dim3(256), 0, st, arr);
    return hipGetLastError();
}

pod_status pod::ckpt_reserve(pod_ctx *ctx, int32_t need)
{
    if (need > ctx->ck_max) need = ctx->ck_max;
    if (need <= ctx->ck_cap) return POD_OK;
    int32_t cap = 2 * ctx->ck_cap;
    if (cap < need) cap = need;
    if (cap > ctx->ck_max) cap = ctx->ck_max;
    const size_t mr = (size_t)ctx->prm.m * ctx->r, r = (size_t)ctx->r, pm2 = (size_t)ctx->pmax * ctx->pmax;
    const size_t w = (size_t)ctx->prm.w;
    void *nU = nullptr;
    double *nS = nullptr, *nR = nullptr, *nV = nullptr, *nSc = nullptr;
    int32_t *nM = nullptr, *nRH = nullptr, *nRows = nullptr;
    hipError_t e = hipMalloc(&nU, (size_t)cap * mr * ctx->esz + 16);
    if (e == hipSuccess) e = hipMalloc((void **)&nS, sizeof(double) * cap * r + 16);
    if (e == hipSuccess) e = hipMalloc((void **)&nR, sizeof(double) * cap * pm2 + 16);
    if (e == hipSuccess) e = hipMalloc((void **)&nM, sizeof(int32_t) * 4 * cap + 16);
    if (w > 0) {
        if (e == hipSuccess) e = hipMalloc((void **)&nV, sizeof(double) * cap * pm2 + 16);
        if (e == hipSuccess) e = hipMalloc((void **)&nSc, sizeof(double) * cap * w + 16);
        if (e == hipSuccess) e = hipMalloc((void **)&nRows, sizeof(int32_t) * cap * w + 16);
        if (e == hipSuccess) e = hipMalloc((void **)&nRH, sizeof(int32_t) * 2 * cap + 16);
    }
    if (e != hipSuccess) {
        (void)hipFree(nU);
        (void)hipFree(nS);
        (void)hipFree(nR);
        (void)hipFree(nM);
        (void)hipFree(nV);
        (void)hipFree(nSc);
        (void)hipFree(nRows);
        (void)hipFree(nRH);
        (void)hipGetLastError();
        if (e != hipErrorOutOfMemory) ctx->failed = 1;
        return (e == hipErrorOutOfMemory) ? POD_ENOMEM : POD_EHIP;
    }
    const size_t old = (size_t)ctx->ck_cap;
    if (e == hipSuccess) e = hipMemsetAsync(nM, 0, sizeof(int32_t) * 4 * cap, ctx->st);
    if (old > 0) {
        // checkpoints written by merges already enqueued land in the old
        // buffers before these stream-ordered copies
        if (e == hipSuccess) e = hipMemcpyAsync(nU, ctx->ckU, old * mr * ctx->esz, hipMemcpyDeviceToDevice, ctx->st);
        if (e == hipSuccess) e = hipMemcpyAsync(nS, ctx->ckS, sizeof(double) * old * r, hipMemcpyDeviceToDevice, ctx->st);
        if (e == hipSuccess) e = hipMemcpyAsync(nR, ctx->ckR, sizeof(double) * old * pm2, hipMemcpyDeviceToDevice, ctx->st);
        if (e == hipSuccess) e = hipMemcpyAsync(nM, ctx->ckMeta, sizeof(int32_t) * 4 * old, hipMemcpyDeviceToDevice, ctx->st);
        if (w > 0) {
            if (e == hipSuccess) e = hipMemcpyAsync(nV, ctx->ckV, sizeof(double) * old * pm2, hipMemcpyDeviceToDevice, ctx->st);
            if (e == hipSuccess) e = hipMemcpyAsync(nSc, ctx->ckSc, sizeof(double) * old * w, hipMemcpyDeviceToDevice, ctx->st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(nRows, ctx->ckRows, sizeof(int32_t) * old * w, hipMemcpyDeviceToDevice, ctx->st);
            if (e == hipSuccess) e = hipMemcpyAsync(nRH, ctx->ckRH, sizeof(int32_t) * 2 * old, hipMemcpyDeviceToDevice, ctx->st);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
    if (e != hipSuccess) {
        ctx->failed = 1;
        return POD_EHIP;
    }
    (void)hipFree(ctx->ckU);
    (void)hipFree(ctx->ckS);
    (void)hipFree(ctx->ckR);
    (void)hipFree(ctx->ckMeta);
    (void)hipFree(ctx->ckV);
    (void)hipFree(ctx->ckSc);
    (void)hipFree(ctx->ckRows);
    (void)hipFree(ctx->ckRH);
    ctx->ckU = nU;
    ctx->ckS = nS;
    ctx->ckR = nR;
    ctx->ckMeta = nM;
    ctx->ckV = nV;
    ctx->ckSc = nSc;
    ctx->ckRows = nRows;
    ctx->ckRH = nRH;
    ctx->ck_cap = cap;
    return POD_OK;
}

extern "C" {

pod_status pod_enable_adjoint(pod_ctx *ctx)
{
    if (!ctx) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    if (ctx->merges > 0 || ctx->pending) return POD_ESTATE;
    const pod_params &p = ctx->prm;
    // row-sampled merges: p <= 64; column draws: p <= 160, p + r <= 208
    if (p.r_update != 0 || (p.w > 0 && ctx->pmax > SMALL_LDS_P)) return POD_EINVAL;
    if (ctx->ckU) return POD_OK;
    // widest reverse-step block [U | A(:, I) | Ubar]: r + min(c, n) + r columns
    const int64_t cmax = (p.c < p.n) ? p.c : p.n;
    const int32_t pb = (int32_t)(((2 * (int64_t)ctx->r + cmax) + 15) & ~15);
    if (pb > 208) return POD_EINVAL;
    ctx->pb = pb;
    // checkpoints for about twice the merges a run takes when every draw is
    // distinct (n / c); later merges grow them (ckpt_reserve)
    ctx->ck_max = (int32_t)((p.max_iter < ctx->n_cap) ? p.max_iter : ctx->n_cap) + 1;
    const int64_t guess = 2 * ((ctx->n_cap + p.c - 1) / p.c) + 8;
    ctx->ck_cap = 0;
    ctx->ck_lost = 0;
    const size_t m = (size_t)p.m, r = (size_t)ctx->r, pm2 = (size_t)ctx->pmax * ctx->pmax;
    hipError_t e = hipSuccess;
    auto al = [&](void **q, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(q, bytes + 16);
    };
    al((void **)&ctx->dsb, sizeof(DevState));
    al((void **)&ctx->partb, sizeof(double) * (size_t)ctx->nblk * pb * pb);
    al((void **)&ctx->Gext, sizeof(double) * (size_t)pb * pb);
    al((void **)&ctx->adj_ws, sizeof(double) * ((ctx->pmax > SMALL_LDS_P) ? adj_wide_ws_doubles(ctx->pmax) : 12 * pm2));
    if (p.w > 0) al((void **)&ctx->adj_rows, sizeof(double) * (2 * pm2 + (size_t)ctx->pmax));
    al((void **)&ctx->sbar[0], sizeof(double) * r);
    al((void **)&ctx->sbar[1], sizeof(double) * r);
    al((void **)&ctx->lossp, sizeof(double) * ((m + 255) / 256));
    al(&ctx->Wt, (size_t)pb * ctx->pmax * ctx->esz);
    al(&ctx->Ubar[0], m * r * ctx->esz);
    al(&ctx->Ubar[1], m * r * ctx->esz);
    pod_status s = (e == hipSuccess) ? POD_OK : (e == hipErrorOutOfMemory) ? POD_ENOMEM : POD_EHIP;
    if (s == POD_OK) s = ckpt_reserve(ctx, (int32_t)(guess < ctx->ck_max ? guess : ctx->ck_max));
    if (s == POD_OK && ctx->ckU) return POD_OK;
    // the forward run stays usable: release what was taken
    void *ptrs[] = {ctx->dsb, ctx->partb, ctx->Gext, ctx->adj_ws, ctx->sbar[0], ctx->sbar[1], ctx->lossp,
                    ctx->Wt, ctx->Ubar[0], ctx->Ubar[1], ctx->ckU, ctx->ckS, ctx->ckR, ctx->ckMeta,
                    ctx->adj_rows, ctx->ckV, ctx->ckSc, ctx->ckRows, ctx->ckRH};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    ctx->dsb = nullptr;
    ctx->partb = ctx->Gext = ctx->adj_ws = ctx->sbar[0] = ctx->sbar[1] = ctx->lossp = nullptr;
    ctx->Wt = ctx->Ubar[0] = ctx->Ubar[1] = ctx->ckU = nullptr;
    ctx->ckS = ctx->ckR = ctx->adj_rows = ctx->ckV = ctx->ckSc = nullptr;
    ctx->ckMeta = ctx->ckRows = ctx->ckRH = nullptr;
    ctx->ck_cap = 0;
    (void)hipGetLastError();
    if (s == POD_EHIP) ctx->failed = 1;
    return (s == POD_OK) ? POD_ENOMEM : s;
}

pod_status pod_backward(pod_ctx *ctx, const void *dU, const double *dsigma, void *dA)
{
    if (!ctx || !dA) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    if (!ctx->ckU || ctx->pending) return POD_ESTATE;
    pod_info info{};
    pod_status s = pod_get_info(ctx, &info);
    if (s != POD_OK) return s;
    const int32_t rT = info.rank;
    if (rT < 1) return POD_ESTATE;
    const int32_t k = (ctx->prm.k < rT) ? ctx->prm.k : rT;
    const size_t m = (size_t)ctx->prm.m;
    A_HIP(hipMemsetAsync(ctx->Ubar[0], 0, m * rT * ctx->esz, ctx->st));
    A_HIP(hipMemsetAsync(ctx->sbar[0], 0, sizeof(double) * rT, ctx->st));
    if (dU) A_HIP(hipMemcpyAsync(ctx->Ubar[0], dU, m * k * ctx->esz, hipMemcpyDeviceToDevice, ctx->st));
    if (dsigma) A_HIP(hipMemcpyAsync(ctx->sbar[0], dsigma, sizeof(double) * k, hipMemcpyDeviceToDevice, ctx->st));
    return reverse_merges(ctx, dA);
}

pod_status pod_loss_grad(pod_ctx *ctx, void *dA, double *loss)
{
    const pod_status s = loss_enqueue(ctx, dA, loss);
    if (s != POD_OK) return s;
    return reverse_merges(ctx, dA);
}

}  // extern "C"

// The loss L = |A - U_k U_k^T A|_F^2 and the explicit part of its gradient
// (dA = 2 (A - U_k B), Ubar = -2 (A - U_k B) B^T, B = U_k^T A) enqueued on the
// run's stream; with `loss` set, L is read back (a synchronisation).
pod_status pod::loss_enqueue(pod_ctx *ctx, void *dA, double *loss)
{
    if (!ctx || !dA) return POD_EINVAL;
    if (ctx->failed) return POD_EHIP;
    if (!ctx->ckU || ctx->pending) return POD_ESTATE;
    pod_info info{};
    pod_status s = pod_get_info(ctx, &info);
    if (s != POD_OK) return s;
    const int32_t rT = info.rank;
    if (rT < 1) return POD_ESTATE;
    const int32_t k = (ctx->prm.k < rT) ? ctx->prm.k : rT;
    if (k > 64) return POD_EINVAL;
    const pod_params &p = ctx->prm;
    const size_t m = (size_t)p.m;
    // B = U_k^T A (one pass over A)
    ProjArgs pa;
    pa.prec = p.precision;
    pa.a_dtype = p.a_dtype;
    pa.m = p.m;
    pa.n = p.n;
    pa.lda = p.lda;
    pa.U = ctx->U[ctx->cur];
    pa.A = ctx->A;
    pa.r = k;
    pa.Bpart = ctx->Bpart;
    pa.nsplit = ctx->nsplit;
    pa.B = ctx->B;
    A_HIP(launch_project_partial(pa, ctx->st));
    A_HIP(launch_project_reduce(pa, ctx->st));
    A_HIP(hipMemsetAsync(ctx->Ubar[0], 0, m * rT * ctx->esz, ctx->st));
    A_HIP(hipMemsetAsync(ctx->sbar[0], 0, sizeof(double) * rT, ctx->st));
    hipError_t e;
    if (p.precision == POD_F64) {
        if (p.a_dtype == POD_F64)
            e = loss_resid_launch<double, double>(ctx->A, p.lda, p.m, p.n, ctx->U[ctx->cur], k, ctx->B, dA,
                                                  ctx->Ubar[0], ctx->lossp, ctx->st);
        else
            e = loss_resid_launch<double, float>(ctx->A, p.lda, p.m, p.n, ctx->U[ctx->cur], k, ctx->B, dA,
                                                 ctx->Ubar[0], ctx->lossp, ctx->st);
    } else {
        e = loss_resid_launch<float, float>(ctx->A, p.lda, p.m, p.n, ctx->U[ctx->cur], k, ctx->B, dA, ctx->Ubar[0],
                                            ctx->lossp, ctx->st);
    }
    A_HIP(e);
    if (loss) {
        const size_t nb = (m + 255) / 256;
        std::vector<double> lp(nb);
        A_HIP(hipMemcpyAsync(lp.data(), ctx->lossp, sizeof(double) * nb, hipMemcpyDeviceToHost, ctx->st));
        A_HIP(hipStreamSynchronize(ctx->st));
        double L = 0.0;
        for (size_t i = 0; i < nb; ++i) L += lp[i];
        *loss = L;
    }
    return POD_OK;
}

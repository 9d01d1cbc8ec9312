// pod_batch.hip -- many independent ISMA runs (Alg. 1) on matrices of uneven
// m, n, k advanced together: every kernel of an iteration is launched once
// for the whole batch (blockIdx.y = matrix), so the single-workgroup FP64
// stages of different matrices run side by side instead of one after the
// other.  The iteration's launch sequence does not depend on host state, so
// it is captured once in a HIP graph and replayed; a device-side stop test
// marks finished matrices, which every batched kernel then skips.
//
// Tile table: the row-block count of the Gram partials per matrix, keyed by
// (merge-width bucket, log2 m bucket, compute type), either the default
// (one 256-row slab per workgroup, at most 256 workgroups) or measured by
// pod_batch_autotune on the batch's own buffers.
#include <math.h>

#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "pod_ctx.h"

using namespace pod;

struct pod_batch {
    int32_t count = 0;
    hipStream_t st = nullptr;          // internal stream (captured)
    std::vector<pod_ctx *> ctx;
    int32_t prec = 0;
    int32_t pmax_max = 0, max_nblk = 0, max_nb = 0;
    DrawArgs *d_draw = nullptr;
    GramArgs *d_g1 = nullptr, *d_g2 = nullptr;
    SmallArgs *d_small = nullptr;
    TallArgs *d_t1 = nullptr, *d_t2 = nullptr;
    DevState **d_ds = nullptr;
    int32_t *d_maxit = nullptr;
    double *d_sintol = nullptr;
    int32_t *d_ndone = nullptr;
    int32_t *h_ndone = nullptr;        // pinned
    std::vector<GramArgs> g1, g2;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t iters = 0;
    CkptArgs *d_ck = nullptr;        // checkpoints of the reverse pass (nullable)
    int64_t max_mr = 0;
    int failed = 0;
};

namespace {

#define B_HIP(call)                                                                                                   \
    do {                                                                                                              \
        hipError_t e_ = (call);                                                                                       \
        if (e_ != hipSuccess) {                                                                                       \
            b->failed = 1;                                                                                            \
            return (e_ == hipErrorOutOfMemory) ? POD_ENOMEM : POD_EHIP;                                               \
        }                                                                                                             \
    } while (0)

void batch_free(pod_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (pod_ctx *c : b->ctx)
        if (c) pod_destroy(c);
    void *ptrs[] = {b->d_draw, b->d_g1, b->d_g2, b->d_small, b->d_t1, b->d_t2, b->d_ds, b->d_maxit, b->d_sintol,
                    b->d_ndone, b->d_ck};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (b->h_ndone) (void)hipHostFree(b->h_ndone);
    if (b->st) (void)hipStreamDestroy(b->st);
}

int32_t width_bucket(int32_t pmax) { return (pmax + 15) / 16; }
int32_t m_bucket(int64_t m)
{
    int32_t e = 0;
    while (((int64_t)1 << (e + 1)) <= m) ++e;
    return e;
}

// One iteration for the whole batch: GET UPDATE, then Alg. 2.
pod_status enqueue_iteration(pod_batch *b)
{
    const int32_t n = b->count;
    B_HIP(launch_draw_cols_b(b->d_draw, n, b->st));
    if (b->d_ck) B_HIP(launch_ckpt_pre_b(b->d_ck, n, b->max_mr, b->prec, b->st));
    B_HIP(launch_gram_partial_b(b->d_g1, n, b->max_nblk, b->pmax_max, b->prec, b->st));
    B_HIP(launch_gram_reduce_b(b->d_g1, n, b->pmax_max, b->st));
    B_HIP(launch_chol_first_b(b->d_small, n, b->pmax_max, b->st));
    B_HIP(launch_gemm_tall_b(b->d_t1, n, b->max_nb, b->pmax_max, b->pmax_max, b->prec, b->st));
    B_HIP(launch_gram_partial_b(b->d_g2, n, b->max_nblk, b->pmax_max, b->prec, b->st));
    B_HIP(launch_gram_reduce_b(b->d_g2, n, b->pmax_max, b->st));
    B_HIP(launch_svd_merge_b(b->d_small, n, b->pmax_max, b->st));
    if (b->d_ck) B_HIP(launch_ckpt_post_b(b->d_ck, n, b->st));
    B_HIP(launch_gemm_tall_b(b->d_t2, n, b->max_nb, b->pmax_max, b->pmax_max, b->prec, b->st));
    B_HIP(launch_batch_done(b->d_ds, b->d_maxit, b->d_sintol, n, b->d_ndone, b->st));
    B_HIP(hipMemcpyAsync(b->h_ndone, b->d_ndone, sizeof(int32_t), hipMemcpyDeviceToHost, b->st));
    return POD_OK;
}

pod_status upload_gram_args(pod_batch *b)
{
    int32_t mx = 1;
    for (const GramArgs &g : b->g1) mx = (g.nblk > mx) ? g.nblk : mx;
    b->max_nblk = mx;
    B_HIP(hipMemcpy(b->d_g1, b->g1.data(), sizeof(GramArgs) * b->count, hipMemcpyHostToDevice));
    B_HIP(hipMemcpy(b->d_g2, b->g2.data(), sizeof(GramArgs) * b->count, hipMemcpyHostToDevice));
    if (b->exec) {   // the captured grid sizes change: capture again
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
    }
    return POD_OK;
}

}  // namespace

extern "C" {

pod_status pod_batch_init(pod_batch **out, int32_t count, const pod_params *prm, void *const *A)
{
    if (!out || count < 1 || !prm || !A) return POD_EINVAL;
    *out = nullptr;
    for (int32_t i = 0; i < count; ++i) {
        if (!A[i]) return POD_EINVAL;
        if (prm[i].w != 0 || prm[i].r_update != 0) return POD_EINVAL;
        if (prm[i].precision != prm[0].precision) return POD_EINVAL;
        if (prm[i].precision == POD_BF16_REFINE) return POD_EINVAL;   // batched kernels: FP64 / FP32
        if (prm[i].col_strategy == POD_COL_ORT) return POD_EINVAL;    // batched draws: L2N / UNF
    }
    pod_batch *b = new (std::nothrow) pod_batch();
    if (!b) return POD_ENOMEM;
    b->count = count;
    b->prec = prm[0].precision;
    pod_status s = POD_OK;
    hipError_t e = hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking);
    if (e != hipSuccess) s = POD_EHIP;
    b->ctx.assign(count, nullptr);
    for (int32_t i = 0; i < count && s == POD_OK; ++i) {
        s = ctx_create(&b->ctx[i], &prm[i], b->st);
        if (s == POD_OK && b->ctx[i]->pmax > 64) s = POD_EINVAL;
        if (s == POD_OK) s = ctx_bind(b->ctx[i], A[i], prm[i].n, prm[i].lda, prm[i].block);
    }
    if (s == POD_OK) {
        e = hipSuccess;
        auto al = [&](void **p, size_t bytes) {
            if (e == hipSuccess) e = hipMalloc(p, bytes);
        };
        al((void **)&b->d_draw, sizeof(DrawArgs) * count);
        al((void **)&b->d_g1, sizeof(GramArgs) * count);
        al((void **)&b->d_g2, sizeof(GramArgs) * count);
        al((void **)&b->d_small, sizeof(SmallArgs) * count);
        al((void **)&b->d_t1, sizeof(TallArgs) * count);
        al((void **)&b->d_t2, sizeof(TallArgs) * count);
        al((void **)&b->d_ds, sizeof(DevState *) * count);
        al((void **)&b->d_maxit, sizeof(int32_t) * count);
        al((void **)&b->d_sintol, sizeof(double) * count);
        al((void **)&b->d_ndone, sizeof(int32_t));
        if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_ndone, sizeof(int32_t), hipHostMallocDefault);
        if (e != hipSuccess) s = (e == hipErrorOutOfMemory) ? POD_ENOMEM : POD_EHIP;
    }
    if (s == POD_OK) {
        std::vector<DrawArgs> dr(count);
        std::vector<SmallArgs> sm(count);
        std::vector<TallArgs> t1(count), t2(count);
        std::vector<DevState *> dss(count);
        std::vector<int32_t> mi(count);
        std::vector<double> tol(count);
        b->g1.resize(count);
        b->g2.resize(count);
        int32_t pm = 16, nb = 1;
        for (int32_t i = 0; i < count; ++i) {
            pod_ctx *c = b->ctx[i];
            pm = (c->pmax > pm) ? c->pmax : pm;
            dr[i] = ctx_draw_args(c);
            sm[i] = ctx_small_args(c);
            const GemmDesc gd = ctx_gather_desc(c), yd = ctx_plain_desc(c, c->Y);
            GramArgs &a1 = b->g1[i], &a2 = b->g2[i];
            a1.d = gd;
            a1.ds = c->ds;
            a1.which_p = -1;
            a1.pmax = c->pmax;
            a1.nblk = c->nblk;
            a1.vec = gemm_vec_ok(gd);
            a1.part = c->part;
            a1.G = c->G;
            a2 = a1;
            a2.d = yd;
            a2.which_p = -2;
            a2.vec = gemm_vec_ok(yd);
            TallArgs &x1 = t1[i], &x2 = t2[i];
            x1.d = gd;
            x1.ds = c->ds;
            x1.sel_in = -1;
            x1.sel_out = -2;
            x1.pin_max = c->pmax;
            x1.pout_max = c->pmax;
            x1.T = c->Tc;
            x1.ldt = c->pmax;
            x1.vec = a1.vec;
            x1.nb = tall_blocks(c->prm.m);
            x1.Yout = c->Y;
            x1.Yout1 = nullptr;
            x1.tri = 1;   // T1 = P R1^-1 (no right factor in batches)
            x2 = x1;
            x2.tri = 0;
            x2.d = yd;
            x2.sel_in = -2;
            x2.sel_out = -3;
            x2.pout_max = (c->r + 15) & ~15;
            x2.vec = a2.vec;
            x2.Yout = c->U[0];
            x2.Yout1 = c->U[1];
            nb = (x1.nb > nb) ? x1.nb : nb;
            dss[i] = c->ds;
            mi[i] = c->prm.max_iter;
            tol[i] = c->prm.theta_tol < 1.5707963267948966 ? sin(c->prm.theta_tol) : 1.0;
        }
        b->pmax_max = pm;
        b->max_nb = nb;
        e = hipMemcpy(b->d_draw, dr.data(), sizeof(DrawArgs) * count, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->d_small, sm.data(), sizeof(SmallArgs) * count, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->d_t1, t1.data(), sizeof(TallArgs) * count, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->d_t2, t2.data(), sizeof(TallArgs) * count, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->d_ds, dss.data(), sizeof(DevState *) * count, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->d_maxit, mi.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->d_sintol, tol.data(), sizeof(double) * count, hipMemcpyHostToDevice);
        if (e != hipSuccess) s = POD_EHIP;
        if (s == POD_OK) s = upload_gram_args(b);
        if (s == POD_OK && hipStreamSynchronize(b->st) != hipSuccess) s = POD_EHIP;
    }
    if (s != POD_OK) {
        batch_free(b);
        delete b;
        return s;
    }
    *out = b;
    return POD_OK;
}

pod_status pod_batch_autotune(pod_batch *b, int32_t *table_entries)
{
    if (!b) return POD_EINVAL;
    if (b->failed) return POD_EHIP;
    // (width bucket, m bucket) -> (representative matrix, best rows per workgroup)
    std::map<std::pair<int32_t, int32_t>, int32_t> rep;
    for (int32_t i = 0; i < b->count; ++i) {
        const auto key = std::make_pair(width_bucket(b->ctx[i]->pmax), m_bucket(b->ctx[i]->prm.m));
        auto it = rep.find(key);
        if (it == rep.end() || b->ctx[it->second]->prm.m < b->ctx[i]->prm.m) rep[key] = i;
    }
    hipEvent_t e0, e1;
    B_HIP(hipEventCreate(&e0));
    B_HIP(hipEventCreate(&e1));
    std::map<std::pair<int32_t, int32_t>, int64_t> best_rows;
    for (const auto &kv : rep) {
        pod_ctx *c = b->ctx[kv.second];
        const int64_t m = c->prm.m;
        // the Y workspace as a plain source of pmax columns (timing only)
        GemmDesc yd = ctx_plain_desc(c, c->Y);
        float best = 1e30f;
        int64_t brows = 256;
        for (int64_t rows : {256, 512, 1024, 2048, 4096}) {
            int64_t nblk = (m + rows - 1) / rows;
            if (nblk > c->nblk) continue;
            if (nblk < 1) nblk = 1;
            for (int rep2 = 0; rep2 < 2; ++rep2) {   // the first launch warms up
                B_HIP(hipEventRecord(e0, b->st));
                for (int q = 0; q < 5; ++q) {
                    B_HIP(launch_gram_partial(yd, c->ds, c->pmax, c->pmax, c->part, (int32_t)nblk, b->st));
                    B_HIP(launch_gram_reduce_sel(c->part, (int32_t)nblk, c->pmax, c->ds, c->pmax, c->G, b->st));
                }
                B_HIP(hipEventRecord(e1, b->st));
                B_HIP(hipEventSynchronize(e1));
            }
            float ms = 0.0f;
            B_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                brows = rows;
            }
        }
        best_rows[kv.first] = brows;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int32_t i = 0; i < b->count; ++i) {
        pod_ctx *c = b->ctx[i];
        const int64_t rows = best_rows[std::make_pair(width_bucket(c->pmax), m_bucket(c->prm.m))];
        int64_t nblk = (c->prm.m + rows - 1) / rows;
        if (nblk > c->nblk) nblk = c->nblk;
        if (nblk < 1) nblk = 1;
        b->g1[i].nblk = (int32_t)nblk;
        b->g2[i].nblk = (int32_t)nblk;
    }
    if (table_entries) *table_entries = (int32_t)best_rows.size();
    return upload_gram_args(b);
}

pod_status pod_batch_run(pod_batch *b, int32_t use_graph, int32_t max_rounds, int32_t *rounds_out)
{
    if (!b || max_rounds < 1) return POD_EINVAL;
    if (b->failed) return POD_EHIP;
    *b->h_ndone = 0;
    int32_t rounds = 0;
    if (use_graph && !b->exec) {
        // one eager round first: every launch configuration is set up before capture
        pod_status s = enqueue_iteration(b);
        if (s != POD_OK) return s;
        B_HIP(hipStreamSynchronize(b->st));
        ++rounds;
        if (*b->h_ndone < b->count && rounds < max_rounds) {
            B_HIP(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
            s = enqueue_iteration(b);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(b->st, &g);
            if (s != POD_OK) return s;
            B_HIP(e);
            b->graph = g;
            B_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        }
    }
    while (rounds < max_rounds && *b->h_ndone < b->count) {
        if (b->d_ck) {
            // room for this round's checkpoints: a matrix merges at most once
            // per round; the captured launches read the argument array
            bool grown = false;
            for (int32_t i = 0; i < b->count; ++i) {
                pod_ctx *c = b->ctx[i];
                const int32_t before = c->ck_cap;
                const pod_status s = ckpt_reserve(c, b->iters + rounds + 1);
                if (s == POD_ENOMEM) c->ck_lost = 1;
                else if (s != POD_OK) return s;
                grown = grown || c->ck_cap != before;
            }
            if (grown) {
                std::vector<CkptArgs> ck(b->count);
                for (int32_t i = 0; i < b->count; ++i) ck[i] = ctx_ckpt_args(b->ctx[i]);
                B_HIP(hipMemcpy(b->d_ck, ck.data(), sizeof(CkptArgs) * b->count, hipMemcpyHostToDevice));
            }
        }
        if (use_graph) {
            B_HIP(hipGraphLaunch(b->exec, b->st));
        } else {
            pod_status s = enqueue_iteration(b);
            if (s != POD_OK) return s;
        }
        B_HIP(hipStreamSynchronize(b->st));
        ++rounds;
    }
    b->iters += rounds;
    if (rounds_out) *rounds_out = rounds;
    return (*b->h_ndone >= b->count) ? POD_OK : POD_ESTATE;
}

pod_status pod_batch_enable_adjoint(pod_batch *b)
{
    if (!b) return POD_EINVAL;
    if (b->failed) return POD_EHIP;
    if (b->iters > 0) return POD_ESTATE;
    if (b->d_ck) return POD_OK;
    std::vector<CkptArgs> ck(b->count);
    int64_t mr = 1;
    for (int32_t i = 0; i < b->count; ++i) {
        pod_status s = pod_enable_adjoint(b->ctx[i]);
        if (s != POD_OK) return s;
        ck[i] = ctx_ckpt_args(b->ctx[i]);
        const int64_t v = b->ctx[i]->prm.m * b->ctx[i]->r;
        mr = (v > mr) ? v : mr;
    }
    b->max_mr = mr;
    B_HIP(hipMalloc((void **)&b->d_ck, sizeof(CkptArgs) * b->count));
    B_HIP(hipMemcpy(b->d_ck, ck.data(), sizeof(CkptArgs) * b->count, hipMemcpyHostToDevice));
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
    }
    return POD_OK;
}

pod_status pod_batch_loss_grad(pod_batch *b, int32_t i, void *dA, double *loss)
{
    if (!b || i < 0 || i >= b->count) return POD_EINVAL;
    if (b->failed) return POD_EHIP;
    return pod_loss_grad(b->ctx[i], dA, loss);
}

pod_status pod_batch_loss_grad_all(pod_batch *b, void *const *dA, double *loss)
{
    if (!b || !dA) return POD_EINVAL;
    if (b->failed) return POD_EHIP;
    bool together = true;
    for (int32_t i = 0; i < b->count; ++i) {
        if (!dA[i]) return POD_EINVAL;
        if (!b->ctx[i]->ckU) return POD_ESTATE;
        together = together && b->ctx[i]->pb <= 64;
    }
    if (!together) {   // wide reverse steps: one matrix after another
        for (int32_t i = 0; i < b->count; ++i) {
            const pod_status s = pod_loss_grad(b->ctx[i], dA[i], loss ? &loss[i] : nullptr);
            if (s != POD_OK) return s;
        }
        return POD_OK;
    }
    for (int32_t i = 0; i < b->count; ++i) {
        const pod_status s = loss_enqueue(b->ctx[i], dA[i], loss ? &loss[i] : nullptr);
        if (s != POD_OK) return s;
    }
    return reverse_merges_batch(b->ctx.data(), b->count, dA, b->st);
}

pod_status pod_batch_project(pod_batch *b, int32_t i, void *U_out, double *sigma_out, void *V_out)
{
    if (!b || i < 0 || i >= b->count) return POD_EINVAL;
    if (b->failed) return POD_EHIP;
    return pod_project(b->ctx[i], U_out, sigma_out, V_out);
}

pod_status pod_batch_get_info(pod_batch *b, int32_t i, pod_info *info, int32_t *gram_blocks)
{
    if (!b || i < 0 || i >= b->count) return POD_EINVAL;
    if (b->failed) return POD_EHIP;
    if (gram_blocks) *gram_blocks = b->g1[i].nblk;
    return pod_get_info(b->ctx[i], info);
}

void pod_batch_destroy(pod_batch *b)
{
    if (!b) return;
    if (b->st) (void)hipStreamSynchronize(b->st);
    batch_free(b);
    delete b;
}

}  // extern "C"

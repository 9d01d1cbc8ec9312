// pod_incremental.hip -- Alg. 3 (incremental POD for matrices that do not fit
// in memory): ISMA on each column block, then BLOCK MERGE of the block's
// leading pairs into the running (U, Sigma).  Blocks come from device memory
// or from host memory; host blocks are copied on a side stream into two
// device buffers, the copy of block b+1 overlapping the ISMA of block b.
#include <chrono>
#include <new>

#include "pod_ctx.h"

using namespace pod;

struct pod_inc {
    pod_params prm{};
    hipStream_t st = nullptr;      // compute stream (the caller's)
    hipStream_t cs = nullptr;      // copy stream
    pod_ctx *blk = nullptr;        // ISMA on one block, rebound per block
    pod_ctx *glob = nullptr;       // running (U, Sigma), merges only
    void *Ub = nullptr;            // leading pairs of the last block (m x r, compute type)
    double *sb = nullptr;
    void *dbuf[2] = {nullptr, nullptr};
    size_t dbuf_bytes = 0;
    hipEvent_t copied[2] = {nullptr, nullptr}, consumed[2] = {nullptr, nullptr};
    hipEvent_t c0[2] = {nullptr, nullptr};
    int32_t blocks = 0;
    int64_t columns = 0;
    double copy_ms = 0.0, wall_ms = 0.0, bytes = 0.0;
    int failed = 0;
};

namespace {

#define INC_HIP(call)                                                                                                 \
    do {                                                                                                              \
        hipError_t e_ = (call);                                                                                       \
        if (e_ != hipSuccess) {                                                                                       \
            inc->failed = 1;                                                                                          \
            return (e_ == hipErrorOutOfMemory) ? POD_ENOMEM : POD_EHIP;                                               \
        }                                                                                                             \
    } while (0)

void inc_free(pod_inc *inc)
{
    if (inc->blk) pod_destroy(inc->blk);
    if (inc->glob) pod_destroy(inc->glob);
    if (inc->Ub) (void)hipFree(inc->Ub);
    if (inc->sb) (void)hipFree(inc->sb);
    for (int b = 0; b < 2; ++b) {
        if (inc->dbuf[b]) (void)hipFree(inc->dbuf[b]);
        if (inc->copied[b]) (void)hipEventDestroy(inc->copied[b]);
        if (inc->consumed[b]) (void)hipEventDestroy(inc->consumed[b]);
        if (inc->c0[b]) (void)hipEventDestroy(inc->c0[b]);
    }
    if (inc->cs) (void)hipStreamDestroy(inc->cs);
}

// ISMA (Alg. 1) on the bound block, its final step, and the merge.
pod_status run_block(pod_inc *inc)
{
    pod_ctx *b = inc->blk;
    for (;;) {
        pod_status s = pod_sample(b, nullptr, nullptr);
        if (s == POD_EXHAUSTED || s == POD_ESTATE) break;
        if (s != POD_OK) return s;
        s = pod_merge(b);
        if (s != POD_OK) return s;
        int32_t done = 0;
        s = pod_converged(b, &done, nullptr);
        if (s != POD_OK) return s;
        if (done) break;
    }
    pod_info info{};
    pod_status s = pod_get_info(b, &info);
    if (s != POD_OK) return s;
    const int32_t rank = info.rank;
    if (rank < 1) return POD_OK;   // a block without drawable columns adds nothing
    s = ctx_project(b, inc->Ub, inc->sb, nullptr, rank);
    if (s != POD_OK) return s;
    return ctx_merge_basis(inc->glob, inc->Ub, inc->sb, rank);
}

}  // namespace

extern "C" {

pod_status pod_inc_init(pod_inc **out, const pod_params *prm, void *stream)
{
    if (!out || !prm) return POD_EINVAL;
    *out = nullptr;
    if (prm->center_rows) return POD_EINVAL;   // centring needs the whole matrix
    pod_inc *inc = new (std::nothrow) pod_inc();
    if (!inc) return POD_ENOMEM;
    inc->prm = *prm;
    inc->prm.lda = prm->m;
    inc->st = (hipStream_t)stream;
    const int32_t r = prm->r ? prm->r : prm->k;
    pod_status s = ctx_create(&inc->blk, &inc->prm, stream);
    if (s == POD_OK) {
        pod_params g = inc->prm;
        g.n = r;
        g.c = r;
        g.w = 0;
        g.r_update = 0;
        g.a_dtype = (prm->precision == POD_F64) ? POD_F64 : POD_F32;
        s = ctx_create(&inc->glob, &g, stream);
    }
    if (s == POD_OK) {
        const size_t esz = (prm->precision == POD_F64) ? 8 : 4;
        const size_t aesz = (prm->a_dtype == POD_F64) ? 8 : 4;
        inc->dbuf_bytes = (size_t)prm->m * prm->n * aesz;
        hipError_t e = hipMalloc(&inc->Ub, (size_t)prm->m * r * esz);
        if (e == hipSuccess) e = hipMalloc((void **)&inc->sb, sizeof(double) * r);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&inc->cs, hipStreamNonBlocking);
        for (int b = 0; b < 2 && e == hipSuccess; ++b) {
            e = hipEventCreate(&inc->copied[b]);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&inc->consumed[b], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreate(&inc->c0[b]);
        }
        if (e != hipSuccess) s = (e == hipErrorOutOfMemory) ? POD_ENOMEM : POD_EHIP;
    }
    if (s != POD_OK) {
        inc_free(inc);
        delete inc;
        return s;
    }
    *out = inc;
    return POD_OK;
}

pod_status pod_inc_add_block(pod_inc *inc, const void *B_dev, int64_t nb, int64_t ldb)
{
    if (!inc || !B_dev || nb < 1 || nb > inc->prm.n || ldb < inc->prm.m) return POD_EINVAL;
    if (inc->failed) return POD_EHIP;
    pod_status s = ctx_bind(inc->blk, const_cast<void *>(B_dev), nb, ldb, (uint64_t)inc->blocks);
    if (s == POD_OK) s = run_block(inc);
    if (s != POD_OK) {
        inc->failed = 1;
        return s;
    }
    inc->blocks += 1;
    inc->columns += nb;
    return POD_OK;
}

pod_status pod_inc_add_host_blocks(pod_inc *inc, const void *const *B_host, const int64_t *nb, int32_t count)
{
    if (!inc || !B_host || !nb || count < 0) return POD_EINVAL;
    if (inc->failed) return POD_EHIP;
    for (int32_t i = 0; i < count; ++i)
        if (!B_host[i] || nb[i] < 1 || nb[i] > inc->prm.n) return POD_EINVAL;
    if (count == 0) return POD_OK;
    const size_t aesz = (inc->prm.a_dtype == POD_F64) ? 8 : 4;
    for (int b = 0; b < 2; ++b)
        if (!inc->dbuf[b]) INC_HIP(hipMalloc(&inc->dbuf[b], inc->dbuf_bytes));
    const auto t0 = std::chrono::steady_clock::now();
    auto enqueue_copy = [&](int32_t i) -> hipError_t {
        const int q = i & 1;
        // the buffer's previous block must be finished on the compute stream
        hipError_t e = hipStreamWaitEvent(inc->cs, inc->consumed[q], 0);
        if (e == hipSuccess) e = hipEventRecord(inc->c0[q], inc->cs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(inc->dbuf[q], B_host[i], (size_t)inc->prm.m * nb[i] * aesz, hipMemcpyHostToDevice,
                               inc->cs);
        if (e == hipSuccess) e = hipEventRecord(inc->copied[q], inc->cs);
        return e;
    };
    // consumed[] start signalled
    for (int b = 0; b < 2; ++b) INC_HIP(hipEventRecord(inc->consumed[b], inc->st));
    INC_HIP(enqueue_copy(0));
    for (int32_t i = 0; i < count; ++i) {
        const int q = i & 1;
        if (i + 1 < count) INC_HIP(enqueue_copy(i + 1));
        INC_HIP(hipStreamWaitEvent(inc->st, inc->copied[q], 0));
        pod_status s = pod_inc_add_block(inc, inc->dbuf[q], nb[i], inc->prm.m);
        if (s != POD_OK) return s;
        INC_HIP(hipEventRecord(inc->consumed[q], inc->st));
        // copy time of block i (complete: the compute stream waited for it)
        float ms = 0.0f;
        INC_HIP(hipEventSynchronize(inc->copied[q]));
        INC_HIP(hipEventElapsedTime(&ms, inc->c0[q], inc->copied[q]));
        inc->copy_ms += ms;
        inc->bytes += (double)inc->prm.m * nb[i] * aesz;
    }
    INC_HIP(hipStreamSynchronize(inc->st));
    inc->wall_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return POD_OK;
}

pod_status pod_inc_result(pod_inc *inc, void *U_out, double *sigma_out, int32_t *k_out)
{
    if (!inc) return POD_EINVAL;
    if (inc->failed) return POD_EHIP;
    pod_ctx *g = inc->glob;
    int32_t rank = 0;
    pod_status s = pod_get_basis(g, nullptr, nullptr, &rank);
    if (s != POD_OK) return s;
    const int32_t k = (inc->prm.k < rank) ? inc->prm.k : rank;
    if (k_out) *k_out = k;
    if (k < 1) return POD_ESTATE;
    const size_t esz = g->esz;
    if (U_out) {
        INC_HIP(hipMemcpyAsync(U_out, g->U[g->cur], (size_t)inc->prm.m * k * esz, hipMemcpyDeviceToDevice, inc->st));
        INC_HIP(launch_sign_fix(inc->prm.precision, U_out, inc->prm.m, k, nullptr, 0, g->signv, g->signi, inc->st));
    }
    if (sigma_out)
        INC_HIP(hipMemcpyAsync(sigma_out, g->sig[g->cur], sizeof(double) * k, hipMemcpyDeviceToDevice, inc->st));
    INC_HIP(hipStreamSynchronize(inc->st));
    return POD_OK;
}

pod_status pod_inc_get_info(pod_inc *inc, pod_inc_info *info)
{
    if (!inc || !info) return POD_EINVAL;
    info->blocks = inc->blocks;
    info->columns = inc->columns;
    info->host_bytes = inc->bytes;
    info->wall_ms = inc->wall_ms;
    info->copy_ms = inc->copy_ms;
    return POD_OK;
}

void pod_inc_destroy(pod_inc *inc)
{
    if (!inc) return;
    if (inc->st) (void)hipStreamSynchronize(inc->st);
    if (inc->cs) (void)hipStreamSynchronize(inc->cs);
    inc_free(inc);
    delete inc;
}

}  // extern "C"

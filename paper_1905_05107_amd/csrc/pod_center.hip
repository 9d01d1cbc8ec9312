// pod_center.hip -- row centring of the snapshot matrix (the POD is taken of
// the mean-subtracted snapshots, Sec. 1): mean_i = (1/n) sum_j a_ij in FP64,
// then a_ij <- a_ij - mean_i rounded to the storage type.  Used by pod_init
// (center_rows = 1) and by the stand-alone pod_center_rows.
#include <mutex>

#include "pod_ctx.h"

#pragma clang fp contract(off)

namespace pod {

// Threads run along rows (coalesced in column-major storage); the n columns
// are split into `nsplit` ranges whose FP64 partial sums are added in range
// order.  The split only adds parallelism for short columns: enough ranges
// for about 2048 workgroups, at most 8.
int32_t center_splits(int64_t m)
{
    const int64_t blocks = (m + 255) / 256;
    int64_t ns = (2048 + blocks - 1) / blocks;
    return (int32_t)(ns < 1 ? 1 : (ns > 8 ? 8 : ns));
}

template <typename T>
__global__ __launch_bounds__(256) void k_row_partial(const T *__restrict__ A, int64_t m, int64_t n, int64_t lda,
                                                     int32_t nsplit, double *__restrict__ part)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int32_t sp = blockIdx.y;
    const int64_t j0 = (n * sp) / nsplit, j1 = (n * (sp + 1)) / nsplit;
    double acc = 0.0;
    for (int64_t j = j0; j < j1; ++j) acc += (double)A[j * lda + i];
    part[(int64_t)sp * m + i] = acc;
}

// mean_i into part[i] (the first range's slot: each thread reads its row's
// partials before it writes)
__global__ __launch_bounds__(256) void k_row_mean(double *__restrict__ part, int64_t m, int64_t n, int32_t nsplit)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double acc = 0.0;
    for (int32_t sp = 0; sp < nsplit; ++sp) acc += part[(int64_t)sp * m + i];
    part[i] = acc / (double)n;
}

template <typename T>
__global__ __launch_bounds__(256) void k_center(T *__restrict__ A, int64_t m, int64_t lda,
                                                const double *__restrict__ mean)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    T *a = A + (int64_t)blockIdx.y * lda + i;
    *a = (T)((double)*a - mean[i]);
}

// The whole centring on `scratch` (center_splits(m) * m doubles).
hipError_t launch_center_rows(void *A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, double *scratch,
                              hipStream_t st)
{
    const int32_t ns = center_splits(m);
    dim3 g1((unsigned)((m + 255) / 256), (unsigned)ns);
    if (a_dtype == POD_F64)
        hipLaunchKernelGGL(k_row_partial<double>, g1, dim3(256), 0, st, (const double *)A, m, n, lda, ns, scratch);
    else
        hipLaunchKernelGGL(k_row_partial<float>, g1, dim3(256), 0, st, (const float *)A, m, n, lda, ns, scratch);
    hipLaunchKernelGGL(k_row_mean, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, scratch, m, n, ns);
    // one grid row per column; at most 65535 columns per launch
    for (int64_t j0 = 0; j0 < n; j0 += 65535) {
        const int64_t nj = (n - j0 < 65535) ? (n - j0) : 65535;
        dim3 g((unsigned)((m + 255) / 256), (unsigned)nj);
        if (a_dtype == POD_F64)
            hipLaunchKernelGGL(k_center<double>, g, dim3(256), 0, st, (double *)A + j0 * lda, m, lda, scratch);
        else
            hipLaunchKernelGGL(k_center<float>, g, dim3(256), 0, st, (float *)A + j0 * lda, m, lda, scratch);
    }
    return hipGetLastError();
}

}  // namespace pod

using namespace pod;

// Device scratch of pod_center_rows_noalloc: 2^23 doubles (64 MiB), one copy
// per device, held until the process ends.  Host code never uses this name
// as an address: the per-device pointers below come from hipGetSymbolAddress.
constexpr size_t CENTER_SCRATCH_DOUBLES = (size_t)1 << 23;
static __device__ __align__(256) double scratch[CENTER_SCRATCH_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double *scratch_ptr[MAX_DEVICES] = {};

// The current device's copy of `scratch`, looked up once per device.
pod_status scratch_for_current_device(double **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return POD_EHIP;
    if (dev < 0 || dev >= MAX_DEVICES) return POD_EINVAL;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return POD_EHIP;
        scratch_ptr[dev] = (double *)ptr;
    }
    *out = scratch_ptr[dev];
    return POD_OK;
}
}  // namespace

extern "C" {

pod_status pod_center_rows(void *A_dev, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, void *stream)
{
    if (!A_dev || m < 1 || n < 1 || lda < m || (a_dtype != POD_F64 && a_dtype != POD_F32)) return POD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    double *scratch = nullptr;
    hipError_t e = hipMalloc((void **)&scratch, sizeof(double) * (size_t)center_splits(m) * (size_t)m);
    if (e != hipSuccess) return (e == hipErrorOutOfMemory) ? POD_ENOMEM : POD_EHIP;
    e = launch_center_rows(A_dev, a_dtype, m, n, lda, scratch, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    const hipError_t ef = hipFree(scratch);
    if (e == hipSuccess) e = ef;
    return (e == hipSuccess) ? POD_OK : POD_EHIP;
}

pod_status pod_center_rows_noalloc(void *A_dev, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, void *stream)
{
    if (!A_dev || m < 1 || n < 1 || lda < m || (a_dtype != POD_F64 && a_dtype != POD_F32)) return POD_EINVAL;
    if ((size_t)center_splits(m) * (size_t)m > CENTER_SCRATCH_DOUBLES) return POD_EINVAL;
    double *ws = nullptr;
    const pod_status s = scratch_for_current_device(&ws);
    if (s != POD_OK) return s;
    // every scratch entry the kernels read is written first in the same call
    return (launch_center_rows(A_dev, a_dtype, m, n, lda, ws, (hipStream_t)stream) == hipSuccess) ? POD_OK
                                                                                                   : POD_EHIP;
}

}  // extern "C"

// pod_sample.hip -- column squared norms, integer sampling weights
// and the Philox column draw of GET UPDATE (Alg. 1) for gfx950.
//
// The column norms and the draw must reproduce the same integers on every
// run and on any machine that follows the same definition, so this file is
// compiled without floating-point contraction and every sum has a fixed order.
#include "pod_internal.h"

#pragma clang fp contract(off)

namespace pod {

// ---------------------------------------------------------------------------
// Column squared norms nu_j = sum_i a_ij^2 (Eq. LTSVD_prob), one workgroup of
// 256 threads per column, FP64 accumulation.  Fixed order: thread t adds, in
// increasing row order, rows s*256*V + t*V + q (V = 16 / sizeof(T) values
// per 16-byte vector) with acc = fma(x, x, acc); the 64 lanes of each wave
// combine by XOR butterfly (offsets 32..1); the four wave sums are added
// left to right.  Loads are 16-byte vectors (unrolled by 8 for memory-level
// parallelism) when the column is 16-byte aligned, scalar otherwise; the
// order of the additions is the same either way.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef f32x4 type; };
template <> struct Vec16<double> { typedef f64x2 type; };

template <typename T>
__device__ __forceinline__ void acc_vec(double &acc, const typename Vec16<T>::type &v);
template <>
__device__ __forceinline__ void acc_vec<float>(double &acc, const f32x4 &v)
{
    acc = fma((double)v[0], (double)v[0], acc);
    acc = fma((double)v[1], (double)v[1], acc);
    acc = fma((double)v[2], (double)v[2], acc);
    acc = fma((double)v[3], (double)v[3], acc);
}
template <>
__device__ __forceinline__ void acc_vec<double>(double &acc, const f64x2 &v)
{
    acc = fma(v[0], v[0], acc);
    acc = fma(v[1], v[1], acc);
}

template <typename T>
__global__ __launch_bounds__(256) void k_col_sqnorms(const T *__restrict__ A, int64_t m, int64_t lda,
                                                     double *__restrict__ nu)
{
    typedef typename Vec16<T>::type VT;
    constexpr int V = 16 / sizeof(T);
    constexpr int64_t L = 256 * V;
    constexpr int UNR = 8;
    const int t = threadIdx.x;
    const T *col = A + (int64_t)blockIdx.x * lda;
    const int64_t nfull = m / L;
    double acc = 0.0;
    int64_t s = 0;
    if (((uintptr_t)col & 15) == 0) {
        const VT *cv = reinterpret_cast<const VT *>(col) + t;
        for (; s + UNR <= nfull; s += UNR) {
            VT v[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) v[u] = __builtin_nontemporal_load(cv + (s + u) * 256);
#pragma unroll
            for (int u = 0; u < UNR; ++u) acc_vec<T>(acc, v[u]);
        }
        for (; s < nfull; ++s) {
            VT v = __builtin_nontemporal_load(cv + s * 256);
            acc_vec<T>(acc, v);
        }
    } else {
        for (; s < nfull; ++s) {
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const double x = (double)col[s * L + (int64_t)t * V + q];
                acc = fma(x, x, acc);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < V; ++q) {
        const int64_t i = nfull * L + (int64_t)t * V + q;
        if (i < m) {
            const double x = (double)col[i];
            acc = fma(x, x, acc);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc = acc + __shfl_xor(acc, o, 64);
    __shared__ double ws[4];
    if ((t & 63) == 0) ws[t >> 6] = acc;
    __syncthreads();
    if (t == 0) nu[blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

hipError_t launch_col_sqnorms(const void *A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, double *nu,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    ProfScope ps(POD_K_COLNORMS, st);
    if (a_dtype == POD_F64)
        hipLaunchKernelGGL(k_col_sqnorms<double>, dim3((unsigned)n), dim3(256), 0, st, (const double *)A, m, lda,
                           nu);
    else
        hipLaunchKernelGGL(k_col_sqnorms<float>, dim3((unsigned)n), dim3(256), 0, st, (const float *)A, m, lda, nu);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Integer sampling weights (one workgroup).  With B = 63 - ceil(log2 len) and
// e the exponent of max(v) (max < 2^e), w_j = floor(v_j 2^(B-1-e)), so the
// total stays below 2^62 and Pr[j] = w_j / sum w reproduces p_j = v_j / sum v
// up to one quantum.  A negative, infinite or NaN value raises FLAG_NONFINITE
// and zeroes every weight.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_quantize(const double *__restrict__ v, int64_t len,
                                                   uint64_t *__restrict__ w, DevState *ds, int32_t guard)
{
    if (guard && merge_halted(ds)) return;
    __shared__ double smax[16];
    __shared__ int sbad[16];
    const int t = threadIdx.x;
    double mx = 0.0;
    int bad = 0;
    for (int64_t i = t; i < len; i += 1024) {
        const double x = v[i];
        if (!(x >= 0.0) || isinf(x)) bad = 1;
        else mx = fmax(mx, x);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o, 64));
        bad |= __shfl_xor(bad, o, 64);
    }
    if ((t & 63) == 0) {
        smax[t >> 6] = mx;
        sbad[t >> 6] = bad;
    }
    __syncthreads();
    double vmax = 0.0;
    int anybad = 0;
    for (int q = 0; q < 16; ++q) {
        vmax = fmax(vmax, smax[q]);
        anybad |= sbad[q];
    }
    int cl = 0;
    while (((int64_t)1 << cl) < len) ++cl;
    const int B = 63 - cl;
    int e = 0;
    if (vmax > 0.0) (void)frexp(vmax, &e);
    for (int64_t i = t; i < len; i += 1024) {
        uint64_t q = 0;
        if (!anybad && vmax > 0.0) q = (uint64_t)floor(ldexp(v[i], B - 1 - e));
        w[i] = q;
    }
    if (t == 0 && anybad && ds) atomicOr(&ds->flags, (int32_t)FLAG_NONFINITE);
}

hipError_t launch_quantize(const double *v, int64_t len, uint64_t *w, DevState *ds, int32_t guard, hipStream_t st)
{
    ProfScope ps(POD_K_DRAW, st);
    hipLaunchKernelGGL(k_quantize, dim3(1), dim3(1024), 0, st, v, len, w, ds, guard);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Column draw of GET UPDATE (one workgroup of 1024 threads).
//   weights over S: L2N (quantised norms) or, from the second iteration, 1
//   (UNF); W = their total.  W == 0 marks S as exhausted.
//   c draws: u_d = word (d mod 4) of Philox(key (seed, 0),
//   counter (it, d/4, block, 0)); t = floor(u_d W / 2^64); index = first j
//   with F_j > t (F = inclusive prefix sum).  Thread chunks of the weight
//   vector are scanned in LDS; each draw finds its chunk by binary search
//   and its column by a short walk inside the chunk.
//   Distinct indices in ascending order with multiplicities, S <- S \ I_c,
//   appended to the column log.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void draw_cols_body(const DrawArgs &a)
{
    __shared__ uint64_t sincl[1024];   // inclusive prefix of chunk sums
    __shared__ int64_t sdraw[1024];
    __shared__ int64_t ssorted[1024];
    __shared__ int32_t sflag[1024];
    __shared__ int32_t spos[1024];
    __shared__ uint64_t swave[16];
    const int t = threadIdx.x;
    DevState *ds = a.ds;
    if (ds->done) return;   // a batched or device-driven run that has stopped
    const int32_t it = ds->it;
    const bool unf = a.unf && it > 0;
    const int64_t n = a.n;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t j0 = (int64_t)t * chunk;
    const int64_t j1 = (j0 + chunk < n) ? j0 + chunk : n;

    int32_t g = 0;
    if (a.forced) {
        // replay: the caller supplies the distinct columns (ascending) and counts
        g = a.forced_g;
        for (int32_t d = t; d < g; d += 1024) {
            a.cols[d] = a.forced[d];
            a.ccnt[d] = a.forced[1024 + d];
        }
        __syncthreads();
    } else {
        uint64_t csum = 0;
        for (int64_t j = j0; j < j1; ++j)
            if (a.inS[j]) csum += unf ? 1ULL : a.wq[j];
        // inclusive scan of csum over 1024 threads (wave scan + wave totals)
        uint64_t x = csum;
        const int lane = t & 63, wv = t >> 6;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) swave[wv] = x;
        __syncthreads();
        uint64_t off = 0;
        for (int q = 0; q < wv; ++q) off += swave[q];
        x += off;
        sincl[t] = x;
        __syncthreads();
        const uint64_t W = sincl[1023];
        if (W == 0) {
            if (t == 0) {
                ds->exhausted = 1;
                ds->s_empty = 1;
                ds->g = 0;
                ds->wtot = 0;
            }
            return;
        }
        const int32_t c = a.c;
        for (int32_t d = t; d < c; d += 1024) {
            uint64_t ctr[4] = {(uint64_t)it, (uint64_t)(d >> 2), a.block, 0};
            philox4x64_10(ctr, a.seed, 0);
            const uint64_t u = ctr[d & 3];
            const uint64_t tg = __umul64hi(u, W);
            // chunk q: first with sincl[q] > tg
            int lo = 0, hi = 1023;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (sincl[mid] > tg) hi = mid;
                else lo = mid + 1;
            }
            uint64_t run = (lo > 0) ? sincl[lo - 1] : 0;
            const int64_t q0 = (int64_t)lo * chunk;
            const int64_t q1 = (q0 + chunk < n) ? q0 + chunk : n;
            int64_t sel = q1 - 1;
            for (int64_t j = q0; j < q1; ++j) {
                if (a.inS[j]) run += unf ? 1ULL : a.wq[j];
                if (run > tg) {
                    sel = j;
                    break;
                }
            }
            sdraw[d] = sel;
        }
        __syncthreads();
        // rank sort (stable) of the c draws, then keep first occurrences
        for (int32_t d = t; d < c; d += 1024) {
            const int64_t v = sdraw[d];
            int32_t rk = 0;
            for (int32_t e = 0; e < c; ++e) {
                const int64_t u = sdraw[e];
                rk += (u < v) || (u == v && e < d);
            }
            ssorted[rk] = v;
        }
        __syncthreads();
        for (int32_t d = t; d < c; d += 1024) sflag[d] = (d == 0) || (ssorted[d] != ssorted[d - 1]);
        __syncthreads();
        if (t == 0) {
            int32_t run2 = 0;
            for (int32_t d = 0; d < c; ++d) {
                spos[d] = run2;
                run2 += sflag[d];
            }
            g = run2;
            spos[1023] = g;
        }
        __syncthreads();
        g = spos[1023];
        for (int32_t d = t; d < c; d += 1024) {
            if (sflag[d]) {
                int32_t e = d + 1;
                while (e < c && ssorted[e] == ssorted[d]) ++e;
                a.cols[spos[d]] = (int32_t)ssorted[d];
                a.ccnt[spos[d]] = e - d;
            }
        }
        if (t == 0) ds->wtot = W;
        __syncthreads();
    }
    // S update and log
    const int32_t base = ds->col_log_len;
    for (int32_t d = t; d < g; d += 1024) {
        const int32_t j = a.cols[d];
        a.inS[j] = 0;
        if (base + d < a.n) {
            a.col_log[base + d] = j;
            a.ccnt_log[base + d] = a.ccnt[d];
        }
    }
    __syncthreads();
    // does S keep a drawable column for the next iteration?
    int left = 0;
    const uint64_t *wl = a.wq_left ? a.wq_left : a.wq;
    for (int64_t j = j0; j < j1; ++j)
        if (a.inS[j] && (a.unf || wl[j] != 0)) left = 1;
    left = __syncthreads_or(left);
    if (t == 0) {
        ds->s_empty = !left;
        ds->g = g;
        ds->h = 0;
        ds->ru = g;
        ds->p0 = ds->rs + g;
        ds->p = ds->rs + g;
        if (it < a.max_iter) {
            a.col_log_off[it] = base;
            a.col_log_off[it + 1] = base + g;
        }
        ds->col_log_len = base + g;
        ds->exhausted = 0;
    }
}

__global__ __launch_bounds__(1024) void k_draw_cols(DrawArgs a) { draw_cols_body(a); }

// Batched: one workgroup per matrix (blockIdx.y), stopped matrices skipped.
__global__ __launch_bounds__(1024) void k_draw_cols_b(const DrawArgs *__restrict__ arr)
{
    const DrawArgs a = arr[blockIdx.y];
    if (a.ds->done) return;
    draw_cols_body(a);
}

hipError_t launch_draw_cols_b(const DrawArgs *arr, int32_t count, hipStream_t st)
{
    if (count < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_draw_cols_b, dim3(1, (unsigned)count), dim3(1024), 0, st, arr);
    return hipGetLastError();
}

// Stop test of Alg. 1 for every matrix of a batch (the host-side rule of a
// single run): S exhausted, max_iter merges, a non-finite value, or, from
// the second merge, a convergence sine below the tolerance.  *ndone gets the
// number of stopped matrices.
__global__ __launch_bounds__(256) void k_batch_done(DevState *const *__restrict__ dss,
                                                    const int32_t *__restrict__ max_iter,
                                                    const double *__restrict__ sin_tol, int32_t count,
                                                    int32_t *__restrict__ ndone)
{
    __shared__ int32_t sw[4];
    int32_t c = 0;
    for (int32_t b = threadIdx.x; b < count; b += 256) {
        DevState *ds = dss[b];
        if (!ds->done) {
            const bool d = ds->exhausted || ds->s_empty || ds->it >= max_iter[b] || (ds->flags & FLAG_FATAL) ||
                           (ds->it >= 2 && ds->sin_theta < sin_tol[b]);
            if (d) ds->done = 1;
        }
        c += ds->done ? 1 : 0;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) *ndone = ((sw[0] + sw[1]) + sw[2]) + sw[3];
}

// Stop test of a device-driven single run, after each merge: logs the merge's
// convergence sine (sin_log[it - 1]; rewriting the same value when the draw
// found S exhausted and nothing was merged) and sets `done` under the rule of
// pod_converged: a non-finite value or a Cholesky breakdown, S exhausted,
// max_iter merges, or, when stop_conv is set and from the second merge, a
// sine below tol.
__global__ void k_run_done(DevState *ds, int32_t max_iter, double tol, int32_t stop_conv, double *sin_log,
                           int32_t log_cap)
{
    if (threadIdx.x != 0 || ds->done) return;
    const int32_t it = ds->it;
    if (it >= 1 && it <= log_cap) sin_log[it - 1] = ds->sin_theta;
    const bool d = ds->exhausted || ds->s_empty || it >= max_iter || (ds->flags & FLAG_FATAL) ||
                   (stop_conv && it >= 2 && ds->sin_theta < tol);
    if (d) ds->done = 1;
}

hipError_t launch_run_done(DevState *ds, int32_t max_iter, double tol, int32_t stop_conv, double *sin_log,
                           int32_t log_cap, hipStream_t st)
{
    hipLaunchKernelGGL(k_run_done, dim3(1), dim3(64), 0, st, ds, max_iter, tol, stop_conv, sin_log, log_cap);
    return hipGetLastError();
}

hipError_t launch_batch_done(DevState *const *dss, const int32_t *max_iter, const double *sin_tol, int32_t count,
                             int32_t *ndone, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_done, dim3(1), dim3(256), 0, st, dss, max_iter, sin_tol, count, ndone);
    return hipGetLastError();
}

// ORT weights (see launch_ort_resid), one thread per column.
__global__ __launch_bounds__(256) void k_ort_resid(const double *__restrict__ nu, const double *__restrict__ B,
                                                   int32_t r, int64_t n, const uint8_t *__restrict__ inS,
                                                   double floor_rel, const DevState *ds, double *__restrict__ rho)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n || merge_halted(ds)) return;
    if (ds->it == 0) {
        rho[j] = nu[j];
        return;
    }
    double v = 0.0;
    if (inS[j]) {
        const int rs = ds->rs;
        double s = 0.0;
        for (int i = 0; i < rs; ++i) s = fma(B[i + j * r], B[i + j * r], s);
        const double res = nu[j] - s;
        v = (res > floor_rel * nu[j]) ? res : 0.0;
    }
    rho[j] = v;
}

hipError_t launch_ort_resid(const double *nu, const double *B, int32_t r, int64_t n, const uint8_t *inS,
                            double floor_rel, const DevState *ds, double *rho, hipStream_t st)
{
    ProfScope ps(POD_K_DRAW, st);
    hipLaunchKernelGGL(k_ort_resid, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, nu, B, r, n, inS, floor_rel,
                       ds, rho);
    return hipGetLastError();
}

hipError_t launch_draw_cols(const DrawArgs &a, hipStream_t st)
{
    ProfScope ps(POD_K_DRAW, st);
    hipLaunchKernelGGL(k_draw_cols, dim3(1), dim3(1024), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// SAMPLE AND SCALE UNIQUE ROWS (Alg. 1), row probabilities.
//   L2: rho_i = sum over the g distinct columns (ascending) of d_il^2 (the
//       squared row norms of D, Eq. of the row-norm probabilities);
//   LS: from the second iteration rho_i = sum_{l < min(k, r)} u_il^2, the
//       leverage scores of the current basis (Table of sampling strategies).
// Each sum is an fma chain in FP64 in column order.  Threads run along rows,
// so each column read is coalesced.
// ---------------------------------------------------------------------------
template <typename T, typename TU>
__global__ __launch_bounds__(256) void k_row_sqnorms(const T *__restrict__ A, int64_t m, int64_t lda,
                                                     const int32_t *__restrict__ cols, const TU *__restrict__ U0,
                                                     const TU *__restrict__ U1, int32_t k_ls, const DevState *ds,
                                                     double *__restrict__ rho, const double *__restrict__ cscale)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m || merge_halted(ds)) return;
    const TU *U = (ds->it & 1) ? U1 : U0;   // current basis
    double acc = 0.0;
    if (U && ds->it > 0) {
        const int kk = (k_ls < ds->rs) ? k_ls : ds->rs;
        for (int l = 0; l < kk; ++l) {
            const double x = (double)U[(int64_t)l * m + i];
            acc = fma(x, x, acc);
        }
    } else {
        const int g = ds->g;
        for (int l = 0; l < g; ++l) {
            double x = (double)A[(int64_t)cols[l] * lda + i];
            if (cscale) x *= cscale[l];   // rows of the scaled sample C (one-shot CTSVD)
            acc = fma(x, x, acc);
        }
    }
    rho[i] = acc;
}

hipError_t launch_row_sqnorms(const void *A, int32_t a_dtype, int64_t m, int64_t lda, const int32_t *cols,
                              const void *U0, const void *U1, int32_t u_prec, int32_t k_ls, const DevState *ds,
                              double *rho, hipStream_t st, const double *cscale)
{
    ProfScope ps(POD_K_DRAW, st);
    const unsigned nb = (unsigned)((m + 255) / 256);
    if (a_dtype == POD_F64)
        hipLaunchKernelGGL((k_row_sqnorms<double, double>), dim3(nb), dim3(256), 0, st, (const double *)A, m, lda,
                           cols, (const double *)U0, (const double *)U1, k_ls, ds, rho, cscale);
    else if (u_prec == POD_F64)
        hipLaunchKernelGGL((k_row_sqnorms<float, double>), dim3(nb), dim3(256), 0, st, (const float *)A, m, lda,
                           cols, (const double *)U0, (const double *)U1, k_ls, ds, rho, cscale);
    else
        hipLaunchKernelGGL((k_row_sqnorms<float, float>), dim3(nb), dim3(256), 0, st, (const float *)A, m, lda,
                           cols, (const float *)U0, (const float *)U1, k_ls, ds, rho, cscale);
    return hipGetLastError();
}

// Row draw (one workgroup of 1024 threads): w draws with replacement from the
// integer row weights, Philox key (seed, 1), counter (it, d/4, block, 0),
// word d mod 4; the same inverse-CDF rule as the column draw; distinct rows
// in ascending order with their multiplicities t_hat.
__global__ __launch_bounds__(1024) void k_draw_rows(RowDrawArgs a)
{
    __shared__ uint64_t sincl[1024];
    __shared__ int64_t sdraw[1024];
    __shared__ int64_t ssorted[1024];
    __shared__ int32_t sflag[1024];
    __shared__ int32_t spos[1025];
    __shared__ uint64_t swave[16];
    const int t = threadIdx.x;
    DevState *ds = a.ds;
    if (merge_halted(ds)) return;
    const int32_t it = ds->it;
    const int64_t m = a.m;
    const int64_t chunk = (m + 1023) / 1024;
    const int64_t j0 = (int64_t)t * chunk;
    const int64_t j1 = (j0 + chunk < m) ? j0 + chunk : m;
    uint64_t csum = 0;
    for (int64_t j = j0; j < j1; ++j) csum += a.wr[j];
    uint64_t x = csum;
    const int lane = t & 63, wv = t >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) swave[wv] = x;
    __syncthreads();
    uint64_t off = 0;
    for (int q = 0; q < wv; ++q) off += swave[q];
    sincl[t] = x + off;
    __syncthreads();
    const uint64_t W = sincl[1023];
    if (W == 0) {
        if (t == 0) {
            atomicOr(&ds->flags, (int32_t)FLAG_ZERO_ROWS);
            ds->h = 0;
            ds->wrow_tot = 0;
        }
        return;
    }
    const int32_t c = a.w;
    if (a.forced) {
        // replay: the caller's distinct rows (ascending) and multiplicities;
        // a row of zero weight would get an infinite scale
        const int32_t h = a.forced_h;
        const bool logit = it < a.max_iter;
        int zero = 0;
        for (int32_t d = t; d < h; d += 1024) {
            const int32_t row = a.forced[2048 + d], cnt = a.forced[3072 + d];
            a.rows[d] = row;
            a.rcnt[d] = cnt;
            zero |= (a.wr[row] == 0);
            if (logit) {
                a.row_log[(int64_t)it * c + d] = row;
                a.rcnt_log[(int64_t)it * c + d] = cnt;
            }
        }
        zero = __syncthreads_or(zero);
        if (t == 0) {
            if (zero) atomicOr(&ds->flags, (int32_t)FLAG_NONFINITE);
            ds->h = h;
            ds->wrow_tot = W;
        }
        return;
    }
    for (int32_t d = t; d < c; d += 1024) {
        uint64_t ctr[4] = {(uint64_t)it, (uint64_t)(d >> 2), a.block, 0};
        philox4x64_10(ctr, a.seed, 1);
        const uint64_t tg = __umul64hi(ctr[d & 3], W);
        int lo = 0, hi = 1023;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sincl[mid] > tg) hi = mid;
            else lo = mid + 1;
        }
        uint64_t run = (lo > 0) ? sincl[lo - 1] : 0;
        const int64_t q0 = (int64_t)lo * chunk;
        const int64_t q1 = (q0 + chunk < m) ? q0 + chunk : m;
        int64_t sel = q1 - 1;
        for (int64_t j = q0; j < q1; ++j) {
            run += a.wr[j];
            if (run > tg) {
                sel = j;
                break;
            }
        }
        sdraw[d] = sel;
    }
    __syncthreads();
    for (int32_t d = t; d < c; d += 1024) {
        const int64_t v = sdraw[d];
        int32_t rk = 0;
        for (int32_t e = 0; e < c; ++e) {
            const int64_t u = sdraw[e];
            rk += (u < v) || (u == v && e < d);
        }
        ssorted[rk] = v;
    }
    __syncthreads();
    for (int32_t d = t; d < c; d += 1024) sflag[d] = (d == 0) || (ssorted[d] != ssorted[d - 1]);
    __syncthreads();
    if (t == 0) {
        int32_t r2 = 0;
        for (int32_t d = 0; d < c; ++d) {
            spos[d] = r2;
            r2 += sflag[d];
        }
        spos[1024] = r2;
    }
    __syncthreads();
    const int32_t h = spos[1024];
    const bool logit = it < a.max_iter;
    for (int32_t d = t; d < c; d += 1024) {
        if (sflag[d]) {
            int32_t e = d + 1;
            while (e < c && ssorted[e] == ssorted[d]) ++e;
            a.rows[spos[d]] = (int32_t)ssorted[d];
            a.rcnt[spos[d]] = e - d;
            if (logit) {
                a.row_log[(int64_t)it * c + spos[d]] = (int32_t)ssorted[d];
                a.rcnt_log[(int64_t)it * c + spos[d]] = e - d;
            }
        }
    }
    if (t == 0) {
        ds->h = h;
        ds->wrow_tot = W;
    }
}

hipError_t launch_draw_rows(const RowDrawArgs &a, hipStream_t st)
{
    ProfScope ps(POD_K_DRAW, st);
    hipLaunchKernelGGL(k_draw_rows, dim3(1), dim3(1024), 0, st, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_basis_state(DevState *ds, int32_t rb, int32_t r, int32_t first,
                                                     int32_t *cols)
{
    for (int i = threadIdx.x; i < rb; i += 256) cols[i] = i;
    if (threadIdx.x == 0) {
        if (first) {
            const int32_t rr = (rb < r) ? rb : r;
            ds->rs = rr;
            ds->it = 1;
            ds->g = 0;
            ds->p0 = rr;
            ds->p = rr;
        } else {
            ds->g = rb;
            ds->p0 = ds->rs + rb;
            ds->p = ds->rs + rb;
        }
        ds->h = 0;
        ds->exhausted = 0;
        ds->s_empty = 0;
    }
}

hipError_t launch_basis_state(DevState *ds, int32_t rb, int32_t r, int32_t first, int32_t *cols, hipStream_t st)
{
    hipLaunchKernelGGL(k_basis_state, dim3(1), dim3(256), 0, st, ds, rb, r, first, cols);
    return hipGetLastError();
}

}  // namespace pod

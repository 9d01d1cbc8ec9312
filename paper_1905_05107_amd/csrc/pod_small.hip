// pod_small.hip -- FP64 small-matrix algebra of the merge (Alg. 2) on gfx950.
//
// One workgroup of 1024 threads works on p x p matrices (p <= 64) held in LDS:
// Cholesky factors of the CholeskyQR2 Grams, triangular inverses, the
// one-sided Jacobi SVD of the merge factor R (the paper's E), the rank guard,
// the convergence angles of Alg. 1 and the Rayleigh-Ritz step of the final
// projection.  These kernels are latency bound; they keep everything in LDS
// and use all 16 waves for every step.
#include "pod_internal.h"

namespace pod {

constexpr int NT = 512;

// ---------------------------------------------------------------------------
// In-place Cholesky S = R^T R of the symmetric p x p matrix S (LDS,
// column-major); on success the upper triangle holds R and the strict lower
// triangle is zeroed.  Fails (returns 1, uniformly across the block) when a
// pivot is not above `thr`.
// ---------------------------------------------------------------------------
__device__ int chol_upper(double *S, int p, double thr)
{
    for (int j = 0; j < p; ++j) {
        const double d = S[j + j * p];
        if (!(d > thr)) return 1;
        const double rjj = sqrt(d);
        __syncthreads();
        for (int k = j + (int)threadIdx.x; k < p; k += NT) S[j + k * p] = (k == j) ? rjj : S[j + k * p] / rjj;
        __syncthreads();
        const int q = p - j - 1;
        for (int idx = threadIdx.x; idx < q * q; idx += NT) {
            const int ii = idx % q, kk = idx / q;
            if (ii <= kk) {
                const int i = j + 1 + ii, k = j + 1 + kk;
                S[i + k * p] -= S[j + i * p] * S[j + k * p];
            }
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < p * p; idx += NT) {
        const int i = idx % p, k = idx / p;
        if (i > k) S[idx] = 0.0;
    }
    __syncthreads();
    return 0;
}

// In-place inverse of the upper-triangular p x p matrix R (LDS, column-major).
// Column j of the inverse: X(j,j) = 1/R(j,j), X(0:j-1, j) = -X(0:j-1,0:j-1) R(0:j-1, j) / R(j,j),
// using the already inverted leading block.  Each of the j dot products is
// split over G threads and combined by shuffles.  `tmp` holds p doubles.
__device__ void trinv_upper(double *R, int p, double *tmp)
{
    int G = 64;
    while (G > 1 && p * G > NT) G >>= 1;
    const int row = threadIdx.x / G, gl = threadIdx.x % G;
    for (int j = 0; j < p; ++j) {
        const double rjj = R[j + j * p];
        const double inv = 1.0 / rjj;
        double s = 0.0;
        if (row < j) {
            // X(row, l) for l in [row, j) is already inverted; R(l, j) is still original
            for (int l = row + gl; l < j; l += G) s += R[row + l * p] * R[l + j * p];
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
            if (o < G) s += __shfl_xor(s, o, 64);
        if (row < j && gl == 0) tmp[row] = -s * inv;
        __syncthreads();
        if (row < j && gl == 0) R[row + j * p] = tmp[row];
        if (threadIdx.x == 0) R[j + j * p] = inv;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Wave-local helpers: sums over aligned groups of G lanes by DPP moves
// (mirror / half-mirror / quad permutations: no LDS traffic), and an FP64
// reciprocal square root from the FP32 estimate refined by two Newton steps
// (relative error below 1e-15).
// ---------------------------------------------------------------------------
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int G> __device__ __forceinline__ double group_sum(double v)
{
    if (G >= 16) v += dpp_f64<0x140>(v);   // row_mirror
    if (G >= 8) v += dpp_f64<0x141>(v);    // row_half_mirror
    if (G >= 4) v += dpp_f64<0x4E>(v);     // quad_perm [2,3,0,1]
    if (G >= 2) v += dpp_f64<0xB1>(v);     // quad_perm [1,0,3,2]
    return v;
}
__device__ __forceinline__ double rsqrt_f64(double x)
{
    // x = f 2^e with f in [0.5, 2) and e even keeps the FP32 estimate in range
    int e;
    double f = frexp(x, &e);
    if (e & 1) {
        f *= 2.0;
        e -= 1;
    }
    double y = (double)__frsqrt_rn((float)f);
    y = y * fma(-0.5 * f * y, y, 1.5);
    y = y * fma(-0.5 * f * y, y, 1.5);
    return ldexp(y, -e / 2);
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi on the columns of X (rows x cols, column-major,
// ld = rows, LDS, rows <= 64), parallel round-robin ordering: each step
// rotates cols/2 disjoint pairs, G threads per pair (a pair's two columns
// are held in registers for the step).  A pair is rotated when
// (x_a^T x_b)^2 > tol^2 |x_a|^2 |x_b|^2, with
//   tau = |x_b|^2 - |x_a|^2, rho = 2 x_a^T x_b, h = sqrt(tau^2 + rho^2),
//   d = |tau| + h, c = d / sqrt(d^2 + rho^2), s = sign(tau) rho / sqrt(d^2 + rho^2),
// the closed form of the classical angle t = sign(zeta)/(|zeta| + sqrt(1+zeta^2)),
// zeta = tau/rho, written without divisions by rho.  The sweep loop stops
// after a sweep without rotation.  `sched` holds (cols|1)*(cols+1)/2 short2.
// Returns the number of sweeps or -1.
// ---------------------------------------------------------------------------
template <int G>
__device__ int jacobi_cols_g(double *X, int rows, int cols, double tol, int max_sweeps, short2 *sched)
{
    constexpr int MAXR = 64 / G;
    const int np = (cols + 1) & ~1;
    const int npair = np / 2;
    for (int i = threadIdx.x; i < (np - 1) * npair; i += NT) {
        const int s = i / npair, q = i % npair;
        const int a = (q == 0) ? 0 : ((q - 1 + s) % (np - 1)) + 1;
        const int b = ((np - 2 - q + s) % (np - 1)) + 1;
        sched[i] = make_short2((short)a, (short)b);
    }
    __syncthreads();
    const int q = threadIdx.x / G, gl = threadIdx.x % G;
    const bool active = q < npair;
    const double tol2 = tol * tol;
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        int rotated = 0;
        for (int s = 0; s < np - 1; ++s) {
            const short2 ab = active ? sched[s * npair + q] : make_short2(0, 0);
            const int a = ab.x, b = ab.y;
            const bool real = active && a < cols && b < cols;
            double xa[MAXR], xb[MAXR];
            double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
            for (int i = 0; i < MAXR; ++i) {
                const int r = gl + i * G;
                const bool ok = real && r < rows;
                xa[i] = ok ? X[a * rows + r] : 0.0;
                xb[i] = ok ? X[b * rows + r] : 0.0;
                al = fma(xa[i], xa[i], al);
                be = fma(xb[i], xb[i], be);
                ga = fma(xa[i], xb[i], ga);
            }
            al = group_sum<G>(al);
            be = group_sum<G>(be);
            ga = group_sum<G>(ga);
            if (real && ga * ga > tol2 * al * be) {
                const double tau = be - al, rho = 2.0 * ga;
                const double x1 = fma(tau, tau, rho * rho);
                const double h = x1 * rsqrt_f64(x1);
                const double d = fabs(tau) + h;
                const double iw = rsqrt_f64(fma(d, d, rho * rho));
                const double c = d * iw;
                const double sn = (tau >= 0.0 ? rho : -rho) * iw;
#pragma unroll
                for (int i = 0; i < MAXR; ++i) {
                    const int r = gl + i * G;
                    if (r < rows) {
                        X[a * rows + r] = c * xa[i] - sn * xb[i];
                        X[b * rows + r] = sn * xa[i] + c * xb[i];
                    }
                }
                rotated = 1;
            }
            __syncthreads();
        }
        if (__syncthreads_or(rotated) == 0) return sweep;
    }
    return -1;
}

__device__ int jacobi_cols(double *X, int rows, int cols, double tol, int max_sweeps, short2 *sched)
{
    if (cols < 2) return 1;
    const int npair = ((cols + 1) & ~1) / 2;
    if (npair * 16 <= NT) return jacobi_cols_g<16>(X, rows, cols, tol, max_sweeps, sched);
    return jacobi_cols_g<8>(X, rows, cols, tol, max_sweeps, sched);
}

// After jacobi_cols: sigma_i = |x_i|, sorted descending (ties by index);
// out (rows x cols, ld ldo) = x_i / sigma_i in sorted order (0 if sigma = 0).
__device__ void jacobi_finish(const double *X, int rows, int cols, double *sig_sorted, double *out, int ldo,
                              double *snorm, int *sperm)
{
    for (int i = threadIdx.x; i < cols; i += NT) {
        double s = 0.0;
        for (int r = 0; r < rows; ++r) s += X[r + (int64_t)i * rows] * X[r + (int64_t)i * rows];
        snorm[i] = sqrt(s);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cols; i += NT) {
        const double si = snorm[i];
        int rk = 0;
        for (int j = 0; j < cols; ++j) {
            const double sj = snorm[j];
            rk += (sj > si) || (sj == si && j < i);
        }
        sperm[rk] = i;
        sig_sorted[rk] = si;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < rows * cols; idx += NT) {
        const int r = idx % rows, o = idx / rows;
        const int i = sperm[o];
        const double s = sig_sorted[o];
        out[r + (int64_t)o * ldo] = (s > 0.0) ? X[r + (int64_t)i * rows] / s : 0.0;
    }
    __syncthreads();
}

template <typename T> __device__ __forceinline__ void store_t(void *base, int64_t idx, double v)
{
    reinterpret_cast<T *>(base)[idx] = (T)v;
}
__device__ __forceinline__ void store_c(void *base, int prec, int64_t idx, double v)
{
    if (prec == POD_F64) store_t<double>(base, idx, v);
    else store_t<float>(base, idx, v);
}

// ---------------------------------------------------------------------------
// CholeskyQR pass 1 factor: G1 = P^T G0 P with P = diag(Sigma_r, I_g) (the
// basis block enters the merge weighted by its singular values, Alg. 2),
// R1 = chol(G1) (shifted by s = p u tr(G1) if a pivot breaks down),
// T1 = P R1^-1 written in the compute type for the tall GEMM Y = X0 T1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_chol_first(SmallArgs a)
{
    extern __shared__ double lds[];
    __shared__ double sP[64];
    __shared__ double sred[16];
    __shared__ int sbad;
    DevState *ds = a.ds;
    if (ds->exhausted) return;
    const int p = ds->p, rs = ds->rs;
    const int pm = a.pmax;
    double *S = lds;
    double *tmp = lds + p * p;
    if (threadIdx.x == 0) sbad = 0;
    for (int i = threadIdx.x; i < p; i += NT) sP[i] = (i < rs) ? a.sigma[i] : 1.0;
    __syncthreads();
    double tr = 0.0;
    int bad = 0;
    for (int idx = threadIdx.x; idx < p * p; idx += NT) {
        const int i = idx % p, j = idx / p;
        const double v = a.G[i + j * pm] * sP[i] * sP[j];
        if (!isfinite(v)) bad = 1;
        S[idx] = v;
        a.work[idx] = v;
        if (i == j) tr += v;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) tr += __shfl_xor(tr, o, 64);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = tr;
    if (bad) sbad = 1;
    __syncthreads();
    double trace = 0.0;
    for (int q = 0; q < NT / 64; ++q) trace += sred[q];
    if (sbad) {
        if (threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)FLAG_NONFINITE);
        for (int idx = threadIdx.x; idx < p * p; idx += NT) S[idx] = (idx % p == idx / p) ? 1.0 : 0.0;
        __syncthreads();
    } else {
        const double thr = a.urnd * trace;
        int fail = chol_upper(S, p, thr * 1e-3);
        if (fail) {
            const double shift = (double)p * a.urnd * trace;
            __syncthreads();
            for (int idx = threadIdx.x; idx < p * p; idx += NT)
                S[idx] = a.work[idx] + ((idx % p == idx / p) ? shift : 0.0);
            __syncthreads();
            if (threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)FLAG_SHIFT);
            fail = chol_upper(S, p, 0.0);
            if (fail) {
                if (threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)FLAG_NONFINITE);
                for (int idx = threadIdx.x; idx < p * p; idx += NT) S[idx] = (idx % p == idx / p) ? 1.0 : 0.0;
                __syncthreads();
            }
        }
    }
    for (int idx = threadIdx.x; idx < pm * pm; idx += NT) {
        const int i = idx % pm, j = idx / pm;
        a.R1[idx] = (i < p && j < p) ? S[i + j * p] : 0.0;
    }
    __syncthreads();
    trinv_upper(S, p, tmp);
    for (int idx = threadIdx.x; idx < pm * pm; idx += NT) {
        const int i = idx % pm, j = idx / pm;
        const double v = (i < p && j < p) ? sP[i] * S[i + j * p] : 0.0;
        store_c(a.Tc, a.prec, idx, v);
    }
}

hipError_t launch_chol_first(const SmallArgs &a, hipStream_t st)
{
    const size_t lds = (size_t)(a.pmax * a.pmax + a.pmax) * sizeof(double);
    ProfScope ps(POD_K_CHOL, st);
    hipLaunchKernelGGL(k_chol_first, dim3(1), dim3(NT), lds, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CholeskyQR pass 2 and the small SVD of the merge:
//   R2 = chol(G2) (G2 = Y^T Y), R = R2 R1 (upper triangular, the paper's E up
//   to an orthogonal left factor), R = U_R Sigma_R V_R^T by one-sided Jacobi
//   on the columns of R, rank guard r' = min(r, #{sigma_i > p u sigma_1}),
//   Z2 = R2^-1 U_R(:, 0:r') in the compute type for U_new = Y Z2,
//   Sigma_new = Sigma_R(0:r').
// Convergence (Alg. 1): the first k columns of M = [U Sigma | C] span the old
// modes, and M = Q R with R upper triangular, so in the basis Q the old
// subspace is span(e_1..e_k) and the new one span(U_R(:, 0:k)).  The sines of
// the principal angles are the singular values of U_R(k:p, 0:k); the mode
// criterion compares R(:, i)/|R(:, i)| with U_R(:, i) one by one.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_svd_merge(SmallArgs a)
{
    extern __shared__ double lds[];
    __shared__ double ssig[64];
    __shared__ double snorm[64];
    __shared__ int sperm[64];
    __shared__ short2 ssched[64 * 32];
    __shared__ double sred[16];
    DevState *ds = a.ds;
    if (ds->exhausted) return;
    const int p = ds->p, rs = ds->rs;
    const int pm = a.pmax;
    double *S1 = lds;              // G2 -> R2 -> R2^-1
    double *S2 = lds + p * p;      // R1 -> U_R
    double *S3 = lds + 2 * p * p;  // R -> scratch
    double *tmp = lds + 3 * p * p; // p
    // ---- pass-2 Cholesky
    double tr = 0.0;
    for (int idx = threadIdx.x; idx < p * p; idx += NT) {
        const int i = idx % p, j = idx / p;
        const double v = a.G[i + j * pm];
        S1[idx] = v;
        S2[idx] = a.R1[i + j * pm];
        if (i == j) tr += v;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) tr += __shfl_xor(tr, o, 64);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = tr;
    __syncthreads();
    double trace = 0.0;
    for (int q = 0; q < NT / 64; ++q) trace += sred[q];
    int fail = isfinite(trace) ? chol_upper(S1, p, a.urnd * trace * 1e-3) : 1;
    if (fail) {
        const double shift = (double)p * a.urnd * (isfinite(trace) ? trace : 1.0);
        __syncthreads();
        for (int idx = threadIdx.x; idx < p * p; idx += NT) {
            const int i = idx % p, j = idx / p;
            S1[idx] = a.G[i + j * pm] + ((i == j) ? shift : 0.0);
        }
        __syncthreads();
        if (threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)FLAG_SHIFT);
        fail = isfinite(trace) ? chol_upper(S1, p, 0.0) : 1;
        if (fail) {
            if (threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)FLAG_NONFINITE);
            for (int idx = threadIdx.x; idx < p * p; idx += NT) S1[idx] = (idx % p == idx / p) ? 1.0 : 0.0;
            __syncthreads();
        }
    }
    // ---- R = R2 R1 (both upper triangular)
    for (int idx = threadIdx.x; idx < p * p; idx += NT) {
        const int i = idx % p, j = idx / p;
        double s = 0.0;
        for (int l = i; l <= j; ++l) s += S1[i + l * p] * S2[l + j * p];
        S3[idx] = (i <= j) ? s : 0.0;
    }
    __syncthreads();
    const int kk0 = (a.k < rs) ? a.k : rs;
    if (a.criterion == POD_CRIT_MODE && kk0 > 0) {
        for (int idx = threadIdx.x; idx < p * kk0; idx += NT) a.work[idx] = S3[idx];
    }
    __syncthreads();
    // ---- one-sided Jacobi SVD of R
    const double tol = (double)p * 1.1102230246251565e-16;
    const int sw = jacobi_cols(S3, p, p, tol, 60, ssched);
    if (threadIdx.x == 0) {
        ds->sweeps = (sw < 0 || ds->sweeps < 0) ? -1 : (sw > ds->sweeps ? sw : ds->sweeps);
        ds->sweeps_total += (sw > 0) ? sw : 0;
        if (sw < 0) atomicOr(&ds->flags, (int32_t)FLAG_NOCONV);
    }
    jacobi_finish(S3, p, p, ssig, S2, p, snorm, sperm);   // S2 <- U_R (sorted), ssig <- Sigma_R
    // ---- rank guard
    int nz = 0;
    const double thr = (double)p * a.urnd * ssig[0];
    for (int i = 0; i < p; ++i) nz += (ssig[i] > thr);
    const int rnew = (a.r < nz) ? a.r : nz;
    // ---- convergence angle
    const int kk = (kk0 < rnew) ? kk0 : rnew;
    double sin_max = __builtin_nan("");
    if (kk > 0) {
        if (a.criterion == POD_CRIT_MODE) {
            // per mode: sin of the angle between R(:,i)/|R(:,i)| and U_R(:,i)
            double mx = 0.0;
            if (threadIdx.x < 64) {
                for (int i = 0; i < kk; ++i) {
                    double nr = 0.0, dt = 0.0;
                    for (int r = threadIdx.x; r < p; r += 64) {
                        const double x = a.work[r + i * p];
                        nr += x * x;
                        dt += x * S2[r + i * p];
                    }
#pragma unroll
                    for (int o = 32; o >= 1; o >>= 1) {
                        nr += __shfl_xor(nr, o, 64);
                        dt += __shfl_xor(dt, o, 64);
                    }
                    const double inv = 1.0 / sqrt(nr);
                    double res = 0.0;
                    for (int r = threadIdx.x; r < p; r += 64) {
                        const double d = S2[r + i * p] - a.work[r + i * p] * inv * (dt * inv);
                        res += d * d;
                    }
#pragma unroll
                    for (int o = 32; o >= 1; o >>= 1) res += __shfl_xor(res, o, 64);
                    mx = fmax(mx, sqrt(res));
                }
            }
            if (threadIdx.x == 0) sred[0] = mx;
            __syncthreads();
            sin_max = sred[0];
        } else {
            const int br = p - kk;
            if (br <= 0) {
                sin_max = 0.0;
            } else {
                for (int idx = threadIdx.x; idx < br * kk; idx += NT) {
                    const int r = idx % br, c = idx / br;
                    S3[idx] = S2[(kk + r) + c * p];
                }
                __syncthreads();
                (void)jacobi_cols(S3, br, kk, tol, 60, ssched);
                double mx = 0.0;
                for (int c = threadIdx.x; c < kk; c += NT) {
                    double s = 0.0;
                    for (int r = 0; r < br; ++r) s += S3[r + c * br] * S3[r + c * br];
                    mx = fmax(mx, sqrt(s));
                }
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
                if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = mx;
                __syncthreads();
                double m2 = 0.0;
                for (int q = 0; q < NT / 64; ++q) m2 = fmax(m2, sred[q]);
                sin_max = m2;
                __syncthreads();
            }
        }
    }
    // ---- Z2 = R2^-1 U_R(:, 0:rnew)
    trinv_upper(S1, p, tmp);
    for (int idx = threadIdx.x; idx < pm * pm; idx += NT) {
        const int i = idx % pm, j = idx / pm;
        double s = 0.0;
        if (i < p && j < rnew)
            for (int l = i; l < p; ++l) s += S1[i + l * p] * S2[l + j * p];
        store_c(a.Tc, a.prec, idx, s);
    }
    for (int i = threadIdx.x; i < a.r; i += NT) a.sigma_new[i] = (i < rnew) ? ssig[i] : 0.0;
    if (threadIdx.x == 0) {
        ds->rnew = rnew;
        ds->sin_theta = sin_max;
        ds->rs = rnew;
        ds->it = ds->it + 1;
        ds->g = 0;
    }
}

hipError_t launch_svd_merge(const SmallArgs &a, hipStream_t st)
{
    const size_t lds = (size_t)(3 * a.pmax * a.pmax + a.pmax) * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_svd_merge, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(3 * 64 * 64 + 64) * (int)sizeof(double));
        if (e != hipSuccess) return e;
        attr = true;
    }
    ProfScope ps(POD_K_SVD, st);
    hipLaunchKernelGGL(k_svd_merge, dim3(1), dim3(NT), lds, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz of the final step: G_B = B B^T (r x r) with B = U^T A, its
// eigen-decomposition by one-sided Jacobi on the columns of G_B
// (G_B = U_B Lambda U_B^T, so the rotated columns converge to U_B Lambda),
// Sigma_B = sqrt(Lambda); U_B(:, 0:k) is written in the compute type.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_rr_small(RRArgs a)
{
    extern __shared__ double lds[];
    __shared__ double ssig[64];
    __shared__ double snorm[64];
    __shared__ int sperm[64];
    __shared__ short2 ssched[64 * 32];
    const int r = a.r;
    double *S = lds;
    double *Uo = lds + r * r;
    // G_B entries, one wave per entry group, lanes along n
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int e = wv; e < r * r; e += NT / 64) {
        const int i = e % r, j = e / r;
        if (i > j) continue;
        double s = 0.0;
        for (int64_t c = lane; c < a.n; c += 64) s += a.B[i + c * r] * a.B[j + c * r];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) {
            S[i + j * r] = s;
            S[j + i * r] = s;
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < r * r; idx += NT) a.GB[idx] = S[idx];
    const double tol = (double)r * 1.1102230246251565e-16;
    const int sw = jacobi_cols(S, r, r, tol, 60, ssched);
    if (threadIdx.x == 0 && sw < 0) atomicOr(&a.ds->flags, (int32_t)FLAG_NOCONV);
    jacobi_finish(S, r, r, ssig, Uo, r, snorm, sperm);
    for (int idx = threadIdx.x; idx < r * r; idx += NT) a.UB[idx] = Uo[idx];
    for (int i = threadIdx.x; i < r; i += NT) a.sig[i] = sqrt(ssig[i]);
    for (int idx = threadIdx.x; idx < r * a.k; idx += NT) store_c(a.Zc, a.prec, idx, Uo[idx]);
}

hipError_t launch_rr_small(const RRArgs &a, hipStream_t st)
{
    const size_t lds = (size_t)(2 * a.r * a.r) * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_rr_small, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(2 * 64 * 64) * (int)sizeof(double));
        if (e != hipSuccess) return e;
        attr = true;
    }
    ProfScope ps(POD_K_RR, st);
    hipLaunchKernelGGL(k_rr_small, dim3(1), dim3(NT), lds, st, a);
    return hipGetLastError();
}

// V = B^T U_B(:, 0:k) Sigma_B^-1 (n x k, compute type).
__global__ __launch_bounds__(256) void k_rr_v(const double *__restrict__ B, int64_t n, int32_t r, int32_t k,
                                             const double *__restrict__ UB, const double *__restrict__ sig,
                                             int32_t prec, void *V)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    for (int c = 0; c < k; ++c) {
        double s = 0.0;
        for (int i = 0; i < r; ++i) s += B[i + j * r] * UB[i + c * r];
        const double v = (sig[c] > 0.0) ? s / sig[c] : 0.0;
        store_c(V, prec, j + (int64_t)c * n, v);
    }
}

hipError_t launch_rr_v(const double *B, int64_t n, int32_t r, int32_t k, const double *UB, const double *sig,
                       int32_t prec, void *V, hipStream_t st)
{
    ProfScope ps(POD_K_RR, st);
    hipLaunchKernelGGL(k_rr_v, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, B, n, r, k, UB, sig, prec, V);
    return hipGetLastError();
}

// Sign convention of the outputs: u_i is negated (with v_i) unless its
// largest-magnitude entry (lowest index on ties) is positive.  Pass 1: each
// workgroup (column i, chunk c) finds its chunk's candidate; pass 2: the
// candidates of a column are combined in chunk order and the column flipped.
constexpr int SIGN_CHUNKS = 64;

template <typename T>
__global__ __launch_bounds__(256) void k_sign_partial(const T *U, int64_t m, double *cv, int64_t *ci)
{
    __shared__ double sv[4];
    __shared__ int64_t si[4];
    const int col = blockIdx.y, ch = blockIdx.x;
    const int64_t r0 = (m * ch) / SIGN_CHUNKS, r1 = (m * (ch + 1)) / SIGN_CHUNKS;
    const T *u = U + (int64_t)col * m;
    double best = -1.0;
    int64_t bi = r0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) {
        const double x = fabs((double)u[i]);
        if (x > best) {
            best = x;
            bi = i;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int64_t oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
    if ((threadIdx.x & 63) == 0) {
        sv[threadIdx.x >> 6] = best;
        si[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = sv[0];
        int64_t ii = si[0];
        for (int q = 1; q < 4; ++q)
            if (sv[q] > b || (sv[q] == b && si[q] < ii)) {
                b = sv[q];
                ii = si[q];
            }
        cv[col * SIGN_CHUNKS + ch] = (b >= 0.0) ? (double)u[ii] : 0.0;   // signed value of the candidate
        ci[col * SIGN_CHUNKS + ch] = ii;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_sign_apply(T *U, int64_t m, T *V, int64_t n, const double *cv,
                                                   const int64_t *ci)
{
    const int col = blockIdx.y;
    double b = -1.0, bs = 0.0;
    int64_t ii = 0;
    for (int q = 0; q < SIGN_CHUNKS; ++q) {
        const double v = cv[col * SIGN_CHUNKS + q];
        const int64_t i = ci[col * SIGN_CHUNKS + q];
        if (fabs(v) > b || (fabs(v) == b && i < ii)) {
            b = fabs(v);
            bs = v;
            ii = i;
        }
    }
    if (!(bs < 0.0)) return;
    const int64_t r0 = (m * blockIdx.x) / gridDim.x, r1 = (m * (blockIdx.x + 1)) / gridDim.x;
    T *u = U + (int64_t)col * m;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) u[i] = -u[i];
    if (V) {
        const int64_t c0 = (n * blockIdx.x) / gridDim.x, c1 = (n * (blockIdx.x + 1)) / gridDim.x;
        T *v = V + (int64_t)col * n;
        for (int64_t i = c0 + threadIdx.x; i < c1; i += 256) v[i] = -v[i];
    }
}

hipError_t launch_sign_fix(int32_t prec, void *U, int64_t m, int32_t k, void *V, int64_t n, double *cv,
                           int64_t *ci, hipStream_t st)
{
    if (k <= 0) return hipSuccess;
    ProfScope ps(POD_K_SIGN, st);
    dim3 g1(SIGN_CHUNKS, k), g2(64, k);
    if (prec == POD_F64) {
        hipLaunchKernelGGL(k_sign_partial<double>, g1, dim3(256), 0, st, (const double *)U, m, cv, ci);
        hipLaunchKernelGGL(k_sign_apply<double>, g2, dim3(256), 0, st, (double *)U, m, (double *)V, n, cv, ci);
    } else {
        hipLaunchKernelGGL(k_sign_partial<float>, g1, dim3(256), 0, st, (const float *)U, m, cv, ci);
        hipLaunchKernelGGL(k_sign_apply<float>, g2, dim3(256), 0, st, (float *)U, m, (float *)V, n, cv, ci);
    }
    return hipGetLastError();
}

}  // namespace pod

// pod_symeig.h -- FP64 symmetric eigensolver for one workgroup (n <= 160),
// used for the small matrices of the merge (R R^T), of the convergence test
// and of the final Rayleigh-Ritz step.  Included by pod_small.hip.
//
// The method keeps the dependent-step count low (a Jacobi SVD of a 60 x 60
// matrix needs ~700 dependent rotation steps):
//   1. Householder reduction to tridiagonal form (n-2 steps, 3 barriers each;
//      Golub & Van Loan, Alg. 8.3.1), reflectors kept in the strict lower
//      triangle of the input;
//   2. eigenvalues by multisection with Sturm counts (each group of lanes
//      evaluates the count at G points of its interval per round; LAPACK's
//      dstebz uses the same count with a pivot floor);
//   3. eigenvectors of the tridiagonal by inverse iteration with partial
//      pivoting, re-orthogonalised inside clusters of close eigenvalues
//      (LAPACK's dstein strategy);
//   4. back-transformation by the stored reflectors.
// Eigenvalues are absolutely accurate to ~u |A|; eigenvectors of
// eigenvalues separated by gap have errors ~u |A| / gap.
#pragma once

#include "pod_internal.h"

namespace pod {

constexpr int EIG_NT = 512;   // threads of the workgroups that call these routines
constexpr int EIG_NMAX = 160;

// 1/x from the hardware FP64 reciprocal estimate (relative error about 2^-24
// on gfx950) refined by one third-order step: with e = 1 - x y,
// 1/x = y (1 + e + e^2 + O(e^3)), so the truncation is O(2^-72) and the
// result is within about one ulp; three dependent operations after the
// estimate instead of the four of two Newton steps.
__device__ __forceinline__ double rcp_nr(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, y, 1.0);
    return fma(y, fma(e, e, e), y);
}

// One Newton step only: relative error ~2^-50, enough for the Sturm counts
// (only the signs of the pivots matter, away from the bisection tolerance).
__device__ __forceinline__ double rcp_nr1(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}

// Reductions over aligned groups of G lanes by DPP moves inside a row of 16
// (mirror, half-mirror, quad permutations) and, across rows, the gfx950 lane
// swaps (v_permlane16_swap / v_permlane32_swap exchange the odd 16-lane rows
// with the even ones, the upper 32 lanes with the lower ones): no LDS
// traffic.  Every lane of a group gets the result.
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v)
{
    // (the permutations used here read lanes of the same row only: no bound control needed)
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
// {a, b} = {v[l], v[l ^ W]} in every lane l (W = 16 or 32; order unspecified)
template <int W> __device__ __forceinline__ void xor_pair(double v, double &a, double &b)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    if constexpr (W == 16) {
        const auto x = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto y = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        a = __hiloint2double((int)y[0], (int)x[0]);
        b = __hiloint2double((int)y[1], (int)x[1]);
    } else {
        const auto x = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto y = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        a = __hiloint2double((int)y[0], (int)x[0]);
        b = __hiloint2double((int)y[1], (int)x[1]);
    }
}
struct OpSum { __device__ static double f(double a, double b) { return a + b; } };
struct OpMax { __device__ static double f(double a, double b) { return fmax(a, b); } };
struct OpMin { __device__ static double f(double a, double b) { return fmin(a, b); } };
template <int G, typename Op> __device__ __forceinline__ double group_reduce(double v)
{
    if (G >= 16) v = Op::f(v, dpp_f64<0x140>(v));   // row_mirror
    if (G >= 8) v = Op::f(v, dpp_f64<0x141>(v));    // row_half_mirror
    if (G >= 4) v = Op::f(v, dpp_f64<0x4E>(v));     // quad_perm [2,3,0,1]
    if (G >= 2) v = Op::f(v, dpp_f64<0xB1>(v));     // quad_perm [1,0,3,2]
    if (G >= 32) {
        double a, b;
        xor_pair<16>(v, a, b);
        v = Op::f(a, b);
    }
    if (G >= 64) {
        double a, b;
        xor_pair<32>(v, a, b);
        v = Op::f(a, b);
    }
    return v;
}
template <int G> __device__ __forceinline__ double group_sum(double v) { return group_reduce<G, OpSum>(v); }
__device__ __forceinline__ double wave_sum(double v) { return group_reduce<64, OpSum>(v); }
__device__ __forceinline__ double wave_max(double v) { return group_reduce<64, OpMax>(v); }
__device__ __forceinline__ double wave_min(double v) { return group_reduce<64, OpMin>(v); }

// The value of lane `lane` (a wave-uniform index) in every lane.
__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// 1/sqrt(x) (x > 0 normal) from the hardware estimate (relative error about
// 2^-24 on gfx950) and one third-order step: with e = 1 - x y^2,
// x^-1/2 = y (1 + e/2 + 3 e^2/8 + O(e^3)); y e and the polynomial are formed
// side by side, so four dependent operations follow the estimate (six for two
// Newton steps) and the result is within about one ulp.
__device__ __forceinline__ double rsqrt_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-(x * y), y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// ---------------------------------------------------------------------------
// Householder tridiagonalisation of the symmetric n x n matrix A (LDS,
// column-major, ld = n, both triangles stored).  On return d[0..n) is the
// diagonal, e[0..n-1) the sub-diagonal of T = Q^T A Q with
// Q = H_0 H_1 ... H_{n-3}, H_j = I - tau_j v_j v_j^T acting on rows j+1..n-1;
// v_j is stored in A(j+1:n, j) and tau_j in tau[j].  `pv` holds n doubles,
// `sc` 4 doubles.
// ---------------------------------------------------------------------------
__device__ void tridiag(double *A, int n, double *d, double *e, double *tau, double *pv, double *sc)
{
    const int t = threadIdx.x;
    const int lane = t & 63;
    (void)sc;
    for (int j = 0; j + 2 < n; ++j) {
        const int q = n - j - 1;          // length of x = A(j+1:n, j)
        double *x = A + j * n + (j + 1);
        // -- reflector, computed redundantly by every wave (no barrier):
        //    alpha = -sign(x0) |x|, v = x - alpha e1, tau = 1/(alpha^2 - alpha x0)
        double ss = 0.0;
        for (int l = lane; l < q; l += 64) ss += x[l] * x[l];
        ss = wave_sum(ss);
        const double x0 = x[0];
        double alpha, tj;
        if (ss > 0.0 && (ss - x0 * x0) > 0.0) {
            alpha = (x0 >= 0.0) ? -sqrt(ss) : sqrt(ss);
            tj = 1.0 / (alpha * alpha - alpha * x0);
        } else {
            alpha = x0;   // column already reduced
            tj = 0.0;
        }
        const double v0 = x0 - alpha;
        if (tj != 0.0) {
            // -- p = tau * A22 v  (8 lanes per row of A22 = rows j+1.. of A)
            double *A22 = A + (j + 1) * n + (j + 1);
            const int gl = t & 7;
            // the 8 lanes of a group share `row`, so a group is active or idle as a whole
            // (x[0] still holds x0 during this step: v = x + (v0 - x0) e1)
            const double dv = v0 - x0;
            for (int row = t >> 3; row < q; row += EIG_NT / 8) {
                double s0 = 0.0, s1 = 0.0;
                int k = gl;
                for (; k + 8 < q; k += 16) {
                    s0 += A22[row + k * n] * x[k];
                    s1 += A22[row + (k + 8) * n] * x[k + 8];
                }
                if (k < q) s0 += A22[row + k * n] * x[k];
                double s = s0 + s1;
                if (gl == 0) s += A22[row] * dv;
                s = group_sum<8>(s);
                if (gl == 0) pv[row] = tj * s;
            }
            __syncthreads();
            // -- K = tau/2 p^T v (every wave), w = p - K v, A22 -= v w^T + w v^T
            double kp = 0.0;
            for (int l = lane; l < q; l += 64) kp += pv[l] * x[l];
            if (lane == 0) kp += pv[0] * dv;
            const double kk = 0.5 * tj * wave_sum(kp);
            const int tx = t & 31, ty = t >> 5;
            for (int b = ty; b < q; b += EIG_NT / 32) {
                const double xb = x[b];
                const double vb = (b == 0) ? v0 : xb;
                const double wb = pv[b] - kk * vb;
                for (int a = tx; a < q; a += 32) {
                    const double xa = x[a], pa = pv[a];
                    const double va = (a == 0) ? v0 : xa;
                    const double wa = pa - kk * va;
                    A22[a + b * n] -= va * wb + wa * vb;
                }
            }
        }
        if (t == 0) {
            if (tj != 0.0) x[0] = v0;
            tau[j] = tj;
            d[j] = A[j + j * n];
            e[j] = alpha;
        }
        __syncthreads();
    }
    if (t == 0) {
        if (n >= 2) {
            d[n - 2] = A[(n - 2) + (n - 2) * n];
            e[n - 2] = A[(n - 1) + (n - 2) * n];
        }
        d[n - 1] = A[(n - 1) + (n - 1) * n];
        for (int j = (n >= 2 ? n - 2 : 0); j < n; ++j) tau[j] = 0.0;
    }
    __syncthreads();
}

// Number of eigenvalues of the tridiagonal (d, e2 = e^2) below x.
__device__ __forceinline__ int sturm_count(const double *d, const double *e2, int n, double x, double pivmin)
{
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
    int i = 1;
    for (; i + 1 < n; i += 2) {
        const double da = d[i] - x, db = d[i + 1] - x, ea = e2[i - 1], eb = e2[i];
        q = da - ea * rcp_nr1(q);
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
        q = db - eb * rcp_nr1(q);
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
    }
    if (i < n) {
        q = (d[i] - x) - e2[i - 1] * rcp_nr1(q);
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
    }
    return cnt;
}

// ---------------------------------------------------------------------------
// The nv largest eigenvalues of the tridiagonal (d, e), descending, into ev.
// Groups of G lanes (G = largest power of two with nv * G <= 512, G <= 64)
// each refine one eigenvalue by multisection: G Sturm counts per round at
// equally spaced interior points, the interval shrinking to the sub-interval
// where the count passes the eigenvalue's index.  Stops at width
// <= max(2 u max(|a|, |b|), 4 u |T|) + 4 pivmin (|T| from the Gershgorin
// interval).  `e2` holds n doubles.
// ---------------------------------------------------------------------------
__device__ void bisect_top(const double *d, const double *e, int n, int nv, double *ev, double *e2, double *sc)
{
    const int t = threadIdx.x;
    const double u = 1.1102230246251565e-16;
    if (t < n) e2[t] = (t + 1 < n) ? e[t] * e[t] : 0.0;
    if (t == 0) {
        double lo = d[0], hi = d[0], emax = 0.0;
        for (int i = 0; i < n; ++i) {
            const double r = ((i > 0) ? fabs(e[i - 1]) : 0.0) + ((i + 1 < n) ? fabs(e[i]) : 0.0);
            lo = fmin(lo, d[i] - r);
            hi = fmax(hi, d[i] + r);
            if (i + 1 < n) emax = fmax(emax, e[i] * e[i]);
        }
        const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax) * 4.0;
        const double wid = fmax(fabs(lo), fabs(hi));
        sc[0] = lo - 2.0 * u * wid * n - 2.0 * pivmin;
        sc[1] = hi + 2.0 * u * wid * n + 2.0 * pivmin;
        sc[2] = pivmin;
    }
    __syncthreads();
    int G = 64;
    while (G > 1 && nv * G > EIG_NT) G >>= 1;
    const int grp = t / G, gl = t % G;
    const int lane = t & 63;
    const double pivmin = sc[2];
    const bool active = grp < nv;
    const int idx = n - 1 - grp;            // ascending index of the target eigenvalue
    double a = sc[0], b = sc[1];
    // lanes of the group as a bit-field within the wave
    const int gbase = lane - gl;
    // absolute accuracy 4 u |T| (LAPACK's default for bisection), or relative 2 u
    const double atol = 4.0 * u * fmax(fabs(sc[0]), fabs(sc[1]));
    for (int round = 0; round < 80; ++round) {
        const bool done = !active || (b - a) <= fmax(2.0 * u * fmax(fabs(a), fabs(b)), atol) + 4.0 * pivmin;
        // all lanes of a group share `done`; a wave leaves when all its groups are done
        if (__all(done)) break;
        const double x = a + (b - a) * (double)(gl + 1) / (double)(G + 1);
        const int cnt = done ? 0 : sturm_count(d, e2, n, x, pivmin);
        const unsigned long long m = __ballot(!done && cnt > idx);
        const unsigned long long gm = (G == 64) ? m : ((m >> gbase) & ((1ULL << G) - 1));
        if (!done) {
            if (gm == 0) {
                a = a + (b - a) * (double)G / (double)(G + 1);
            } else {
                const int g0 = __ffsll((long long)gm) - 1;   // first point with count > idx
                const double nb = a + (b - a) * (double)(g0 + 1) / (double)(G + 1);
                const double na = (g0 == 0) ? a : a + (b - a) * (double)g0 / (double)(G + 1);
                a = na;
                b = nb;
            }
        }
    }
    if (active && gl == 0) ev[grp] = 0.5 * (a + b);
    __syncthreads();
}

// Number of eigenvalues of the tridiagonal above thr (every thread gets it).
__device__ int count_above(const double *d, const double *e2, int n, double thr, double pivmin, int *sint)
{
    if (threadIdx.x == 0) sint[0] = n - sturm_count(d, e2, n, thr, pivmin);
    __syncthreads();
    const int c = sint[0];
    __syncthreads();
    return c;
}

// ---------------------------------------------------------------------------
// Eigenvectors of the tridiagonal (d, e) for ev[0..nv) (descending) by
// inverse iteration: (T - lambda I) = P L U with partial pivoting, three
// solves from a fixed start vector, each followed by re-orthogonalisation
// against the earlier members of the cluster and normalisation.  A cluster
// is a run of eigenvalues whose neighbours differ by less than 1e-3 of their
// magnitude (a relative gap: the eigenvalues of R R^T span many orders of
// magnitude, and an absolute threshold would chain all small ones into one
// serial cluster).  One thread handles one cluster, its members in order.
// Y (n x nv, ld n) receives unit vectors.  `lu` holds eig_lu_stride(n)
// doubles per active thread (odd stride: no LDS bank conflicts between
// threads), at most EIG_LU_THREADS threads.
// ---------------------------------------------------------------------------
constexpr int EIG_LU_THREADS = 16;
// doubles per thread of the `lu` scratch: three diagonals of U, the
// multipliers and n interchange flags (ints, two per double), made odd
__host__ __device__ constexpr int eig_lu_stride(int n) { return (4 * n + (n + 1) / 2) | 1; }
// doubles of the whole `lu` scratch for dimension n
__host__ __device__ constexpr int eig_lu_doubles(int n) { return EIG_LU_THREADS * eig_lu_stride(n); }

__device__ void tri_invit(const double *d, const double *e, int n, const double *ev, int nv, double *Y, double *lu,
                          int *scl)
{
    const int t = threadIdx.x;
    const double u = 1.1102230246251565e-16;
    // cluster starts (thread 0): scl[0..nc] (scl[nc] = nv), scl[EIG_NMAX + 1] = nc
    if (t == 0) {
        double tn = 0.0;
        for (int i = 0; i < nv; ++i) tn = fmax(tn, fabs(ev[i]));
        for (int i = 0; i < n; ++i) tn = fmax(tn, fabs(d[i]) + ((i + 1 < n) ? fabs(e[i]) : 0.0));
        int nc = 0;
        for (int i = 0; i < nv; ++i)
            if (i == 0 || fabs(ev[i - 1] - ev[i]) > 1e-3 * fmax(fabs(ev[i - 1]), fabs(ev[i])) + 8.0 * u * tn)
                scl[nc++] = i;
        scl[nc] = nv;
        scl[EIG_NMAX + 1] = nc;
        ((double *)(scl + EIG_NMAX + 2))[0] = tn;
    }
    __syncthreads();
    const int nc = scl[EIG_NMAX + 1];
    const double tn = ((const double *)(scl + EIG_NMAX + 2))[0];
    for (int cb = 0; cb < nc; cb += EIG_LU_THREADS) {
        const int c = cb + t;
        if (t < EIG_LU_THREADS && c < nc) {
            double *u1 = lu + (size_t)t * eig_lu_stride(n), *u2 = u1 + n, *u3 = u2 + n, *ml = u3 + n;
            int *sw = reinterpret_cast<int *>(ml + n);   // row interchange at step i
            const int i0 = scl[c], i1 = scl[c + 1];
            for (int mi = i0; mi < i1; ++mi) {
                // perturb equal eigenvalues inside a cluster so the solves differ
                const double lam = ev[mi] + (double)(mi - i0) * 4.0 * u * tn;
                // factor: rows (r0, r1, r2) at cols (i, i+1, i+2); u1 keeps 1 / pivot
                double r0 = d[0] - lam, r1 = (n > 1) ? e[0] : 0.0, r2 = 0.0;
#pragma unroll 4
                for (int i = 0; i + 1 < n; ++i) {
                    const double s0 = e[i], s1 = d[i + 1] - lam, s2 = (i + 2 < n) ? e[i + 1] : 0.0;
                    const bool swap = !(fabs(r0) >= fabs(s0));
                    double p0 = swap ? s0 : r0;
                    const double p1 = swap ? s1 : r1, p2 = swap ? s2 : r2;
                    const double o1 = swap ? r1 : s1, o2 = swap ? r2 : s2;
                    if (p0 == 0.0) p0 = u * tn + 1e-300;
                    const double ip = rcp_nr(p0);
                    const double mult = (swap ? r0 : s0) * ip;
                    u1[i] = ip; u2[i] = p1; u3[i] = p2; ml[i] = mult;
                    sw[i] = swap ? 1 : 0;
                    r0 = o1 - mult * p1;
                    r1 = o2 - mult * p2;
                    r2 = 0.0;
                }
                if (r0 == 0.0) r0 = u * tn + 1e-300;
                u1[n - 1] = rcp_nr(r0);
                u2[n - 1] = 0.0;
                u3[n - 1] = 0.0;
                double *y = Y + (size_t)mi * n;
                // start vector: fixed, not orthogonal to any eigenvector in practice
                for (int i = 0; i < n; ++i) y[i] = 1.0 + 0.5 * (double)(((i + 3 * mi) * 2654435761u) % 1009u) / 1009.0;
                for (int itn = 0; itn < 2; ++itn) {
                    // forward: the row operations, carrying the current row in a register
                    // (loads batched by the unrolling; the chain runs through `cur`)
                    double cur = y[0];
#pragma unroll 8
                    for (int i = 0; i + 1 < n; ++i) {
                        const double nx = y[i + 1];
                        const bool s = sw[i] != 0;
                        const double top = s ? nx : cur, bot = s ? cur : nx;
                        y[i] = top;
                        cur = bot - ml[i] * top;
                    }
                    y[n - 1] = cur;
                    // back substitution with U (3 diagonals), last two values in registers
                    double x1 = 0.0, x2 = 0.0;
#pragma unroll 8
                    for (int i = n - 1; i >= 0; --i) {
                        const double sv = (y[i] - u2[i] * x1 - u3[i] * x2) * u1[i];
                        y[i] = sv;
                        x2 = x1;
                        x1 = sv;
                    }
                    // re-orthogonalise inside the cluster, normalise
                    for (int pj = i0; pj < mi; ++pj) {
                        const double *z = Y + (size_t)pj * n;
                        double dt = 0.0;
#pragma unroll 8
                        for (int i = 0; i < n; ++i) dt += z[i] * y[i];
#pragma unroll 8
                        for (int i = 0; i < n; ++i) y[i] -= dt * z[i];
                    }
                    double m4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
                    for (int i = 0; i < n; ++i) m4[i & 3] = fmax(m4[i & 3], fabs(y[i]));
                    const double mx = fmax(fmax(m4[0], m4[1]), fmax(m4[2], m4[3]));
                    const double sm = (mx > 0.0) ? 1.0 / mx : 1.0;
                    double q4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
                    for (int i = 0; i < n; ++i) {
                        const double v = y[i] * sm;
                        q4[i & 3] += v * v;
                    }
                    const double f = sm / sqrt((q4[0] + q4[1]) + (q4[2] + q4[3]));
#pragma unroll 8
                    for (int i = 0; i < n; ++i) y[i] *= f;
                }
            }
        }
        __syncthreads();
    }
}

// Y (n x nv, ld n) <- Q Y with Q = H_0 ... H_{n-3} stored by tridiag() in A.
__device__ void tridiag_backtransform(const double *A, const double *tau, int n, double *Y, int nv, double *dots)
{
    const int t = threadIdx.x;
    int G = 64;
    while (G > 1 && nv * G > EIG_NT) G >>= 1;
    const int col = t / G, gl = t % G;
    for (int j = n - 3; j >= 0; --j) {
        const double tj = tau[j];
        if (tj == 0.0) continue;   // uniform across the block
        const int q = n - j - 1;
        const double *v = A + j * n + (j + 1);
        double s0 = 0.0, s1 = 0.0;
        if (col < nv) {
            const double *y = Y + (size_t)col * n + j + 1;
            int i = gl;
            for (; i + G < q; i += 2 * G) {
                s0 += v[i] * y[i];
                s1 += v[i + G] * y[i + G];
            }
            if (i < q) s0 += v[i] * y[i];
        }
        double s = s0 + s1;
        switch (G) {   // groups are aligned and uniformly active
        case 64: s = group_sum<64>(s); break;
        case 32: s = group_sum<32>(s); break;
        case 16: s = group_sum<16>(s); break;
        case 8: s = group_sum<8>(s); break;
        case 4: s = group_sum<4>(s); break;
        case 2: s = group_sum<2>(s); break;
        default: break;
        }
        if (col < nv && gl == 0) dots[col] = tj * s;
        __syncthreads();
        for (int idx = t; idx < q * nv; idx += EIG_NT) {
            const int i = idx % q, c = idx / q;
            Y[(size_t)c * n + j + 1 + i] -= dots[c] * v[i];
        }
        __syncthreads();
    }
}

}  // namespace pod

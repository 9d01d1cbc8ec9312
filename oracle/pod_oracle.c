/*
 * pod_oracle.c -- plain, slow, FP64 CPU reference for the iterative
 * sample-and-merge POD (ISMA) of Charumathi, Ramakrishna & Vasudevan,
 * "Fast and Accurate Proper Orthogonal Decomposition using Efficient
 * Sampling and Iterative Techniques for SVD" (arXiv 1905.05107).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity oracle for the HIP
 * library.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or helper with the
 * GPU path and never calls it.
 *
 * Everything is single-threaded FP64 with explicit loops: no BLAS, no LAPACK.
 * Compile with -ffp-contract=off so every multiply-add below rounds exactly
 * as written (fma() is used only where it is written).
 *
 * Contents (paper passage each routine follows):
 *   or_philox4x64_10     counter-based generator (Salmon et al., SC'11) that
 *                        stands in for the paper's numpy RNG (Sec. 4 setup)
 *   or_col_sqnorms       |a_j|^2 of Eq. (LTSVD_prob), fixed summation order
 *   or_row_sqnorms       |d^i|^2 of Eq. (CTSVD_prob) / Alg. 1 GET UPDATE
 *   or_quantize          integer weights w_j ~ p_j (probabilities over S)
 *   or_draw              draws with replacement, Pr[s=j] = w_j / sum(w)
 *                        (Alg. 1 GET UPDATE and SAMPLE AND SCALE UNIQUE ROWS)
 *   or_unique            distinct indices and multiplicities t_hat
 *   or_householder_qr    QR used by Alg. 2 BLOCK MERGE and the final step
 *   or_jacobi_svd        one-sided (Hestenes) Jacobi SVD: SVD(E), SVD(R)
 *   or_jacobi_eig        cyclic two-sided Jacobi: SVD(W^T W) of GET UPDATE
 *   or_merge             Alg. 2 BLOCK MERGE on [U1 S1 | C], with truncation
 *                        and the rank guard r <- min(r, max{i: s_i != 0})
 *   or_subspace_sines    sines of principal angles (Bjorck & Golub), used by
 *                        the convergence test of Alg. 1
 *   or_project           final step of Alg. 1: QR(A^T U), SVD(R), rotation
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_U64_EPS (1.1102230246251565e-16) /* unit roundoff 2^-53 */

/* ------------------------------------------------------------------------ */
/* Philox-4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).  One block maps a     */
/* 256-bit counter and a 128-bit key to four 64-bit words.                  */
/* ------------------------------------------------------------------------ */
/* Threads of the OpenMP loops (over independent columns only, so every
 * result is bitwise the same for any count).  Used to time the oracle. */
void or_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

void or_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        __uint128_t p0 = (__uint128_t)0xD2E7470EE14C6C93ULL * c0;
        __uint128_t p1 = (__uint128_t)0xCA5A826395121157ULL * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Column squared norms nu_j = sum_i a_ij^2 (Eq. LTSVD_prob numerator).     */
/*                                                                          */
/* Summation order (a fixed reading, so that the integer sampling weights   */
/* derived from nu are reproducible bit for bit on any machine):            */
/*   V = 16 / elem_bytes values per 16-byte vector (4 for FP32, 2 for FP64) */
/*   256 accumulators t = 0..255; accumulator t adds, in increasing row     */
/*   order, the rows s*256*V + t*V + q (s = 0,1,..., q = 0..V-1), each as   */
/*   acc = fma(x, x, acc) in FP64 (for FP32 data x*x is exact, so this is   */
/*   also acc + x*x);                                                       */
/*   the 256 accumulators form 4 groups of 64; inside a group, six rounds   */
/*   v[l] <- v[l] + v[l ^ o] for o = 32,16,8,4,2,1 leave the group sum;      */
/*   nu = ((g0 + g1) + g2) + g3.                                            */
/* ------------------------------------------------------------------------ */
static double or_fixed_order_sumsq(const double *x, int64_t m, int elem_bytes)
{
    const int T = 256;
    const int V = 16 / elem_bytes;
    const int64_t L = (int64_t)T * V;
    double acc[256];
    for (int t = 0; t < T; ++t) {
        double a = 0.0;
        for (int64_t s = 0; s * L < m; ++s) {
            for (int q = 0; q < V; ++q) {
                int64_t i = s * L + (int64_t)t * V + q;
                if (i < m) a = fma(x[i], x[i], a);
            }
        }
        acc[t] = a;
    }
    double gsum[4];
    for (int w = 0; w < 4; ++w) {
        double v[64], nv[64];
        for (int l = 0; l < 64; ++l) v[l] = acc[64 * w + l];
        for (int o = 32; o >= 1; o >>= 1) {
            for (int l = 0; l < 64; ++l) nv[l] = v[l] + v[l ^ o];
            for (int l = 0; l < 64; ++l) v[l] = nv[l];
        }
        gsum[w] = v[0];
    }
    return ((gsum[0] + gsum[1]) + gsum[2]) + gsum[3];
}

void or_col_sqnorms(const double *A, int64_t m, int64_t n, int64_t lda, int elem_bytes, double *nu)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) nu[j] = or_fixed_order_sumsq(A + j * lda, m, elem_bytes);
}

/* Row squared norms of the gathered m x g block D (column-major, ld = m):
 * rho_i = sum over the g columns in their stored (ascending index) order,
 * rho = fma(d, d, rho).  Eq. (CTSVD_prob), q_i = |d^i|^2 / |D|_F^2. */
void or_row_sqnorms(const double *D, int64_t m, int64_t g, double *rho)
{
    for (int64_t i = 0; i < m; ++i) {
        double a = 0.0;
        for (int64_t l = 0; l < g; ++l) a = fma(D[i + l * m], D[i + l * m], a);
        rho[i] = a;
    }
}

/* ------------------------------------------------------------------------ */
/* Integer sampling weights.  The paper samples with probability             */
/* p_j = nu_j / sum nu (Eq. LTSVD_prob), restricted to the unsampled set S.  */
/* Reading: with B = 63 - ceil(log2 len) and e the binary exponent with      */
/* max(nu) < 2^e, w_j = floor(nu_j * 2^(B-1-e)) (exact in FP64), so that     */
/* sum w < 2^62 and Pr[j] = w_j / sum w.  Weights under one quantum are 0.   */
/* Returns 0, or -1 if a value is negative, infinite or NaN.                 */
/* ------------------------------------------------------------------------ */
int or_quantize(const double *v, int64_t len, uint64_t *w)
{
    int cl = 0;
    while (((int64_t)1 << cl) < len) ++cl;
    const int B = 63 - cl;
    double vmax = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        if (!(v[i] >= 0.0) || isinf(v[i])) return -1;
        if (v[i] > vmax) vmax = v[i];
    }
    if (vmax == 0.0) {
        for (int64_t i = 0; i < len; ++i) w[i] = 0;
        return 0;
    }
    int e;
    (void)frexp(vmax, &e); /* vmax = f * 2^e, 0.5 <= f < 1 */
    for (int64_t i = 0; i < len; ++i) w[i] = (uint64_t)floor(ldexp(v[i], B - 1 - e));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* cnt draws with replacement, Pr[j] = w_j / W, W = sum w.                  */
/* Draw d uses Philox block key = (seed, stream),                           */
/* counter = (iter, floor(d/4), block, 0), word d mod 4 -> u.               */
/* target t = floor(u * W / 2^64); index = min { j : F_j > t } with F the   */
/* inclusive prefix sum of w.  Requires W > 0.  Returns W.                  */
/* ------------------------------------------------------------------------ */
uint64_t or_draw(const uint64_t *w, int64_t len, int32_t cnt, uint64_t seed, uint64_t stream,
                 uint64_t iter, uint64_t block, int64_t *out)
{
    uint64_t *F = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(len > 0 ? len : 1));
    uint64_t run = 0;
    for (int64_t j = 0; j < len; ++j) {
        run += w[j];
        F[j] = run;
    }
    const uint64_t W = run;
    if (W == 0) {
        free(F);
        return 0;
    }
    for (int32_t d = 0; d < cnt; ++d) {
        uint64_t ctr[4] = {iter, (uint64_t)(d / 4), block, 0};
        uint64_t key[2] = {seed, stream};
        uint64_t u[4];
        or_philox4x64_10(ctr, key, u);
        uint64_t t = (uint64_t)(((__uint128_t)u[d % 4] * W) >> 64);
        int64_t lo = 0, hi = len - 1; /* first j with F[j] > t; F[len-1] = W > t */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (F[mid] > t) hi = mid;
            else lo = mid + 1;
        }
        out[d] = lo;
    }
    free(F);
    return W;
}

static int or_cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Distinct values of draws[0..cnt) in ascending order with their
 * multiplicities (Alg. 1: "duplicates are removed", t_hat).  Returns count. */
int32_t or_unique(const int64_t *draws, int32_t cnt, int64_t *uniq, int32_t *counts)
{
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cnt > 0 ? cnt : 1));
    memcpy(tmp, draws, sizeof(int64_t) * (size_t)cnt);
    qsort(tmp, (size_t)cnt, sizeof(int64_t), or_cmp_i64);
    int32_t g = 0;
    for (int32_t d = 0; d < cnt; ++d) {
        if (g > 0 && uniq[g - 1] == tmp[d]) {
            counts[g - 1] += 1;
        } else {
            uniq[g] = tmp[d];
            counts[g] = 1;
            ++g;
        }
    }
    free(tmp);
    return g;
}

/* ------------------------------------------------------------------------ */
/* Householder QR of the m x p matrix X (column-major, ld = m, m >= p).     */
/* On return R (p x p, column-major, upper triangular) and Q (m x p) with   */
/* X = Q R.  X is left unchanged.  Golub & Van Loan, Alg. 5.2.1.            */
/* ------------------------------------------------------------------------ */
void or_householder_qr(const double *X, int64_t m, int64_t p, double *R, double *Q)
{
    double *A = (double *)malloc(sizeof(double) * (size_t)(m * p));
    double *Vh = (double *)calloc((size_t)(m * p), sizeof(double));
    double *beta = (double *)calloc((size_t)p, sizeof(double));
    memcpy(A, X, sizeof(double) * (size_t)(m * p));
    for (int64_t j = 0; j < p; ++j) {
        double *x = A + j * m;
        double nrm2 = 0.0;
        for (int64_t i = j; i < m; ++i) nrm2 += x[i] * x[i];
        double nrm = sqrt(nrm2);
        double *v = Vh + j * m;
        if (nrm == 0.0) {
            beta[j] = 0.0;
            continue;
        }
        double alpha = (x[j] >= 0.0) ? -nrm : nrm;
        for (int64_t i = j; i < m; ++i) v[i] = x[i];
        v[j] = x[j] - alpha;
        double vn2 = 0.0;
        for (int64_t i = j; i < m; ++i) vn2 += v[i] * v[i];
        beta[j] = (vn2 > 0.0) ? 2.0 / vn2 : 0.0;
        /* columns are updated independently: any thread count gives the same bits */
#pragma omp parallel for schedule(static) if ((m - j) * (p - j) > 65536)
        for (int64_t k = j; k < p; ++k) {
            double *a = A + k * m;
            double s = 0.0;
            for (int64_t i = j; i < m; ++i) s += v[i] * a[i];
            s *= beta[j];
            for (int64_t i = j; i < m; ++i) a[i] -= s * v[i];
        }
        x[j] = alpha;
        for (int64_t i = j + 1; i < m; ++i) x[i] = 0.0;
    }
    for (int64_t k = 0; k < p; ++k)
        for (int64_t i = 0; i < p; ++i) R[i + k * p] = (i <= k) ? A[i + k * m] : 0.0;
    /* Q = H_0 H_1 ... H_{p-1} [I_p; 0], accumulated backwards. */
    for (int64_t k = 0; k < p; ++k)
        for (int64_t i = 0; i < m; ++i) Q[i + k * m] = (i == k) ? 1.0 : 0.0;
    for (int64_t j = p - 1; j >= 0; --j) {
        if (beta[j] == 0.0) continue;
        const double *v = Vh + j * m;
#pragma omp parallel for schedule(static) if ((m - j) * (p - j) > 65536)
        for (int64_t k = j; k < p; ++k) {
            double *q = Q + k * m;
            double s = 0.0;
            for (int64_t i = j; i < m; ++i) s += v[i] * q[i];
            s *= beta[j];
            for (int64_t i = j; i < m; ++i) q[i] -= s * v[i];
        }
    }
    free(A);
    free(Vh);
    free(beta);
}

/* ------------------------------------------------------------------------ */
/* One-sided (Hestenes) Jacobi SVD of X (rows x cols, column-major,         */
/* ld = rows).  Columns are rotated pairwise until every pair is orthogonal */
/* to tol = rows * 2^-53 relative (Demmel & Veselic, 1992).  On return      */
/*   sigma[i] = |x_i| sorted descending, U (rows x cols) = x_i / sigma_i    */
/*   (zero column when sigma_i = 0), V (cols x cols, nullable) the          */
/*   accumulated rotations, so X_in V = U diag(sigma).                       */
/* X is left unchanged.  Returns the number of sweeps, or -1 if it did not  */
/* converge in max_sweeps.                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    double s;
    int64_t i;
} or_sv_pair;

static int or_cmp_sv(const void *a, const void *b)
{
    const or_sv_pair *x = (const or_sv_pair *)a, *y = (const or_sv_pair *)b;
    if (x->s > y->s) return -1;
    if (x->s < y->s) return 1;
    return (x->i > y->i) - (x->i < y->i);
}

int or_jacobi_svd(const double *Xin, int64_t rows, int64_t cols, double *sigma, double *U, double *V,
                  int max_sweeps)
{
    double *X = (double *)malloc(sizeof(double) * (size_t)(rows * cols));
    memcpy(X, Xin, sizeof(double) * (size_t)(rows * cols));
    double *Vw = (double *)calloc((size_t)(cols * cols), sizeof(double));
    for (int64_t i = 0; i < cols; ++i) Vw[i + i * cols] = 1.0;
    const double tol = (double)(rows > 1 ? rows : 1) * OR_U64_EPS;
    int sweeps = 0, converged = 0;
    for (sweeps = 1; sweeps <= max_sweeps; ++sweeps) {
        int rotated = 0;
        for (int64_t i = 0; i < cols - 1; ++i) {
            for (int64_t j = i + 1; j < cols; ++j) {
                double *xi = X + i * rows, *xj = X + j * rows;
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int64_t r = 0; r < rows; ++r) {
                    alpha += xi[r] * xi[r];
                    beta += xj[r] * xj[r];
                    gamma += xi[r] * xj[r];
                }
                if (gamma == 0.0 || fabs(gamma) <= tol * sqrt(alpha) * sqrt(beta)) continue;
                rotated = 1;
                double zeta = (beta - alpha) / (2.0 * gamma);
                double t;
                if (fabs(zeta) > 1e150) t = 0.5 / zeta;
                else t = ((zeta >= 0.0) ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = c * t;
                for (int64_t r = 0; r < rows; ++r) {
                    double a = xi[r], b = xj[r];
                    xi[r] = c * a - s * b;
                    xj[r] = s * a + c * b;
                }
                double *vi = Vw + i * cols, *vj = Vw + j * cols;
                for (int64_t r = 0; r < cols; ++r) {
                    double a = vi[r], b = vj[r];
                    vi[r] = c * a - s * b;
                    vj[r] = s * a + c * b;
                }
            }
        }
        if (!rotated) {
            converged = 1;
            break;
        }
    }
    or_sv_pair *pr = (or_sv_pair *)malloc(sizeof(or_sv_pair) * (size_t)(cols > 0 ? cols : 1));
    for (int64_t i = 0; i < cols; ++i) {
        double s2 = 0.0;
        for (int64_t r = 0; r < rows; ++r) s2 += X[r + i * rows] * X[r + i * rows];
        pr[i].s = sqrt(s2);
        pr[i].i = i;
    }
    qsort(pr, (size_t)cols, sizeof(or_sv_pair), or_cmp_sv);
    for (int64_t o = 0; o < cols; ++o) {
        int64_t i = pr[o].i;
        sigma[o] = pr[o].s;
        if (U) {
            for (int64_t r = 0; r < rows; ++r)
                U[r + o * rows] = (pr[o].s > 0.0) ? X[r + i * rows] / pr[o].s : 0.0;
        }
        if (V) {
            for (int64_t r = 0; r < cols; ++r) V[r + o * cols] = Vw[r + i * cols];
        }
    }
    free(pr);
    free(X);
    free(Vw);
    return converged ? sweeps : -1;
}

/* ------------------------------------------------------------------------ */
/* Cyclic two-sided Jacobi eigen-decomposition of the symmetric n x n G     */
/* (Golub & Van Loan, Alg. 8.5.3).  evals sorted descending, evecs columns  */
/* matching.  G is left unchanged.  Returns sweeps or -1.                   */
/* ------------------------------------------------------------------------ */
int or_jacobi_eig(const double *Gin, int64_t n, double *evals, double *evecs, int max_sweeps)
{
    double *A = (double *)malloc(sizeof(double) * (size_t)(n * n));
    memcpy(A, Gin, sizeof(double) * (size_t)(n * n));
    double *Vw = (double *)calloc((size_t)(n * n), sizeof(double));
    for (int64_t i = 0; i < n; ++i) Vw[i + i * n] = 1.0;
    const double tol = (double)(n > 1 ? n : 1) * OR_U64_EPS;
    int sweeps, converged = 0;
    for (sweeps = 1; sweeps <= max_sweeps; ++sweeps) {
        int rotated = 0;
        for (int64_t p = 0; p < n - 1; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                double apq = A[p + q * n];
                double app = A[p + p * n], aqq = A[q + q * n];
                if (apq == 0.0 || fabs(apq) <= tol * sqrt(fabs(app)) * sqrt(fabs(aqq))) continue;
                rotated = 1;
                double tau = (aqq - app) / (2.0 * apq);
                double t;
                if (fabs(tau) > 1e150) t = 0.5 / tau;
                else t = ((tau >= 0.0) ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                for (int64_t k = 0; k < n; ++k) { /* A <- A J */
                    double akp = A[k + p * n], akq = A[k + q * n];
                    A[k + p * n] = c * akp - s * akq;
                    A[k + q * n] = s * akp + c * akq;
                }
                for (int64_t k = 0; k < n; ++k) { /* A <- J^T A */
                    double apk = A[p + k * n], aqk = A[q + k * n];
                    A[p + k * n] = c * apk - s * aqk;
                    A[q + k * n] = s * apk + c * aqk;
                }
                A[p + q * n] = 0.0;
                A[q + p * n] = 0.0;
                for (int64_t k = 0; k < n; ++k) {
                    double vkp = Vw[k + p * n], vkq = Vw[k + q * n];
                    Vw[k + p * n] = c * vkp - s * vkq;
                    Vw[k + q * n] = s * vkp + c * vkq;
                }
            }
        }
        if (!rotated) {
            converged = 1;
            break;
        }
    }
    or_sv_pair *pr = (or_sv_pair *)malloc(sizeof(or_sv_pair) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        pr[i].s = A[i + i * n];
        pr[i].i = i;
    }
    qsort(pr, (size_t)n, sizeof(or_sv_pair), or_cmp_sv);
    for (int64_t o = 0; o < n; ++o) {
        evals[o] = pr[o].s;
        for (int64_t r = 0; r < n; ++r) evecs[r + o * n] = Vw[r + pr[o].i * n];
    }
    free(pr);
    free(A);
    free(Vw);
    return converged ? sweeps : -1;
}

/* ------------------------------------------------------------------------ */
/* Alg. 2 BLOCK MERGE with the second block given as C = U2 S2 (m x g).     */
/* The paper projects U2 on the complement of U1, takes QR of the result    */
/* and assembles E = [[S1, U1^T U2 S2], [0, R S2]]; that E is the R factor  */
/* of [U1 S1 | U2 S2] with Q = [U1 U_o].  Here the QR of [U1 S1 | C] is     */
/* taken directly by Householder reflections (backward stable), then        */
/* SVD(E) = U_E S_E V_E^T by one-sided Jacobi, U = Q U_E, S = S_E, the rank */
/* guard keeps r' = min(r, #{s_i > p u s_1}) and both are truncated.         */
/* U1 is m x r1 (r1 may be 0: first iteration = SVD of C).                   */
/* Returns r' (>= 0) or -1 if the Jacobi SVD did not converge.               */
/* ------------------------------------------------------------------------ */
int32_t or_merge(const double *U1, const double *s1, int64_t m, int32_t r1, const double *C, int32_t g,
                 int32_t r, double *Uout, double *sout)
{
    const int64_t p = (int64_t)r1 + g;
    double *M = (double *)malloc(sizeof(double) * (size_t)(m * p));
    for (int32_t j = 0; j < r1; ++j)
        for (int64_t i = 0; i < m; ++i) M[i + j * m] = U1[i + j * m] * s1[j];
    memcpy(M + (int64_t)r1 * m, C, sizeof(double) * (size_t)(m * g));
    double *Q = (double *)malloc(sizeof(double) * (size_t)(m * p));
    double *E = (double *)malloc(sizeof(double) * (size_t)(p * p));
    or_householder_qr(M, m, p, E, Q);
    double *UE = (double *)malloc(sizeof(double) * (size_t)(p * p));
    double *sE = (double *)malloc(sizeof(double) * (size_t)p);
    int sw = or_jacobi_svd(E, p, p, sE, UE, NULL, 100);
    int32_t rr = 0;
    if (sw >= 0) {
        const double thr = (double)p * OR_U64_EPS * sE[0];
        int32_t nz = 0;
        for (int64_t i = 0; i < p; ++i)
            if (sE[i] > thr) ++nz;
        rr = (r < nz) ? r : nz;
#pragma omp parallel for schedule(static)
        for (int32_t c = 0; c < rr; ++c) {
            sout[c] = sE[c];
            for (int64_t i = 0; i < m; ++i) {
                double a = 0.0;
                for (int64_t l = 0; l < p; ++l) a += Q[i + l * m] * UE[l + c * p];
                Uout[i + c * m] = a;
            }
        }
    }
    free(M);
    free(Q);
    free(E);
    free(UE);
    free(sE);
    return (sw >= 0) ? rr : -1;
}

/* Sines of the principal angles between span(Ua) and span(Ub), both m x k
 * with orthonormal columns (Bjorck & Golub 1973): the singular values of
 * Ub - Ua (Ua^T Ub), descending.  Returns 0 or -1. */
int or_subspace_sines(const double *Ua, const double *Ub, int64_t m, int32_t k, double *sines)
{
    double *P = (double *)malloc(sizeof(double) * (size_t)(k * k));
    for (int32_t a = 0; a < k; ++a)
        for (int32_t b = 0; b < k; ++b) {
            double s = 0.0;
            for (int64_t i = 0; i < m; ++i) s += Ua[i + a * m] * Ub[i + b * m];
            P[a + b * k] = s;
        }
    double *Rm = (double *)malloc(sizeof(double) * (size_t)(m * k));
    for (int32_t b = 0; b < k; ++b)
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int32_t a = 0; a < k; ++a) s += Ua[i + a * m] * P[a + b * k];
            Rm[i + b * m] = Ub[i + b * m] - s;
        }
    int sw = or_jacobi_svd(Rm, m, k, sines, NULL, NULL, 100);
    free(P);
    free(Rm);
    return sw >= 0 ? 0 : -1;
}

/* ------------------------------------------------------------------------ */
/* Final step of Alg. 1, literally: Y = A^T U (n x r); Q, R = QR(Y);         */
/* U_R S_R V_R^T = SVD(R); U <- U V_R; sigma <- S_R; V = Q U_R.              */
/* A is m x n (column-major, ld = lda), U is m x r.  Vout (n x r) nullable. */
/* Returns 0 or -1.                                                         */
/* ------------------------------------------------------------------------ */
int or_project(const double *A, int64_t m, int64_t n, int64_t lda, const double *U, int32_t r, double *Uout,
               double *sigma, double *Vout)
{
    double *Y = (double *)malloc(sizeof(double) * (size_t)(n * r));
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        const double *a = A + j * lda;
        for (int32_t c = 0; c < r; ++c) {
            const double *u = U + (int64_t)c * m;
            double s = 0.0;
            for (int64_t i = 0; i < m; ++i) s += a[i] * u[i];
            Y[j + c * n] = s;
        }
    }
    double *Q = (double *)malloc(sizeof(double) * (size_t)(n * r));
    double *R = (double *)malloc(sizeof(double) * (size_t)(r * r));
    or_householder_qr(Y, n, r, R, Q);
    double *UR = (double *)malloc(sizeof(double) * (size_t)(r * r));
    double *VR = (double *)malloc(sizeof(double) * (size_t)(r * r));
    int sw = or_jacobi_svd(R, r, r, sigma, UR, VR, 100);
#pragma omp parallel for schedule(static)
    for (int32_t c = 0; c < r; ++c)
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int32_t l = 0; l < r; ++l) s += U[i + (int64_t)l * m] * VR[l + c * r];
            Uout[i + (int64_t)c * m] = s;
        }
    if (Vout) {
        for (int32_t c = 0; c < r; ++c)
            for (int64_t j = 0; j < n; ++j) {
                double s = 0.0;
                for (int32_t l = 0; l < r; ++l) s += Q[j + (int64_t)l * n] * UR[l + c * r];
                Vout[j + (int64_t)c * n] = s;
            }
    }
    free(Y);
    free(Q);
    free(R);
    free(UR);
    free(VR);
    return sw >= 0 ? 0 : -1;
}

// pod_big.h -- FP64 kernels for the small matrices of wide merges
// (64 < n <= 160), one workgroup of 512 threads (8 waves).  The matrices live
// in the device workspace (L2 resident) between the stages; the
// tridiagonalisation keeps its matrix in registers, the back-transformation
// its vectors, and the products run on the FP64 matrix cores.
#pragma once

#include "pod_rl.h"

namespace pod {

// Broadcast of lane O of each aligned group of 8 lanes to the whole group
// (a quad_perm broadcast, then a half-row mirror for the other quad).
template <int O> __device__ __forceinline__ double bcast8(double v)
{
    constexpr int q = O & 3;
    constexpr int ctrl = q | (q << 2) | (q << 4) | (q << 6);
    const double v1 = dpp_f64<ctrl>(v);
    const double v2 = dpp_f64<0x141>(v1);
    return (((threadIdx.x >> 2) & 1) == (O >> 2)) ? v1 : v2;
}

constexpr int BIG_NR = 20;   // rows per wave: row a = w + 8 k, k < BIG_NR (n <= 160)
constexpr int BIG_NS = 3;    // column slots per lane: column l + 64 s

// ---------------------------------------------------------------------------
// C = A B for n x n operands (n <= 160) on v_mfma_f64_16x16x4: the 16 x 16
// output tiles are dealt to the 8 waves, operands read through accessors
// (zero outside n x n), the k range of tile (I, J) set by krange(I, J, k0, k1)
// to [k0, k1) (multiples of 16; default [0, 16 ceil(n / 16))) for triangular
// factors.  `upper`: only tiles I <= J.  No barrier; the caller synchronises.
// ---------------------------------------------------------------------------
template <typename FA, typename FB, typename FC, typename FK>
__device__ __forceinline__ void big_mm(int n, bool upper, FA fa, FB fb, FC fc, FK krange)
{
    const int w = rl_wave(), l = rl_lane();
    const int li = l & 15, lk = l >> 4;
    const int nt = (n + 15) >> 4;
    for (int tile = w; tile < nt * nt; tile += 8) {
        const int ti = tile / nt, tj = tile % nt;
        if (upper && ti > tj) continue;
        int k0 = 0, k1 = 16 * nt;
        krange(ti, tj, k0, k1);
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        for (int k = k0; k < k1; k += 16) {
            double av[4], bv[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = k + 4 * s + lk;
                av[s] = fa(ti * 16 + li, kk);
                bv[s] = fb(kk, tj * 16 + li);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = mfma16x16x4(av[s], bv[s], acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) fc(ti * 16 + acc_row<double>(l, v), tj * 16 + li, acc[v]);
    }
}

// ---------------------------------------------------------------------------
// Householder tridiagonalisation T = Q^T A Q of the symmetric n x n matrix A
// (64 < n <= 160; column-major, ld n, in device memory), Golub & Van Loan
// Alg. 8.3.1, Q = H_0 ... H_{n-3}, H_j = I - tau_j v_j v_j^T, with the matrix
// in registers: wave w keeps rows a = w + 8k (k < 20), lane l columns
// l + 64s (s < 3).  Step j: the wave owning row j (= column j) forms v_j from
// its entries right of the diagonal and publishes it; each wave adds its
// rows' share of p = tau A v (by symmetry a column sum over its rows); after
// the second barrier every wave has p, K = tau/2 p^T v, w = p - K v and
// applies A <- A - v w^T - w v^T to its rows.  Two barriers per step.
// On return d (n), e (n - 1) and tau (n) are in LDS and v_j is stored in
// A(j+1:n, j) (the layout of tridiag_backtransform and big_backtransform);
// the rest of A is overwritten.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void big_tridiag(double *A, int n, double *d, double *e, double *tau)
{
    __shared__ double vs[BIG_NS * 64];
    __shared__ double Pp[8][BIG_NS * 64];
    const int w = rl_wave(), l = rl_lane();
    double r[BIG_NR][BIG_NS];
#pragma unroll
    for (int k = 0; k < BIG_NR; ++k) {
        const int a = w + 8 * k;
#pragma unroll
        for (int s = 0; s < BIG_NS; ++s) {
            const int c = l + 64 * s;
            r[k][s] = (a < n && c < n) ? A[c + (size_t)a * n] : 0.0;   // row a = column a
        }
    }
    __syncthreads();   // every wave has read A before the reflectors overwrite it
#pragma unroll
    for (int J = 0; J < BIG_NR; ++J) {
        for (int w0 = 0; w0 < 8; ++w0) {
            const int j = 8 * J + w0;
            if (j >= n) break;
            if (j + 2 >= n) {
                // the trailing 2 x 2 block is already tridiagonal
                if (w == w0) {
                    const int sj = j >> 6, sj1 = (j + 1 < n) ? (j + 1) >> 6 : sj;
                    const double xj = (sj == 0) ? r[J][0] : ((sj == 1) ? r[J][1] : r[J][2]);
                    const double xj1 = (sj1 == 0) ? r[J][0] : ((sj1 == 1) ? r[J][1] : r[J][2]);
                    const double dj = readlane_f64(xj, j & 63);
                    const double ej = readlane_f64(xj1, (j + 1 < n) ? ((j + 1) & 63) : (j & 63));
                    if (l == 0) {
                        d[j] = dj;
                        if (j + 1 < n) e[j] = ej;
                        tau[j] = 0.0;
                    }
                }
                continue;
            }
            if (w == w0) {
                const int sj = j >> 6, sj1 = (j + 1) >> 6;
                const double xj = (sj == 0) ? r[J][0] : ((sj == 1) ? r[J][1] : r[J][2]);
                const double xj1 = (sj1 == 0) ? r[J][0] : ((sj1 == 1) ? r[J][1] : r[J][2]);
                const double dj = readlane_f64(xj, j & 63);
                const double x0 = readlane_f64(xj1, (j + 1) & 63);
                double xv[BIG_NS], sq = 0.0;
#pragma unroll
                for (int s = 0; s < BIG_NS; ++s) {
                    const int c = l + 64 * s;
                    xv[s] = (c > j && c < n) ? r[J][s] : 0.0;
                    sq = fma(xv[s], xv[s], sq);
                }
                const double ss = wave_sum(sq);
                double alpha, tj;
                if (ss > 0.0 && (ss - x0 * x0) > 0.0) {
                    const double nrm = ss * rsqrt_nr(ss);
                    alpha = (x0 >= 0.0) ? -nrm : nrm;
                    tj = rcp_nr(alpha * alpha - alpha * x0);   // > 0: alpha^2 - alpha x0 = ss + |alpha x0|
                } else {
                    alpha = x0;   // column already reduced
                    tj = 0.0;
                }
#pragma unroll
                for (int s = 0; s < BIG_NS; ++s) {
                    const int c = l + 64 * s;
                    const double v = (c == j + 1) ? x0 - alpha : xv[s];
                    vs[c] = v;
                    if (c > j && c < n) A[c + (size_t)j * n] = v;
                }
                if (l == 0) {
                    tau[j] = tj;
                    d[j] = dj;
                    e[j] = alpha;
                }
            }
            __syncthreads();
            // tau_j = 0 (a column already reduced) gives p = w = 0: no update, no branch
            const double tj = tau[j];
            // column slots s < s0 = J / 8 lie entirely left of column j + 1, where v, p
            // and w vanish: they take no part (s0 is fixed by the unrolled J)
            const int s0 = J >> 3;
            double vl[BIG_NS];
#pragma unroll
            for (int s = 0; s < BIG_NS; ++s) vl[s] = (s >= s0) ? vs[l + 64 * s] : 0.0;
            // v_j is zero outside rows j+1..n-1: rows a <= j (k < J) take no part
            double va[BIG_NR];
#pragma unroll
            for (int k = J; k < BIG_NR; ++k) va[k] = vs[w + 8 * k];
#pragma unroll
            for (int s = 0; s < BIG_NS; ++s) {
                if (s < s0) continue;
                double pa[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k = J; k < BIG_NR; ++k) pa[k & 3] = fma(r[k][s], va[k], pa[k & 3]);
                Pp[w][l + 64 * s] = (pa[0] + pa[1]) + (pa[2] + pa[3]);
            }
            __syncthreads();
            double pl[BIG_NS], kp = 0.0;
#pragma unroll
            for (int s = 0; s < BIG_NS; ++s) {
                pl[s] = 0.0;
                if (s < s0) continue;
                const int c = l + 64 * s;
                double pq[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) pq[q] = Pp[q][c];
                const double sum = ((pq[0] + pq[1]) + (pq[2] + pq[3])) + ((pq[4] + pq[5]) + (pq[6] + pq[7]));
                pl[s] = (c > j && c < n) ? tj * sum : 0.0;
                kp = fma(pl[s], vl[s], kp);
            }
            const double K = 0.5 * tj * wave_sum(kp);
            double wl[BIG_NS];
#pragma unroll
            for (int s = 0; s < BIG_NS; ++s) wl[s] = fma(-K, vl[s], pl[s]);
#pragma unroll
            for (int k = J; k < BIG_NR; ++k) {
                // w at column a = w + 8k: slot (8k) / 64 = k / 8 >= s0 is fixed by k (w < 8)
                const double wa = readlane_f64(wl[(8 * k) >> 6], (w + 8 * k) & 63);   // zero for a <= j, a >= n
#pragma unroll
                for (int s = 0; s < BIG_NS; ++s)
                    if (s >= s0) r[k][s] = fma(-va[k], wl[s], fma(-wa, vl[s], r[k][s]));
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Y (n x nv, column-major, ld n, device memory; n <= 160) <- Q Y with the
// reflectors of big_tridiag (v_j in A(j+1:n, j), tau in LDS).  A group of 8
// lanes owns one column (rows g + 8t in registers) and applies every
// reflector to it; the reflectors are staged in LDS in blocks of BT_NB (the
// next block while the current one is applied), one barrier per block.
// ---------------------------------------------------------------------------
constexpr int BT_NB = 4;

__device__ __forceinline__ void big_backtransform(const double *A, const double *tau, int n, double *Y, int nv)
{
    __shared__ double Vb[2][BT_NB][BIG_NS * 64];
    const int g = threadIdx.x & 7;
    const int nref = n - 2;                       // reflectors j = 0 .. n-3, applied from the last
    const int nblk = (nref + BT_NB - 1) / BT_NB;
    auto stage = [&](int q, int buf) {
        for (int idx = threadIdx.x; idx < BT_NB * BIG_NS * 64; idx += EIG_NT) {
            const int i = idx / (BIG_NS * 64), row = idx % (BIG_NS * 64);
            const int j = n - 3 - (BT_NB * q + i);
            Vb[buf][i][row] = (j >= 0 && row > j && row < n) ? A[row + (size_t)j * n] : 0.0;
        }
    };
    for (int cb = 0; cb < nv; cb += EIG_NT / 8) {
        const int c = cb + (threadIdx.x >> 3);   // whole groups share c
        const bool act = c < nv;
        double y[BIG_NR];
#pragma unroll
        for (int t = 0; t < BIG_NR; ++t) y[t] = (act && g + 8 * t < n) ? Y[g + 8 * t + (size_t)c * n] : 0.0;
        stage(0, 0);
        __syncthreads();
        for (int q = 0; q < nblk; ++q) {
            if (q + 1 < nblk) stage(q + 1, (q + 1) & 1);
            const double(*V)[BIG_NS * 64] = Vb[q & 1];
#pragma unroll
            for (int i = 0; i < BT_NB; ++i) {
                const int j = n - 3 - (BT_NB * q + i);
                if (j < 0) break;
                const double tj = tau[j];
                double s0 = 0.0, s1 = 0.0;
#pragma unroll
                for (int t = 0; t < BIG_NR; t += 2) {
                    s0 = fma(V[i][g + 8 * t], y[t], s0);
                    s1 = fma(V[i][g + 8 * t + 8], y[t + 1], s1);
                }
                const double s = tj * group_sum<8>(s0 + s1);
#pragma unroll
                for (int t = 0; t < BIG_NR; ++t) y[t] = fma(-s, V[i][g + 8 * t], y[t]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int t = 0; t < BIG_NR; ++t)
            if (act && g + 8 * t < n) Y[g + 8 * t + (size_t)c * n] = y[t];
    }
    __syncthreads();
}

}  // namespace pod

namespace pod {

// Row of register k in wave w in the layout of big_chol: wave w keeps the
// row blocks of four 4 (w + 8 q) .. 4 (w + 8 q) + 3 (k = 4 q + t).
__device__ __forceinline__ int big_chol_row(int w, int k) { return 32 * (k >> 2) + 4 * w + (k & 3); }

// ---------------------------------------------------------------------------
// In-place Cholesky S = R^T R of the symmetric n x n matrix S (64 < n <= 160;
// column-major, ld n, device memory; the upper triangle is read), the
// contract of chol_upper: on success the upper triangle holds R and the
// strict lower triangle is zero; returns nonzero, uniformly, when a pivot is
// not above thr.  Outer-product Cholesky (Golub & Van Loan Alg. 4.2.2) with
// the matrix in registers (lane l columns l + 64 s), rows in blocks of four
// held by one wave: the owner scales row j by 1/sqrt(pivot) and subtracts
// R(j, a) times it from the block's later rows a, then publishes the block;
// after one barrier every wave subtracts the block's rows from its rows
// below it.  The published blocks alternate between two LDS buffers, so one
// barrier per block suffices.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int big_chol(double *S, int n, double thr)
{
    __shared__ double Rb[2][4][BIG_NS * 64];
    __shared__ int sfl[8];
    const int w = rl_wave(), l = rl_lane();
    double r[BIG_NR][BIG_NS];
#pragma unroll
    for (int k = 0; k < BIG_NR; ++k) {
        const int a = big_chol_row(w, k);
#pragma unroll
        for (int s = 0; s < BIG_NS; ++s) {
            const int c = l + 64 * s;
            r[k][s] = (a < n && c < n) ? S[(c < a ? c + (size_t)a * n : a + (size_t)c * n)] : 0.0;
        }
    }
    int fail = 0;
#pragma unroll
    for (int H = 0; H < BIG_NR / 4; ++H) {
        const int sj = H >> 1;   // column slot of the block's rows 32 H .. 32 H + 31
        for (int b = 0; b < 8; ++b) {
            const int j0 = 32 * H + 4 * b;   // the block's first row; wave b owns it
            if (j0 >= n) break;
            double(*Rs)[BIG_NS * 64] = Rb[(4 * H + b) & 1];
            if (w == b) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int j = j0 + t;
                    if (j < n) {
                        const double d = readlane_f64(r[4 * H + t][sj], j & 63);
                        if (!(d > thr)) fail = 1;
                        const double sc = rsqrt_nr(fmax(d, 1e-300));
#pragma unroll
                        for (int s = 0; s < BIG_NS; ++s) {
                            const int c = l + 64 * s;
                            r[4 * H + t][s] = (c >= j) ? r[4 * H + t][s] * sc : 0.0;
                        }
#pragma unroll
                        for (int u = t + 1; u < 4; ++u) {
                            const double cf = readlane_f64(r[4 * H + t][sj], (j0 + u) & 63);   // R(j, j0 + u)
                            if (j0 + u < n) {
#pragma unroll
                                for (int s = sj; s < BIG_NS; ++s)
                                    r[4 * H + u][s] = fma(-cf, r[4 * H + t][s], r[4 * H + u][s]);
                            }
                        }
                    }
#pragma unroll
                    for (int s = 0; s < BIG_NS; ++s) Rs[t][l + 64 * s] = r[4 * H + t][s];
                }
            }
            __syncthreads();
            // (the block's rows vanish left of column j0 >= 32 H: slots s < sj = H / 2
            // take no part)
            double rj[4][BIG_NS];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int s = sj; s < BIG_NS; ++s) rj[t][s] = Rs[t][l + 64 * s];
#pragma unroll
            for (int k = 4 * H; k < BIG_NR; ++k) {
                const int a = big_chol_row(w, k);
                if (a > j0 + 3 && a < n) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const double cf = Rs[t][a];   // R(j0 + t, a)
#pragma unroll
                        for (int s = sj; s < BIG_NS; ++s) r[k][s] = fma(-cf, rj[t][s], r[k][s]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < BIG_NR; ++k) {
        const int a = big_chol_row(w, k);
        if (a < n) {
#pragma unroll
            for (int s = 0; s < BIG_NS; ++s) {
                const int c = l + 64 * s;
                if (c < n) {
                    S[a + (size_t)c * n] = (c >= a) ? r[k][s] : 0.0;
                    if (c > a) S[c + (size_t)a * n] = 0.0;
                }
            }
        }
    }
    if (l == 0) sfl[w] = fail;
    __syncthreads();
    int f = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) f |= sfl[q];
    __syncthreads();
    return f;
}

}  // namespace pod

namespace pod {

// ---------------------------------------------------------------------------
// Inverse iteration for the tridiagonal (d, e) of a wide merge: the method and
// arithmetic of tri_invit (LU with partial pivoting of T - lambda I, two
// solves from a fixed start vector, re-orthogonalisation inside clusters of
// relatively close eigenvalues), with one lane of wave 0 per cluster (64 at
// a time), each lane's factors in the device scratch W (BIG_INVIT_DOUBLES)
// and its iterate in LDS (yl, EIG_NMAX * 64 doubles), element i of lane t at
// i * 64 + t (the lanes, which walk the rows in step, touch consecutive
// addresses).  Y (n x nv, ld n) receives unit vectors.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void big_invit(const double *d, const double *e, int n, const double *ev, int nv,
                                          double *Y, double *W, double *yl, int *scl)
{
    constexpr int S = 64;
    constexpr size_t A = (size_t)EIG_NMAX * S;   // one array of the scratch
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
    for (int cb = 0; cb < nc; cb += S) {
        const int c = cb + t;
        if (t < S && c < nc) {
            double *u1 = W + t, *u2 = u1 + A, *u3 = u2 + A, *ml = u3 + A, *sw = ml + A, *y = yl + t;
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
                    u1[i * S] = ip;
                    u2[i * S] = p1;
                    u3[i * S] = p2;
                    ml[i * S] = mult;
                    sw[i * S] = swap ? 1.0 : 0.0;
                    r0 = o1 - mult * p1;
                    r1 = o2 - mult * p2;
                    r2 = 0.0;
                }
                if (r0 == 0.0) r0 = u * tn + 1e-300;
                u1[(n - 1) * S] = rcp_nr(r0);
                u2[(n - 1) * S] = 0.0;
                u3[(n - 1) * S] = 0.0;
                // start vector: fixed, not orthogonal to any eigenvector in practice
                for (int i = 0; i < n; ++i)
                    y[i * S] = 1.0 + 0.5 * (double)(((i + 3 * mi) * 2654435761u) % 1009u) / 1009.0;
                for (int itn = 0; itn < 2; ++itn) {
                    // forward: the row operations, carrying the current row in a register
                    double cur = y[0];
#pragma unroll 8
                    for (int i = 0; i + 1 < n; ++i) {
                        const double nx = y[(i + 1) * S];
                        const bool s = sw[i * S] != 0.0;
                        const double top = s ? nx : cur, bot = s ? cur : nx;
                        y[i * S] = top;
                        cur = bot - ml[i * S] * top;
                    }
                    y[(n - 1) * S] = cur;
                    // back substitution with U (3 diagonals), last two values in registers
                    double x1 = 0.0, x2 = 0.0;
#pragma unroll 8
                    for (int i = n - 1; i >= 0; --i) {
                        const double sv = (y[i * S] - u2[i * S] * x1 - u3[i * S] * x2) * u1[i * S];
                        y[i * S] = sv;
                        x2 = x1;
                        x1 = sv;
                    }
                    // re-orthogonalise inside the cluster, normalise
                    for (int pj = i0; pj < mi; ++pj) {
                        const double *z = Y + (size_t)pj * n;
                        double dt = 0.0;
#pragma unroll 8
                        for (int i = 0; i < n; ++i) dt += z[i] * y[i * S];
#pragma unroll 8
                        for (int i = 0; i < n; ++i) y[i * S] -= dt * z[i];
                    }
                    double m4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
                    for (int i = 0; i < n; ++i) m4[i & 3] = fmax(m4[i & 3], fabs(y[i * S]));
                    const double mx = fmax(fmax(m4[0], m4[1]), fmax(m4[2], m4[3]));
                    const double sm = (mx > 0.0) ? 1.0 / mx : 1.0;
                    double q4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
                    for (int i = 0; i < n; ++i) {
                        const double v = y[i * S] * sm;
                        q4[i & 3] += v * v;
                    }
                    const double f = sm / sqrt((q4[0] + q4[1]) + (q4[2] + q4[3]));
#pragma unroll 8
                    for (int i = 0; i < n; ++i) y[i * S] *= f;
                }
                double *yo = Y + (size_t)mi * n;
                for (int i = 0; i < n; ++i) yo[i] = y[i * S];
            }
        }
        __syncthreads();
    }
}

}  // namespace pod

namespace pod {

// ---------------------------------------------------------------------------
// Sturm counts and multisection for the tridiagonal of a wide merge
// (n <= 160): the division-free minor recurrence of sturm_rl on the same
// power-of-two scaled tridiagonal, its entries in LDS (`sde`: BIG_SDE_LD
// scaled diagonal entries, padded, then as many scaled squared couplings).
// ---------------------------------------------------------------------------
constexpr int BIG_SDE_LD = EIG_NMAX + 8;
constexpr int BIG_TRI_SDE = 2 * BIG_SDE_LD;

struct BigTri {
    double lo, hi, pivmin, tn;
    double sc;          // power of two with sc * max(|lo|, |hi|) in [0.5, 1)
    const double *sde;
};

// Every thread calls this (it ends with a barrier).
__device__ __forceinline__ BigTri big_tri(const double *d, const double *e, int n, double *sde)
{
    const int l = rl_lane();
    const double u = 1.1102230246251565e-16;
    const double inf = __builtin_huge_val();
    double lo = inf, hi = -inf, emax = 0.0, tn = 0.0;
#pragma unroll
    for (int s = 0; s < BIG_NS; ++s) {
        const int i = l + 64 * s;
        if (i < n) {
            const double di = d[i], ei = (i + 1 < n) ? e[i] : 0.0, em = (i >= 1) ? e[i - 1] : 0.0;
            const double rad = fabs(em) + fabs(ei);
            lo = fmin(lo, di - rad);
            hi = fmax(hi, di + rad);
            emax = fmax(emax, ei * ei);
            tn = fmax(tn, fabs(di) + fabs(ei));
        }
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    emax = wave_max(emax);
    BigTri t;
    t.tn = wave_max(tn);
    t.pivmin = 2.2250738585072014e-308 * fmax(1.0, emax) * 4.0;
    const double wid = fmax(fabs(lo), fabs(hi));
    t.lo = lo - 2.0 * u * wid * n - 2.0 * t.pivmin;
    t.hi = hi + 2.0 * u * wid * n + 2.0 * t.pivmin;
    const double big = fmax(fabs(t.lo), fabs(t.hi));
    t.sc = (big > 0.0 && big < inf) ? ldexp(1.0, -ilogb(big) - 1) : 1.0;
    for (int i = threadIdx.x; i < BIG_SDE_LD; i += EIG_NT) {
        // padded rows: d - x > 0 and no coupling (see sturm_rl)
        const double es = (i + 1 < n) ? e[i] * t.sc : 0.0;
        sde[i] = (i < n) ? d[i] * t.sc : 4.0;
        sde[BIG_SDE_LD + i] = (i + 1 < n) ? fmax(es * es, 0x1p-200) : 0.0;
    }
    t.sde = sde;
    __syncthreads();
    return t;
}

// Number of eigenvalues below x (the recurrence and sign counting of sturm_rl).
__device__ __forceinline__ int big_sturm(const BigTri &t, int n, double x)
{
    n = opaque_uniform(n);
    const double xs = x * t.sc;
    const double *ds = t.sde, *e2 = t.sde + BIG_SDE_LD;
    double pm1 = 1.0, pm2 = 0.0, mc = 0.0;
    unsigned cnt = 0, sg = 0;
    double dn[8], en[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        dn[q] = ds[q];
        en[q] = e2[q];
    }
    for (int b = 0; b < n; b += 8) {   // (the next block's entries are loaded a block ahead)
        double dc[8], ec[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            dc[q] = dn[q];
            ec[q] = en[q];
            dn[q] = ds[b + 8 + q];
            en[q] = e2[b + 8 + q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            double mn = -ec[q] * pm1;
            double p = fma(dc[q] - xs, pm1, mc);
            if ((q & 3) == 3) {
                const int ex = max(frexp_e(pm1), frexp_e(pm2));
                p = ldexp(p, -ex);
                mn = ldexp(mn, -ex);
                pm1 = ldexp(pm1, -ex);
            }
            sg = __builtin_amdgcn_alignbit(sg, (unsigned)__double2hiint(p), 31);
            pm2 = pm1;
            pm1 = p;
            mc = mn;
        }
        cnt += __popc((sg ^ (sg >> 1)) & 0xFFu);
        sg &= 1u;
    }
    return (int)cnt;
}

// The nv largest eigenvalues (descending) into ev by multisection (the
// rounds of bisect_top_rl with big_sturm).
__device__ __forceinline__ void big_bisect_top(const BigTri &t, int n, int nv, double *ev)
{
    const int tid = threadIdx.x, lane = tid & 63;
    const double u = 1.1102230246251565e-16;
    int G = 64;
    while (G > 1 && nv * G > EIG_NT) G >>= 1;
    const int grp = tid / G, gl = tid % G;
    const bool active = grp < nv;
    const int idx = n - 1 - grp;   // ascending index of the target eigenvalue
    const int gbase = lane - gl;
    const double atol = 4.0 * u * fmax(fabs(t.lo), fabs(t.hi));
    double a = t.lo, b = t.hi;
    for (int round = 0; round < 80; ++round) {
        const bool done = !active || (b - a) <= fmax(2.0 * u * fmax(fabs(a), fabs(b)), atol) + 4.0 * t.pivmin;
        if (__all(done)) break;
        const double x = a + (b - a) * (double)(gl + 1) / (double)(G + 1);
        const int cnt = done ? 0 : big_sturm(t, n, x);
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

}  // namespace pod

namespace pod {

// LDS of a packed upper triangle of the widest merge
constexpr int BIG_PACKED = EIG_NMAX * (EIG_NMAX + 1) / 2;

// ---------------------------------------------------------------------------
// X = R^-1 for the upper-triangular n x n matrix R (n <= 160; column-major,
// ld n, device memory; X must not alias R): the column-by-column back
// substitution of trinv_cols (one group of 8 lanes per column of X, its
// right-hand side in registers, no barrier between the steps) with R's upper
// triangle first copied to LDS, packed by columns (column i at i (i + 1) / 2:
// Rp, BIG_PACKED doubles), so that every step reads LDS instead of L2.
// `tmp` (n doubles of LDS) holds the reciprocals of the diagonal.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void big_trinv(const double *R, int n, double *X, double *Rp, double *tmp)
{
    for (int i = threadIdx.x; i < n; i += EIG_NT) tmp[i] = 1.0 / R[i + i * n];
    for (int c = rl_wave(); c < n; c += 8)
        for (int r = rl_lane(); r <= c; r += 64) Rp[c * (c + 1) / 2 + r] = R[r + (size_t)c * n];
    __syncthreads();
    const int gl = threadIdx.x & 7;
    for (int j = threadIdx.x >> 3; j < n; j += EIG_NT / 8) {
        double b[BIG_NR];
#pragma unroll
        for (int s = 0; s < BIG_NR; ++s) b[s] = (8 * s + gl == j) ? 1.0 : 0.0;
#pragma unroll
        for (int s = BIG_NR - 1; s >= 0; --s) {
            if (8 * s > j) continue;   // uniform in the group
            double bs = b[s];
#pragma unroll 1
            for (int o = 7; o >= 0; --o) {
                const int i = 8 * s + o;
                if (i > j) continue;
                double bi;
                switch (o) {
                case 0: bi = bcast8<0>(bs); break;
                case 1: bi = bcast8<1>(bs); break;
                case 2: bi = bcast8<2>(bs); break;
                case 3: bi = bcast8<3>(bs); break;
                case 4: bi = bcast8<4>(bs); break;
                case 5: bi = bcast8<5>(bs); break;
                case 6: bi = bcast8<6>(bs); break;
                default: bi = bcast8<7>(bs); break;
                }
                const double xi = bi * tmp[i];
                if (gl == o) X[i + (size_t)j * n] = xi;
                // rows of this slot below lane o, then the earlier slots (all above row i)
                const double *col = Rp + i * (i + 1) / 2;
                if (gl < o) bs -= col[8 * s + gl] * xi;
#pragma unroll
                for (int s2 = 0; s2 < s; ++s2) b[s2] -= col[8 * s2 + gl] * xi;
            }
        }
        for (int l = j + 1 + gl; l < n; l += 8) X[l + (size_t)j * n] = 0.0;
    }
    __syncthreads();
}

}  // namespace pod

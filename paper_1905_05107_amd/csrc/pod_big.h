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
// One 16 x 16 tile (ti, tj) of C = A B on v_mfma_f64_16x16x4 by one wave,
// summing k over [k0, k1) (multiples of 16), operands read through accessors
// fa(i, k), fb(k, j) that return zero outside the matrices; the operands of
// step k + 16 are loaded before the products of step k.  The result goes to
// fc(i, j, v) for the tile's 256 entries.
// ---------------------------------------------------------------------------
template <typename FA, typename FB, typename FC>
__device__ __forceinline__ void mm_tile(int ti, int tj, int k0, int k1, FA fa, FB fb, FC fc)
{
    const int l = rl_lane();
    const int li = l & 15, lk = l >> 4;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    double av[4], bv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        av[s] = fa(ti * 16 + li, k0 + 4 * s + lk);
        bv[s] = fb(k0 + 4 * s + lk, tj * 16 + li);
    }
    for (int k = k0; k < k1; k += 16) {
        double an[4], bn[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int kk = k + 16 + 4 * s + lk;
            an[s] = (k + 16 < k1) ? fa(ti * 16 + li, kk) : 0.0;
            bn[s] = (k + 16 < k1) ? fb(kk, tj * 16 + li) : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = mfma16x16x4(av[s], bv[s], acc);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            av[s] = an[s];
            bv[s] = bn[s];
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) fc(ti * 16 + acc_row<double>(l, v), tj * 16 + li, acc[v]);
}

// The same with every operand of the tile loaded before the first product
// (k1 - k0 <= 16 KS): one round trip to memory per tile, for the kernels whose
// operands come from other workgroups' writes (L2 misses).
template <int KS, typename FA, typename FB, typename FC>
__device__ __forceinline__ void mm_tile_all(int ti, int tj, int k0, int k1, FA fa, FB fb, FC fc)
{
    const int l = rl_lane();
    const int li = l & 15, lk = l >> 4;
    double av[KS][4], bv[KS][4];
#pragma unroll
    for (int q = 0; q < KS; ++q)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int kk = k0 + 16 * q + 4 * s + lk;
            const bool in = k0 + 16 * q < k1;
            av[q][s] = in ? fa(ti * 16 + li, kk) : 0.0;
            bv[q][s] = in ? fb(kk, tj * 16 + li) : 0.0;
        }
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < KS; ++q)
        if (k0 + 16 * q < k1)
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = mfma16x16x4(av[q][s], bv[q][s], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) fc(ti * 16 + acc_row<double>(l, v), tj * 16 + li, acc[v]);
}

// ---------------------------------------------------------------------------
// C = A B for n x n operands (n <= 160): the 16 x 16 output tiles of mm_tile
// dealt to the 8 waves, the k range of tile (I, J) set by krange(I, J, k0, k1)
// to [k0, k1) (multiples of 16; default [0, 16 ceil(n / 16))) for triangular
// factors.  `upper`: only tiles I <= J.  No barrier; the caller synchronises.
// ---------------------------------------------------------------------------
template <typename FA, typename FB, typename FC, typename FK>
__device__ __forceinline__ void big_mm(int n, bool upper, FA fa, FB fb, FC fc, FK krange)
{
    const int w = rl_wave();
    const int nt = (n + 15) >> 4;
    for (int tile = w; tile < nt * nt; tile += 8) {
        const int ti = tile / nt, tj = tile % nt;
        if (upper && ti > tj) continue;
        int k0 = 0, k1 = 16 * nt;
        krange(ti, tj, k0, k1);
        mm_tile(ti, tj, k0, k1, fa, fb, fc);
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
            const bool in = a < n && c < n;
            const double v = A[in ? c + (size_t)a * n : 0];   // row a = column a
            r[k][s] = in ? v : 0.0;
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
    // a block of reflectors is loaded into registers while the previous one
    // is applied, and written to LDS after it
    constexpr int PER = (BT_NB * BIG_NS * 64 + EIG_NT - 1) / EIG_NT;
    double pre[PER];
    auto fetch = [&](int q) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = threadIdx.x + u * EIG_NT;
            const int i = idx / (BIG_NS * 64), row = idx % (BIG_NS * 64);
            const int j = n - 3 - (BT_NB * q + i);
            pre[u] = (idx < BT_NB * BIG_NS * 64 && j >= 0 && row > j && row < n) ? A[row + (size_t)j * n] : 0.0;
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = threadIdx.x + u * EIG_NT;
            if (idx < BT_NB * BIG_NS * 64) Vb[buf][idx / (BIG_NS * 64)][idx % (BIG_NS * 64)] = pre[u];
        }
    };
    for (int cb = 0; cb < nv; cb += EIG_NT / 8) {
        const int c = cb + (threadIdx.x >> 3);   // whole groups share c
        const bool act = c < nv;
        double y[BIG_NR];
#pragma unroll
        for (int t = 0; t < BIG_NR; ++t) y[t] = (act && g + 8 * t < n) ? Y[g + 8 * t + (size_t)c * n] : 0.0;
        fetch(0);
        put(0);
        __syncthreads();
        for (int q = 0; q < nblk; ++q) {
            if (q + 1 < nblk) fetch(q + 1);
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
            if (q + 1 < nblk) put((q + 1) & 1);
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
// Cholesky S = R^T R of the symmetric n x n matrix S (64 < n <= 160), read
// through load(i, j) for i <= j (the upper triangle; each entry is read once,
// all of a thread's loads in flight together) and written through
// store(a, c, v) for every c >= a (v = R(a, c)).  Returns, uniformly, bit 1
// when a pivot is not above thr and bit 2 when an entry of S is not finite.
// Outer-product Cholesky (Golub & Van Loan Alg. 4.2.2) with the matrix in
// registers (lane l columns l + 64 s), rows in blocks of four held by one
// wave: the owner scales row j by 1/sqrt(pivot) and subtracts R(j, a) times
// it from the block's later rows a, then publishes the block; after one
// barrier every wave subtracts the block's rows from its rows below it.  The
// published blocks alternate between two LDS buffers, so one barrier per
// block suffices.
// ---------------------------------------------------------------------------
template <typename FL, typename FS>
__device__ __forceinline__ int big_chol(int n, double thr, FL load, FS store)
{
    __shared__ double Rb[2][4][BIG_NS * 64];
    __shared__ int sfl[8];
    const int w = rl_wave(), l = rl_lane();
    double r[BIG_NR][BIG_NS];
    // (every load issued without a branch, from (0, 0) outside the matrix:
    // a load inside a divergent branch would be waited for there)
#pragma unroll
    for (int k = 0; k < BIG_NR; ++k) {
        const int a = big_chol_row(w, k);
#pragma unroll
        for (int s = 0; s < BIG_NS; ++s) {
            const int c = l + 64 * s;
            const bool in = a < n && c < n;
            const double v = load(in ? min(a, c) : 0, in ? max(a, c) : 0);
            r[k][s] = in ? v : 0.0;
        }
    }
    int fail = 0;
#pragma unroll
    for (int k = 0; k < BIG_NR; ++k)
#pragma unroll
        for (int s = 0; s < BIG_NS; ++s)
            if (!isfinite(r[k][s])) fail = 2;
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
                        if (!(d > thr)) fail |= 1;
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
                        // (slots left of row a's diagonal hold its lower triangle,
                        // which no later step reads: slot a / 64 = k / 8 onwards)
#pragma unroll
                        for (int s = (sj > (k >> 3)) ? sj : (k >> 3); s < BIG_NS; ++s)
                            r[k][s] = fma(-cf, rj[t][s], r[k][s]);
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
                if (c < n && c >= a) store(a, c, r[k][s]);
            }
        }
    }
    // (a wave's flag bits: the pivot test is uniform in the owner wave, the
    // finiteness test per lane)
    fail = (__ballot((fail & 1) != 0) ? 1 : 0) | (__ballot((fail & 2) != 0) ? 2 : 0);
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
    constexpr int FB = 6;                         // rows per block of the solves
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
                    // forward: the row operations, carrying the current row in a
                    // register; the operands of the next FB rows are loaded before
                    // the current FB rows are processed (they are rows those do not write)
                    double cur = y[0];
                    double nxb[FB], swb[FB], mlb[FB];
                    auto fwd_load = [&](int i0, double *nx_, double *sw_, double *ml_) {
#pragma unroll
                        for (int q = 0; q < FB; ++q) {
                            const int i = i0 + q;
                            const bool ok = i + 1 < n;
                            nx_[q] = ok ? y[(i + 1) * S] : 0.0;
                            sw_[q] = ok ? sw[i * S] : 0.0;
                            ml_[q] = ok ? ml[i * S] : 0.0;
                        }
                    };
                    fwd_load(0, nxb, swb, mlb);
                    for (int i0 = 0; i0 + 1 < n; i0 += FB) {
                        double nxn[FB], swn[FB], mln[FB];
                        fwd_load(i0 + FB, nxn, swn, mln);
#pragma unroll
                        for (int q = 0; q < FB; ++q) {
                            const int i = i0 + q;
                            if (i + 1 < n) {
                                const bool s = swb[q] != 0.0;
                                const double top = s ? nxb[q] : cur, bot = s ? cur : nxb[q];
                                y[i * S] = top;
                                cur = bot - mlb[q] * top;
                            }
                        }
#pragma unroll
                        for (int q = 0; q < FB; ++q) {
                            nxb[q] = nxn[q];
                            swb[q] = swn[q];
                            mlb[q] = mln[q];
                        }
                    }
                    y[(n - 1) * S] = cur;
                    // back substitution with U (3 diagonals), last two values in
                    // registers, the next FB rows' operands loaded ahead
                    double x1 = 0.0, x2 = 0.0;
                    double yb[FB], ab1[FB], ab2[FB], ab3[FB];
                    auto back_load = [&](int i0, double *y_, double *a1, double *a2, double *a3) {
#pragma unroll
                        for (int q = 0; q < FB; ++q) {
                            const int i = i0 - q;
                            const bool ok = i >= 0;
                            y_[q] = ok ? y[i * S] : 0.0;
                            a1[q] = ok ? u1[i * S] : 0.0;
                            a2[q] = ok ? u2[i * S] : 0.0;
                            a3[q] = ok ? u3[i * S] : 0.0;
                        }
                    };
                    back_load(n - 1, yb, ab1, ab2, ab3);
                    for (int i0 = n - 1; i0 >= 0; i0 -= FB) {
                        double yn[FB], an1[FB], an2[FB], an3[FB];
                        back_load(i0 - FB, yn, an1, an2, an3);
#pragma unroll
                        for (int q = 0; q < FB; ++q) {
                            const int i = i0 - q;
                            if (i >= 0) {
                                const double sv = (yb[q] - ab2[q] * x1 - ab3[q] * x2) * ab1[q];
                                y[i * S] = sv;
                                x2 = x1;
                                x1 = sv;
                            }
                        }
#pragma unroll
                        for (int q = 0; q < FB; ++q) {
                            yb[q] = yn[q];
                            ab1[q] = an1[q];
                            ab2[q] = an2[q];
                            ab3[q] = an3[q];
                        }
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
                for (int i0 = 0; i0 < n; i0 += FB) {
                    double v[FB];
#pragma unroll
                    for (int q = 0; q < FB; ++q) v[q] = (i0 + q < n) ? y[(i0 + q) * S] : 0.0;
#pragma unroll
                    for (int q = 0; q < FB; ++q)
                        if (i0 + q < n) yo[i0 + q] = v[q];
                }
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
// X = R^-1 for the upper-triangular n x n matrix R (n <= 160): the
// column-by-column back substitution of trinv_cols (one group of 8 lanes per
// column of X, its right-hand side in registers, no barrier between the
// steps) on R's upper triangle packed by columns in LDS (column i at
// i (i + 1) / 2: Rp, BIG_PACKED doubles), so that every step reads LDS
// instead of L2; `tmp` (n doubles of LDS) holds the reciprocals of the
// diagonal.  big_trinv_solve hands X(i, j) to store(i, j, x) for every
// i, j < n (zero below the diagonal); no barrier on entry, one on return.
// ---------------------------------------------------------------------------
// Column j of X = R^-1 by the aligned group of 8 lanes that calls it (j < n):
// the back substitution of trinv_cols with the right-hand side e_j in
// registers (row 8 s + g in slot s of group lane g); X(i, j) goes to
// store(i, j, x) for every i < n.
template <typename FS>
__device__ __forceinline__ void trinv_col8(const double *Rp, const double *tmp, int n, int j, FS store)
{
    const int gl = threadIdx.x & 7;
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
            if (gl == o) store(i, j, xi);
            // rows of this slot below lane o, then the earlier slots (all above row i)
            const double *col = Rp + i * (i + 1) / 2;
            if (gl < o) bs -= col[8 * s + gl] * xi;
#pragma unroll
            for (int s2 = 0; s2 < s; ++s2) b[s2] -= col[8 * s2 + gl] * xi;
        }
    }
    for (int l = j + 1 + gl; l < n; l += 8) store(l, j, 0.0);
}

template <typename FS>
__device__ __forceinline__ void big_trinv_solve(const double *Rp, const double *tmp, int n, FS store)
{
    for (int j = threadIdx.x >> 3; j < n; j += EIG_NT / 8) trinv_col8(Rp, tmp, n, j, store);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Inverses of the 16 x 16 diagonal blocks of the upper-triangular n x n R
// (n <= 160; read through rd(i, k) for i <= k < n; identity beyond n), each
// column-major into dinv + 256 I: wave w takes blocks I = w, w + 8, ..., lane
// c < 16 solves column c by back substitution.  No barrier.
// ---------------------------------------------------------------------------
template <typename FR>
__device__ __forceinline__ void diag_inv16(int n, FR rd, double *dinv)
{
    const int l = rl_lane(), c = l & 15;
    const int nt = (n + 15) >> 4;
    for (int I = rl_wave(); I < nt; I += EIG_NT / 64) {
        const int o = 16 * I;
        auto R = [&](int i, int k) -> double { return (o + k < n) ? rd(o + i, o + k) : ((i == k) ? 1.0 : 0.0); };
        double x[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) x[k] = 0.0;
#pragma unroll
        for (int i = 15; i >= 0; --i) {
            if (i > c) continue;
            double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
            for (int k = i + 1; k < 16; ++k) s -= R(i, k) * x[k];   // x[k] = 0 for k > c
            x[i] = s / R(i, i);
        }
        if (l < 16)
#pragma unroll
            for (int i = 0; i < 16; ++i) dinv[256 * I + 16 * c + i] = x[i];
    }
}

// Column j of the packed upper triangle that holds packed index q.
__device__ __forceinline__ int packed_col(int q)
{
    int c = (int)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
    if (c * (c + 1) / 2 > q) --c;
    if ((c + 1) * (c + 2) / 2 <= q) ++c;
    return c;
}

// Rp and tmp of big_trinv_solve from R (column-major, ld n, device memory),
// eight loads in flight per thread; ends with a barrier.
__device__ __forceinline__ void big_tri_pack(const double *R, int n, double *Rp, double *tmp)
{
    const int np = n * (n + 1) / 2;
    for (int q0 = threadIdx.x; q0 < np; q0 += 8 * EIG_NT) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * EIG_NT;
            const int c = packed_col(q);
            v[u] = (q < np) ? R[(q - c * (c + 1) / 2) + (size_t)c * n] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * EIG_NT;
            if (q < np) {
                Rp[q] = v[u];
                const int c = packed_col(q);
                if (q - c * (c + 1) / 2 == c) tmp[c] = 1.0 / v[u];
            }
        }
    }
    __syncthreads();
}

// X = R^-1 (X column-major, ld n, device memory, not aliasing R).
__device__ __forceinline__ void big_trinv(const double *R, int n, double *X, double *Rp, double *tmp)
{
    big_tri_pack(R, n, Rp, tmp);
    big_trinv_solve(Rp, tmp, n, [&](int i, int j, double x) { X[i + (size_t)j * n] = x; });
}

}  // namespace pod

// pod_rl.h -- register-resident FP64 kernels for the small matrices of the
// merge when n <= 64, for one workgroup of 512 threads (8 waves).
//
// Row layout: wave w keeps rows a = w + 8k (k = 0..7) of an n x n matrix in
// r[k], lane l column l; rows and columns from n to 63 hold zeros.  The
// factorisations below eliminate one row per step: the wave that owns it
// finishes it, publishes it in LDS, and after one barrier every wave updates
// its own rows in registers (no LDS round trip per matrix element).  Row-major
// LDS copies use the odd leading dimension RL_LD.  Products of 64 x 64
// operands run on the FP64 MFMA (16 x 16 x 4).
#pragma once

#include "pod_symeig.h"

namespace pod {

constexpr int RL_LD = 65;

__device__ __forceinline__ int rl_wave() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
__device__ __forceinline__ int rl_lane() { return threadIdx.x & 63; }
// Binary exponent e with |v| in [2^(e-1), 2^e) (frexp; 0 for v = 0).
__device__ __forceinline__ int frexp_e(double v) { return __builtin_amdgcn_frexp_exp(v); }
// A wave-uniform int the optimiser cannot see through: tests against it stay
// where they are written instead of being hoisted out of loops as one
// predicate per unrolled step (which exhausts the scalar registers).
__device__ __forceinline__ int opaque_uniform(int v)
{
    v = __builtin_amdgcn_readfirstlane(v);
    asm volatile("" : "+s"(v));
    return v;
}

// Load rows of the symmetric n x n matrix M (column-major, ld) into r: by
// symmetry row a is column a, so the reads are contiguous.
__device__ __forceinline__ void rl_load_sym(double (&r)[8], const double *M, int ld, int n)
{
    const int w = rl_wave(), l = rl_lane();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int a = w + 8 * k;
        r[k] = (a < n && l < n) ? M[l + (size_t)a * ld] : 0.0;
    }
}

// r <- rows of the row-major LDS matrix S (ld RL_LD, 64 rows).
__device__ __forceinline__ void rl_load_rows(double (&r)[8], const double *S)
{
    const int w = rl_wave(), l = rl_lane();
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = S[(w + 8 * k) * RL_LD + l];
}

// Rs = Xs = I_n (64 x 64, zero-padded).
__device__ __forceinline__ void rl_identity(int n, double *Rs, double *Xs)
{
    const int w = rl_wave(), l = rl_lane();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int a = w + 8 * k;
        const double v = (a == l && a < n) ? 1.0 : 0.0;
        Rs[a * RL_LD + l] = v;
        Xs[a * RL_LD + l] = v;
    }
    __syncthreads();
}

// Row of register k in wave w in the layout of rl_cholinv: wave w keeps the
// row blocks 4w..4w+3 (k = 0..3) and 32+4w..32+4w+3 (k = 4..7).
__device__ __forceinline__ int rl_chol_row(int w, int k) { return 4 * w + 32 * (k >> 2) + (k & 3); }

// rl_load_sym in the row layout of rl_cholinv.
__device__ __forceinline__ void rl_load_sym_chol(double (&r)[8], const double *M, int ld, int n)
{
    const int w = rl_wave(), l = rl_lane();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int a = rl_chol_row(w, k);
        r[k] = (a < n && l < n) ? M[l + (size_t)a * ld] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Cholesky G = R^T R of the symmetric matrix in r (upper triangle read; rows
// in the rl_chol_row layout) and X = R^-T alongside: the rows of [G | I] are
// eliminated in order (outer-product Cholesky, Golub & Van Loan Alg. 4.2.2,
// on the augmented matrix, which carries out the forward substitution
// R^T X = I step by step).  Rows go in blocks of four held by one wave: the
// owner scales row j by 1/sqrt(pivot) and subtracts R(j, a) times it from the
// block's later rows a in registers, then publishes the block; after one
// barrier every wave subtracts the block's four rows from its rows below it,
// in row order (the same operations, in the same order, as eliminating one
// row per barrier).  On return Rs and Xs (LDS, row-major, ld RL_LD, 64 rows,
// zero-padded) hold R and X = R^-T (so R^-1(i, j) = Xs[j * RL_LD + i]).
// Returns nonzero, uniformly, when a pivot is not above thr (the factors are
// then garbage).  r is overwritten; `sfl` is 8 ints of LDS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int rl_cholinv(double (&r)[8], int n, double thr, double *Rs, double *Xs, int *sfl)
{
    const int w = rl_wave(), l = rl_lane();
    double x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int a = rl_chol_row(w, k);
        x[k] = (l == a && a < n) ? 1.0 : 0.0;
    }
    int fail = 0;
#pragma unroll
    for (int H = 0; H < 2; ++H) {
        for (int b = 0; b < 8; ++b) {
            const int j0 = 32 * H + 4 * b;   // the block's first row; wave b owns it
            if (j0 >= n) break;
            if (w == b) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int j = j0 + s;
                    if (j < n) {
                        const double d = readlane_f64(r[4 * H + s], j);
                        if (!(d > thr)) fail = 1;
                        const double sc = rsqrt_nr(fmax(d, 1e-300));
                        r[4 * H + s] = (l >= j) ? r[4 * H + s] * sc : 0.0;
                        x[4 * H + s] = x[4 * H + s] * sc;
#pragma unroll
                        for (int t = s + 1; t < 4; ++t) {
                            const double c = readlane_f64(r[4 * H + s], j0 + t);   // R(j, j0 + t)
                            if (j0 + t < n) {
                                r[4 * H + t] -= c * r[4 * H + s];
                                x[4 * H + t] -= c * x[4 * H + s];
                            }
                        }
                    }
                    Rs[j * RL_LD + l] = r[4 * H + s];
                    Xs[j * RL_LD + l] = x[4 * H + s];
                }
            }
            __syncthreads();
            double rj[4], xj[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                rj[s] = Rs[(j0 + s) * RL_LD + l];
                xj[s] = Xs[(j0 + s) * RL_LD + l];
            }
#pragma unroll
            for (int k = 4 * H; k < 8; ++k) {
                const int a = rl_chol_row(w, k);
                if (a > j0 + 3 && a < n) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const double c = Rs[(j0 + s) * RL_LD + a];
                        r[k] -= c * rj[s];
                        x[k] -= c * xj[s];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int a = rl_chol_row(w, k);
        if (a >= n) {
            Rs[a * RL_LD + l] = 0.0;
            Xs[a * RL_LD + l] = 0.0;
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

// ---------------------------------------------------------------------------
// Householder tridiagonalisation T = Q^T A Q of the symmetric matrix in r
// (Golub & Van Loan Alg. 8.3.1), Q = H_0 ... H_{n-3},
// H_j = I - tau_j v_j v_j^T.  Step j: the owner of row j (= column j) forms
// v_j from its entries right of the diagonal and publishes it; each wave adds
// its rows' share of p = tau A v (by symmetry a column sum over its rows);
// after the second barrier every wave has p, K = tau/2 p^T v, w = p - K v and
// applies A <- A - v w^T - w v^T to its rows.  Two barriers per step.
// On return d (n), e (n - 1) and tau (n) are in LDS and v_j is row j of V
// (row-major, ld RL_LD, zero at columns <= j).  Pp: 8 x 64 doubles of LDS.
// r is destroyed.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rl_tridiag(double (&r)[8], int n, double *d, double *e, double *tau, double *V, double *Pp)
{
    const int w = rl_wave(), l = rl_lane();
#pragma unroll
    for (int J = 0; J < 8; ++J) {
        for (int w0 = 0; w0 < 8; ++w0) {
            const int j = 8 * J + w0;
            if (j >= n) break;
            if (j + 2 >= n) {
                // the trailing 2 x 2 block is already tridiagonal
                if (w == w0) {
                    const double dj = readlane_f64(r[J], j);
                    const double ej = readlane_f64(r[J], (j + 1 < n) ? j + 1 : j);
                    if (l == 0) {
                        d[j] = dj;
                        if (j + 1 < n) e[j] = ej;
                        tau[j] = 0.0;
                    }
                }
                continue;
            }
            if (w == w0) {
                const double xr = r[J];
                const double dj = readlane_f64(xr, j);
                const double x0 = readlane_f64(xr, j + 1);
                const double xv = (l > j && l < n) ? xr : 0.0;
                const double ss = wave_sum(xv * xv);
                double alpha, tj;
                if (ss > 0.0 && (ss - x0 * x0) > 0.0) {
                    const double nrm = ss * rsqrt_nr(ss);
                    alpha = (x0 >= 0.0) ? -nrm : nrm;
                    tj = rcp_nr(alpha * alpha - alpha * x0);   // > 0: alpha^2 - alpha x0 = ss + |alpha x0|
                } else {
                    alpha = x0;   // column already reduced
                    tj = 0.0;
                }
                V[j * RL_LD + l] = (l == j + 1) ? x0 - alpha : xv;
                if (l == 0) {
                    tau[j] = tj;
                    d[j] = dj;
                    e[j] = alpha;
                }
            }
            __syncthreads();
            // tau, v_j and the wave's entries of v_j in one LDS round trip.  With
            // tau_j = 0 (a column already reduced) p = w = 0 and the update below
            // leaves every row unchanged, so that step needs no branch.
            const double tj = tau[j];
            const double vl = V[j * RL_LD + l];
            // v_j is zero outside rows j+1..n-1, so rows a <= j and a >= n take
            // no part and no update below without tests
            double va[8];
#pragma unroll
            for (int k = J; k < 8; ++k) va[k] = V[j * RL_LD + w + 8 * k];
            double pa[4] = {0.0, 0.0, 0.0, 0.0};   // four partial sums: a shorter dependency chain
#pragma unroll
            for (int k = J; k < 8; ++k) pa[k & 3] = fma(r[k], va[k], pa[k & 3]);
            Pp[w * 64 + l] = (pa[0] + pa[1]) + (pa[2] + pa[3]);
            __syncthreads();
            double pq[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) pq[q] = Pp[q * 64 + l];
            double pl = ((pq[0] + pq[1]) + (pq[2] + pq[3])) + ((pq[4] + pq[5]) + (pq[6] + pq[7]));
            pl = (l > j && l < n) ? tj * pl : 0.0;
            const double K = 0.5 * tj * wave_sum(pl * vl);
            const double wl = fma(-K, vl, pl);
#pragma unroll
            for (int k = J; k < 8; ++k) {
                const double wa = readlane_f64(wl, w + 8 * k);   // zero for rows <= j and >= n
                r[k] = fma(-va[k], wl, fma(-wa, vl, r[k]));
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Y (n x nv, LDS column-major, ld n) <- Q Y with the reflectors of
// rl_tridiag.  A group of 8 lanes owns one column (rows g + 8t in registers)
// and applies all reflectors to it: no barrier between reflectors.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rl_backtransform(const double *V, const double *tau, int n, double *Y, int nv)
{
    const int g = threadIdx.x & 7;
    const int c = threadIdx.x >> 3;   // whole groups share c
    if (c < nv) {
        double y[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) y[t] = (g + 8 * t < n) ? Y[g + 8 * t + c * n] : 0.0;
        for (int j = n - 3; j >= 0; --j) {
            const double tj = tau[j];
            if (tj == 0.0) continue;   // uniform
            double vv[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) vv[t] = V[j * RL_LD + g + 8 * t];
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < 8; ++t) s += vv[t] * y[t];
            s = tj * group_sum<8>(s);
#pragma unroll
            for (int t = 0; t < 8; ++t) y[t] -= s * vv[t];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (g + 8 * t < n) Y[g + 8 * t + c * n] = y[t];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// The tridiagonal (d, e) of rl_tridiag in registers (n <= 64): lane i holds
// d_i and e_i (e_i couples rows i and i + 1; zero from n - 1 on), every wave
// its own copy.  lo / hi: Gershgorin bounds widened by 2 n u |T| + 2 pivmin;
// pivmin: the pivot floor of the Sturm counts; tn: max_i |d_i| + |e_i|.
// ---------------------------------------------------------------------------
struct TriRegs {
    double d, e, lo, hi, pivmin, tn;
    double sc;          // power of two with sc * max(|lo|, |hi|) in [0.5, 1)
    const double *sde;  // LDS: sc d_i (72, padded with 4) then (sc e_i)^2 floored at 2^-200 (72, padded with 0)
};
constexpr int TRI_SDE = 144;   // doubles of the `sde` scratch
// Every thread calls this (it ends with a barrier); `sde`: TRI_SDE doubles of LDS.
__device__ __forceinline__ TriRegs tri_regs(const double *d, const double *e, int n, double *sde)
{
    const int l = rl_lane();
    const double u = 1.1102230246251565e-16;
    const double inf = __builtin_huge_val();
    TriRegs t;
    t.d = (l < n) ? d[l] : 0.0;
    t.e = (l + 1 < n) ? e[l] : 0.0;
    const double em = (l >= 1 && l < n) ? e[l - 1] : 0.0;
    const double rad = fabs(em) + fabs(t.e);
    const double lo = wave_min((l < n) ? t.d - rad : inf);
    const double hi = wave_max((l < n) ? t.d + rad : -inf);
    const double emax = wave_max(t.e * t.e);
    t.pivmin = 2.2250738585072014e-308 * fmax(1.0, emax) * 4.0;
    const double wid = fmax(fabs(lo), fabs(hi));
    t.lo = lo - 2.0 * u * wid * n - 2.0 * t.pivmin;
    t.hi = hi + 2.0 * u * wid * n + 2.0 * t.pivmin;
    t.tn = wave_max((l < n) ? fabs(t.d) + fabs(t.e) : 0.0);
    const double big = fmax(fabs(t.lo), fabs(t.hi));
    t.sc = (big > 0.0 && big < inf) ? ldexp(1.0, -ilogb(big) - 1) : 1.0;
    if (threadIdx.x < 64) {
        // padded rows: d - x > 0 and no coupling (see sturm_rl)
        const double es = t.e * t.sc;
        sde[l] = (l < n) ? t.d * t.sc : 4.0;
        sde[72 + l] = (l + 1 < n) ? fmax(es * es, 0x1p-200) : 0.0;
        if (l < 8) {
            sde[64 + l] = 4.0;
            sde[136 + l] = 0.0;
        }
    }
    t.sde = sde;
    __syncthreads();
    return t;
}

// Number of eigenvalues below x: sign changes in the sequence of leading
// principal minors of T - x I (Sturm), p_{-1} = 1, p_0 = d_0 - x,
// p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2} (Wilkinson, The Algebraic
// Eigenvalue Problem, ch. 5).  No division: one fused multiply-add per row on
// the dependency chain, against the reciprocal of the equivalent pivot
// recurrence q_i = p_i / p_{i-1}.  The recurrence runs on T scaled by a power
// of two (|T| ~ 1, couplings floored at 2^-100, far below the rounding level
// of the entries) and rescales its last two terms by a power of two every
// fourth row (between rescalings a term changes by at most a factor 3^4 up,
// and the floor bounds how far a pair can fall), which keeps them in range.  A zero minor takes the sign
// opposite to its predecessor (the next one, -e^2 p_{i-1}, then has that sign
// too, so exactly one change is counted, as for a pivot floored at -pivmin).
// The diagonal and couplings are read from the registers by readlane.
__device__ __forceinline__ int sturm_rl(const TriRegs &t, int n, double x)
{
    n = opaque_uniform(n);   // keep the bound tests inside the caller's loops
    const double xs = x * t.sc;
    const double *ds = t.sde, *e2 = t.sde + 72;
    // Step i has pm1 = p_{i-1} and mc = -e_{i-1}^2 p_{i-2}; it forms the next
    // step's term from p_{i-1} before p_i, so that only one multiply-add per row
    // waits on its predecessor.  The sign bits of the minors are shifted into
    // `sg` (one funnel shift per row: sg = sg << 1 | sign(p_i)); after each block
    // of 8 rows the sign changes between neighbours are counted from it at once
    // (a zero of either sign is fine: either sign gives one change across it and
    // its successor).
    double pm1 = 1.0, pm2 = 0.0, mc = 0.0;
    unsigned cnt = 0, sg = 0;   // bit 0: sign of p_{i-1} (p_{-1} = 1 > 0)
    // blocks of 8 rows (the next block's entries loaded ahead); the padded rows
    // past n have d - x > 0 and no coupling, so their minors keep the sign of p_{n-1}
    double dn[8], en[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        dn[q] = ds[q];
        en[q] = e2[q];
    }
    // (unrolled: the next block's loads are issued a block ahead of their use)
#pragma unroll
    for (int b = 0; b < 64; b += 8) {
        if (b >= n) break;
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
                // power-of-two rescaling of the pair (p_i, p_{i-1}) and of the next
                // term, by the exponent of the larger of p_{i-1}, p_{i-2}
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
        // bits 8..0 of sg: the signs of p_{b-1}, p_b, ..., p_{b+7}
        cnt += __popc((sg ^ (sg >> 1)) & 0xFFu);
        sg &= 1u;
    }
    return (int)cnt;
}

// The nv largest eigenvalues (descending) into ev (LDS) by multisection, as
// bisect_top (groups of G lanes, G Sturm counts per round) with the
// tridiagonal in registers.
__device__ __forceinline__ void bisect_top_rl(const TriRegs &t, int n, int nv, double *ev)
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
        const int cnt = done ? 0 : sturm_rl(t, n, x);
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

// Number of eigenvalues above thr (every thread computes it).
__device__ __forceinline__ int count_above_rl(const TriRegs &t, int n, double thr)
{
    return n - sturm_rl(t, n, thr);
}

// ---------------------------------------------------------------------------
// Eigenvectors for ev[0..nv) (descending) by inverse iteration, as tri_invit
// (P L U of T - lambda I with partial pivoting, two solves from a fixed start
// vector, re-orthogonalisation inside clusters of eigenvalues closer than 1e-3
// of their magnitude, normalisation), for n <= 64 on wave 0: one lane per
// cluster, the iterate in its column of Y, the factor in LDS (`lu`, INVIT_LDS
// doubles: per lane the reciprocal pivots, the first super-diagonal of U
// divided by -pivot, and the multipliers; the second super-diagonal and the
// interchanges come from e and a bit mask).  The sweeps are arranged so that
// one multiply-add per row waits on the previous row.  Y (n x nv, ld n, LDS)
// receives unit vectors; `scl` holds the cluster starts.
// ---------------------------------------------------------------------------
constexpr int INVIT_LANES = 24;
constexpr int INVIT_STRIDE = 4 * 64 + 9;   // u1, b, ml (64 each), the iterate (72), odd
constexpr int INVIT_LDS = INVIT_LANES * INVIT_STRIDE;

__device__ __forceinline__ void tri_invit_rl(const TriRegs &t, int n_in, const double *ev, int nv, double *Y, double *lu,
                                             int *scl)
{
    const double u = 1.1102230246251565e-16;
    const int l = rl_lane();
    if (threadIdx.x < 64 && nv > 0) {
        const double evl = (l < nv) ? ev[l] : 0.0;
        const double tn = fmax(t.tn, wave_max(fabs(evl)));
        const double evp = (l >= 1 && l < nv) ? ev[l - 1] : 0.0;
        const bool start =
            (l < nv) && (l == 0 || fabs(evp - evl) > 1e-3 * fmax(fabs(evp), fabs(evl)) + 8.0 * u * tn);
        const unsigned long long bal = __ballot(start);
        const int nc = __popcll(bal);
        if (start) scl[__popcll(bal & ((1ULL << l) - 1))] = l;
        if (l == 0) scl[nc] = nv;
        for (int cb = 0; cb < nc; cb += INVIT_LANES) {
            const int c = cb + l;
            if (l < INVIT_LANES && c < nc) {
                double *u1 = lu + l * INVIT_STRIDE, *u2 = u1 + 64, *ml = u2 + 64, *yl = ml + 64;
                const int i0 = scl[c], i1 = scl[c + 1];
                for (int mi = i0; mi < i1; ++mi) {
                    // perturb equal eigenvalues inside a cluster so the solves differ
                    const double lam = ev[mi] + (double)(mi - i0) * 4.0 * u * tn;
                    // (t was formed with every lane active: the lane reads below see all rows)
                    const double td = t.d, te = t.e;
                    int n = opaque_uniform(n_in);   // keeps the bound tests of the unrolled loops in place
                    // factor P (T - lambda I) = L U: per row the reciprocal pivot u1, the
                    // first super-diagonal divided by minus the pivot (b, in u2) and the
                    // multiplier ml; the row interchanges go to a bit mask.  A zero
                    // coupling is floored at u tn + 1e-300 as the pivot candidate, so that no
                    // pivot is zero (a perturbation at the rounding level of T).
                    const double tiny = u * tn + 1e-300;
                    unsigned long long swb = 0;
                    double r0 = readlane_f64(td, 0) - lam, r1 = readlane_f64(te, 0);
#pragma unroll
                    for (int i = 0; i < 63; ++i) {
                        if (i + 1 >= n) break;
                        if ((i & 7) == 0) __builtin_amdgcn_sched_barrier(0);
                        const double ei = readlane_f64(te, i);
                        const double s0 = (ei != 0.0) ? ei : tiny;
                        const double s1 = readlane_f64(td, i + 1) - lam;
                        const double s2 = readlane_f64(te, i + 1);
                        const bool sw = !(fabs(r0) >= fabs(s0));
                        const double p0 = sw ? s0 : r0;
                        const double p1 = sw ? s1 : r1, p2 = sw ? s2 : 0.0;
                        const double o1 = sw ? r1 : s1, o2 = sw ? 0.0 : s2;
                        const double ip = rcp_nr1(p0);
                        const double mult = (sw ? r0 : s0) * ip;
                        u1[i] = ip;
                        u2[i] = -p1 * ip;
                        ml[i] = mult;
                        if (sw) swb |= 1ULL << i;
                        r0 = o1 - mult * p1;
                        r1 = o2 - mult * p2;
                    }
                    if (r0 == 0.0) r0 = tiny;
                    u1[n - 1] = rcp_nr1(r0);
                    u2[n - 1] = 0.0;
                    ml[n - 1] = 0.0;
                    // rows past the matrix: no multiplier (the forward sweep only carries
                    // the value along) and a zero row of U^-1 (the back substitution
                    // enters row n - 1 with x_n = x_{n+1} = 0)
                    for (int i = n; i < 64; ++i) {
                        u1[i] = 0.0;
                        u2[i] = 0.0;
                        ml[i] = 0.0;
                    }
                    // start vector: fixed, not orthogonal to any eigenvector in practice
#pragma unroll
                    for (int i = 0; i < 72; ++i)
                        yl[i] = (i < n) ? 1.0 + 0.5 * __builtin_amdgcn_fract((double)(i + 3 * mi) * 0.6180339887498949) : 0.0;
                    const int nb = (n + 7) >> 3;   // blocks of 8 rows
                    double f = 1.0;                // scale of the iterate still to apply
#pragma unroll 1
                    for (int itn = 0; itn < 2; ++itn) {
                        // forward: row interchanges and multipliers, written so that only
                        // cur' = A cur + C nx waits on the previous row (no swap: A = -ml,
                        // C = 1; swap: A = 1, C = -ml); the scale f is applied on the way
                        double cur = f * yl[0];
                        for (int bb = 0; bb < nb; ++bb) {
                            const double *yb = yl + 8 * bb;
                            const double *mb = ml + 8 * bb;
                            const unsigned sb = (unsigned)(swb >> (8 * bb));
                            double nx[8], mv[8];
#pragma unroll
                            for (int q = 0; q < 8; ++q) {
                                nx[q] = f * yb[q + 1];
                                mv[q] = mb[q];
                            }
#pragma unroll
                            for (int q = 0; q < 8; ++q) {
                                const bool sw = (sb >> q) & 1u;
                                const double A = sw ? 1.0 : -mv[q], C = sw ? -mv[q] : 1.0;
                                yl[8 * bb + q] = sw ? nx[q] : cur;
                                cur = fma(A, cur, C * nx[q]);
                            }
                        }
                        // back substitution: x_i = u1_i y_i + b_i x_{i+1} + c_i x_{i+2}
                        // (c_i = -U(i, i+2) / U(i, i), nonzero only after an interchange);
                        // the sum of squares and the largest magnitude come along
                        double x1 = 0.0, x2 = 0.0, ss = 0.0, mx = 0.0;
                        for (int bb = nb - 1; bb >= 0; --bb) {
                            double *yb = yl + 8 * bb;
                            const double *ab = u1 + 8 * bb, *bb2 = u2 + 8 * bb;
                            const unsigned sb = (unsigned)(swb >> (8 * bb));
                            double yv[8], a1[8], a2[8];
#pragma unroll
                            for (int q = 0; q < 8; ++q) {
                                yv[q] = yb[q];
                                a1[q] = ab[q];
                                a2[q] = bb2[q];
                            }
#pragma unroll
                            for (int q = 7; q >= 0; --q) {
                                const int i2 = min(8 * bb + q + 1, 63);
                                const double e3 = ((sb >> q) & 1u) ? readlane_f64(te, i2) : 0.0;
                                const double sv = fma(a2[q], x1, fma(-e3 * a1[q], x2, yv[q] * a1[q]));
                                yb[q] = sv;
                                ss = fma(sv, sv, ss);
                                mx = fmax(mx, fabs(sv));
                                x2 = x1;
                                x1 = sv;
                            }
                        }
                        // re-orthogonalise inside the cluster
                        for (int pj = i0; pj < mi; ++pj) {
                            const double *z = Y + pj * n;
                            double dt = 0.0;
                            for (int i = 0; i < n; ++i) dt += z[i] * yl[i];
                            ss = 0.0;
                            mx = 0.0;
                            for (int i = 0; i < n; ++i) {
                                const double v = yl[i] - dt * z[i];
                                yl[i] = v;
                                ss += v * v;
                                mx = fmax(mx, fabs(v));
                            }
                        }
                        // normalise (through the largest magnitude when the plain sum of
                        // squares left the normal range); the scale goes into the next
                        // forward sweep, or into the column after the last solve
                        if (ss > 1e-290 && ss < 1e290) {
                            f = 1.0 / sqrt(ss);
                        } else {
                            const double sm = (mx > 0.0) ? 1.0 / mx : 1.0;
                            double q2 = 0.0;
                            for (int i = 0; i < n; ++i) {
                                const double v = yl[i] * sm;
                                q2 += v * v;
                            }
                            f = sm / sqrt(q2);
                        }
                    }
                    for (int i = 0; i < n; ++i) Y[mi * n + i] = yl[i] * f;
                }
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// C = A B for 64 x 64 operands on the FP64 MFMA: the 16 output tiles of
// 16 x 16 go two to each wave.  fa(i, k) and fb(k, j) return the operands
// (zero outside the matrices); fc(i, j, v) stores one result.  All loads of
// a tile are issued before its 16 MFMAs.
// ---------------------------------------------------------------------------
template <typename FA, typename FB, typename FC>
__device__ __forceinline__ void rl_mm64(FA fa, FB fb, FC fc)
{
    const int w = rl_wave(), l = rl_lane();
    const int li = l & 15, lk = l >> 4;
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        const int tile = 2 * w + tt, ti = tile >> 2, tj = tile & 3;
        double av[16], bv[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            av[s] = fa(ti * 16 + li, 4 * s + lk);
            bv[s] = fb(4 * s + lk, tj * 16 + li);
        }
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 16; ++s) acc = mfma16x16x4(av[s], bv[s], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) fc(ti * 16 + lk + 4 * v, tj * 16 + li, acc[v]);
    }
}

}  // namespace pod

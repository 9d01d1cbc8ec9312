// pod_small.hip -- FP64 small-matrix algebra of the merge (Alg. 2) on gfx950.
//
// One workgroup of 512 threads works on the p x p matrices of a merge: the
// Cholesky factors of the CholeskyQR2 Grams and their inverses, the SVD of
// the merge factor R (the paper's E up to an orthogonal factor) through the
// symmetric eigen-decomposition of R R^T, the rank guard, the convergence
// angles of Alg. 1 and the Rayleigh-Ritz step of the final projection.  These
// kernels are latency bound.  For p <= 64 the matrices live in registers and
// LDS (pod_rl.h); for wider merges the merge kernels keep them in the device
// workspace between stages and in registers / LDS within a stage
// (pod_big.h), and the other kernels use pod_symeig.h.
#include "pod_internal.h"
#include "pod_symeig.h"
#include "pod_rl.h"
#include "pod_big.h"

namespace pod {

constexpr int NT = EIG_NT;
// Matrices up to SMALL_LDS_P x SMALL_LDS_P live in LDS; larger ones in the
// workspace `ws` (device memory, L2 resident).
// Dynamic LDS of the register-resident kernels (p <= 64, pmax = pm)
constexpr size_t chol_first_lds_rl(int pm) { return (size_t)(2 * 64 * RL_LD + 2 * pm * pm) * sizeof(double); }
constexpr size_t svd_merge_lds_rl(int) { return (size_t)(3 * 64 * RL_LD + 512 + INVIT_LDS) * sizeof(double); }
constexpr size_t lds_limit(bool big)
{
    return big ? (size_t)(BIG_PACKED + EIG_NMAX) * sizeof(double)
               : (size_t)(3 * SMALL_LDS_P * SMALL_LDS_P + eig_lu_doubles(SMALL_LDS_P)) * sizeof(double);
}
static_assert(chol_first_lds_rl(SMALL_LDS_P) <= lds_limit(false), "LDS budget");
static_assert(EIG_NMAX * 64 <= BIG_PACKED, "the wide merge's iterate scratch fits its dynamic LDS");

// ---------------------------------------------------------------------------
// In-place Cholesky S = R^T R of the symmetric p x p matrix S (column-major,
// ld p); on success the upper triangle holds R and the strict lower triangle
// is zeroed.  Fails (returns 1, uniformly across the block) when a pivot is
// not above `thr`.  Blocked right-looking form with panels of 16: the
// diagonal block is factored by wave 0 with its columns in registers (lane c
// holds column c; rows move between lanes by readlane), the panel rows right
// of it are solved one column per thread, and the trailing matrix takes one
// rank-16 update -- three barriers per panel.
// ---------------------------------------------------------------------------
__device__ int chol_upper(double *S, int p, double thr)
{
    __shared__ int sfail;
    __shared__ double srow[16], sinv[16], sW[16 * 16];
    const int t = threadIdx.x;
    if (t == 0) sfail = 0;
    __syncthreads();
    for (int J = 0; J < p; J += 16) {
        const int nb = (p - J < 16) ? p - J : 16;
        const int c0 = J + nb, q = p - c0;
        if (t < 64) {
            // diagonal block: lane c holds column J + c (rows J..J+15) in registers;
            // row k is broadcast through srow after its scaling.  Lanes left of
            // column k hold zeros there and lanes at or below the diagonal only
            // touch entries that are never stored, so no lane is masked.
            double col[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) col[i] = (t < nb && i <= t) ? S[(J + i) + (J + t) * p] : 0.0;
            int fail = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (k < nb) {
                    const double d = readlane_f64(col[k], k);
                    if (!(d > thr)) fail = 1;
                    const double ik = rsqrt_nr(fmax(d, 1e-300));
                    col[k] *= ik;   // lane k: sqrt(d); lanes right of it: row k of R
                    if (t < 16) srow[t] = col[k];
                    if (t == k) sinv[k] = ik;
#pragma unroll
                    for (int i = k + 1; i < 16; ++i) col[i] -= srow[i] * col[k];
                }
            }
            if (t == 0 && fail) sfail = 1;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (t < nb && i <= t) S[(J + i) + (J + t) * p] = col[i];
            // W = R_JJ^-1 (upper, 16 x 16): lane j < nb solves column j by back
            // substitution (fully unrolled: the loads of R are issued together);
            // W is kept in sW (ld 16)
            if (q > 0) {
                const double *Rb = S + J + J * p;
                double w[16];
#pragma unroll
                for (int i = 15; i >= 0; --i) {
                    double v = (i == t) ? 1.0 : 0.0;
#pragma unroll
                    for (int l = i + 1; l < 16; ++l)
                        if (l < nb) v -= Rb[i + l * p] * w[l];
                    w[i] = (i < nb && i <= t) ? v * sinv[i] : 0.0;
                    __builtin_amdgcn_sched_barrier(0);   // keep the loads of one row together
                }
                if (t < 16) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) sW[i + t * 16] = w[i];
                }
            }
        }
        __syncthreads();
        if (sfail) return 1;
        if (q > 0) {
            // rows J..J+nb of the columns right of the block: X = W^T S(J:J+nb, c0:p),
            // one thread per column (the column is read whole before rows are written)
            for (int c = c0 + t; c < p; c += NT) {
                double *bc = S + J + c * p;
                double b[16];
#pragma unroll
                for (int k2 = 0; k2 < 16; ++k2) b[k2] = (k2 < nb) ? bc[k2] : 0.0;
#pragma unroll
                for (int i = 15; i >= 0; --i) {
                    if (i < nb) {
                        double v = 0.0;
#pragma unroll
                        for (int k2 = 0; k2 <= i; ++k2) v += sW[k2 + i * 16] * b[k2];
                        bc[i] = v;
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            __syncthreads();
            // trailing update of the upper triangle: S(i, c) -= sum_k R(k, i) R(k, c)
            const int tx = t & 31, ty = t >> 5;
            for (int c = c0 + ty; c < p; c += NT / 32) {
                const double *rc = S + J + c * p;
                for (int i = c0 + tx; i <= c; i += 32) {
                    const double *ri = S + J + i * p;
                    double a0 = 0.0, a1 = 0.0;
#pragma unroll
                    for (int k2 = 0; k2 < 16; k2 += 2) {
                        if (k2 < nb) a0 += ri[k2] * rc[k2];
                        if (k2 + 1 < nb) a1 += ri[k2 + 1] * rc[k2 + 1];
                    }
                    S[i + c * p] -= a0 + a1;
                }
            }
            __syncthreads();
        }
    }
    for (int idx = t; idx < p * p; idx += NT) {
        const int i = idx % p, k = idx / p;
        if (i > k) S[idx] = 0.0;
    }
    __syncthreads();
    return 0;
}

// X = R^-1 for the upper-triangular p x p matrix R (column-major, ld p); X
// must not alias R.  Column j of X solves R x = e_j by back substitution in
// one group of 8 lanes: lane gl keeps the right-hand side of rows gl, gl+8,
// ... in registers; step i broadcasts b_i from its lane inside the group, sets
// x_i = b_i / R_ii and updates the rows above.  No barrier between the steps;
// `tmp` (p doubles) holds the reciprocals of the diagonal.  SL = ceil(p/8)
// register slots.
template <int SL> __device__ void trinv_cols(const double *R, int p, double *X, double *tmp)
{
    for (int i = threadIdx.x; i < p; i += NT) tmp[i] = 1.0 / R[i + i * p];
    __syncthreads();
    const int gl = threadIdx.x & 7;
    for (int j = threadIdx.x >> 3; j < p; j += NT / 8) {
        double b[SL];
#pragma unroll
        for (int s = 0; s < SL; ++s) b[s] = (8 * s + gl == j) ? 1.0 : 0.0;
#pragma unroll
        for (int s = SL - 1; s >= 0; --s) {
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
                if (gl == o) X[i + j * p] = xi;
                // rows of this slot below lane o, then the earlier slots
                if (gl < o) bs -= R[(8 * s + gl) + i * p] * xi;
#pragma unroll
                for (int s2 = 0; s2 < s; ++s2) b[s2] -= R[(8 * s2 + gl) + i * p] * xi;
            }
        }
        for (int l = j + 1 + gl; l < p; l += 8) X[l + j * p] = 0.0;
    }
    __syncthreads();
}

// p <= 64 (BIG = false) or p <= 160 (BIG = true)
template <bool BIG> __device__ __forceinline__ void trinv_upper(const double *R, int p, double *X, double *tmp)
{
    trinv_cols<BIG ? 20 : 8>(R, p, X, tmp);
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
// basis block enters the merge weighted by its singular values, Alg. 2; a
// merged external basis by its own, Alg. 3; a row-sampled block by its right
// factor, P = blkdiag(Sigma_r, Vt)),
// R1 = chol(G1) (shifted by s = p u tr(G1) if a pivot breaks down),
// T1 = P R1^-1 written in the compute type for the tall GEMM Y = X0 T1.
// ---------------------------------------------------------------------------
// Register-resident form for p <= 64 (pod_rl.h): the factor and its inverse
// come out of one elimination pass.
__device__ __forceinline__ void chol_first_rl(const SmallArgs &a)
{
    extern __shared__ double lds[];
    __shared__ double sP[SMALL_LDS_P], sred[8];
    __shared__ int sfl[8], sbadw[8];
    DevState *ds = a.ds;
    if (merge_halted(ds)) return;
    const int p = ds->p, rs = ds->rs, p0 = ds->p0;
    const int pm = a.pmax;
    const int w = rl_wave(), l = rl_lane();
    double *Rs = lds;                   // R1 (row-major)
    double *Xs = Rs + 64 * RL_LD;       // R1^-T (row-major)
    double *S = Xs + 64 * RL_LD;        // G1 (p x p, ld p) with a dense right factor
    double *GP = S + pm * pm;           // G0 P (p0 x p)
    const double *sigma = (ds->it & 1) ? a.sig1 : a.sig0;
    for (int i = threadIdx.x; i < p; i += NT) sP[i] = (i < rs) ? sigma[i] : (a.sigma2 ? a.sigma2[i - rs] : 1.0);
    __syncthreads();
    double g[8];
    if (a.use_vt) {
        for (int idx = threadIdx.x; idx < p0 * p; idx += NT) {
            const int i = idx % p0, b = idx / p0;
            double v;
            if (b < rs) {
                v = a.G[i + b * pm] * sP[b];
            } else {
                v = 0.0;
                for (int q = 0; q < p0 - rs; ++q) v += a.G[i + (rs + q) * pm] * a.Vt[q + (b - rs) * pm];
            }
            GP[i + b * p0] = v;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < p * p; idx += NT) {
            const int i = idx % p, j = idx / p;
            double v;
            if (i < rs) {
                v = sP[i] * GP[i + j * p0];
            } else {
                v = 0.0;
                for (int q = 0; q < p0 - rs; ++q) v += a.Vt[q + (i - rs) * pm] * GP[(rs + q) + j * p0];
            }
            S[idx] = v;
        }
        __syncthreads();
        // row a, columns >= a: the upper triangle S(a, l), as the factorisation reads it
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int ar = rl_chol_row(w, k);
            g[k] = (ar < p && l < p) ? S[ar + l * p] : 0.0;
        }
    } else {
        // G0 is stored exactly symmetric: row a of G1 is read along column a
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int ar = rl_chol_row(w, k);
            g[k] = (ar < p && l < p) ? a.G[l + ar * pm] * sP[ar] * sP[l] : 0.0;
        }
    }
    int bad = 0;
    double td = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (!isfinite(g[k])) bad = 1;
        if (l == rl_chol_row(w, k)) td += g[k];
    }
    td = wave_sum(td);
    bad = __any(bad);
    if (l == 0) {
        sred[w] = td;
        sbadw[w] = bad;
    }
    __syncthreads();
    double trace = 0.0;
    bad = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        trace += sred[q];
        bad |= sbadw[q];
    }
    double r[8];
    if (bad) {
        if (threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)FLAG_NONFINITE);
        rl_identity(p, Rs, Xs);
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) r[k] = g[k];
        int fail = rl_cholinv(r, p, a.urnd * trace * 1e-3, Rs, Xs, sfl);
        if (fail) {
            const double shift = (double)p * a.urnd * trace;
            if (threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)FLAG_SHIFT);
#pragma unroll
            for (int k = 0; k < 8; ++k) r[k] = g[k] + ((l == rl_chol_row(w, k) && l < p) ? shift : 0.0);
            fail = rl_cholinv(r, p, 0.0, Rs, Xs, sfl);
            if (fail) {
                if (threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)FLAG_NOTPD);
                rl_identity(p, Rs, Xs);
            }
        }
    }
    // R1 (column-major, ld pm, zero-padded) and T1 = P R1^-1 in the compute type
    for (int idx = threadIdx.x; idx < pm * pm; idx += NT) {
        const int i = idx % pm, j = idx / pm;
        a.R1[idx] = (i < p && j < p) ? Rs[i * RL_LD + j] : 0.0;
        double v = 0.0;
        if (!a.use_vt) {
            if (i < p && j < p) v = sP[i] * Xs[j * RL_LD + i];
        } else if (i < p0 && j < p) {
            if (i < rs) {
                v = sP[i] * Xs[j * RL_LD + i];
            } else {
                for (int q = rs; q <= j; ++q) v += a.Vt[(i - rs) + (q - rs) * pm] * Xs[j * RL_LD + q];
            }
        }
        store_c(a.Tc, a.prec, idx, v);
    }
}

template <bool BIG>
__device__ __forceinline__ void chol_first_body(const SmallArgs &a)
{
    if constexpr (!BIG) {
        chol_first_rl(a);
    } else {
    extern __shared__ double lds[];
    __shared__ double sP[EIG_NMAX];
    __shared__ double sred[16];
    DevState *ds = a.ds;
    if (merge_halted(ds)) return;
    const int p = ds->p, rs = ds->rs, p0 = ds->p0;
    const int pm = a.pmax;
    double *S = a.ws;                   // G1 (p x p) when the right factor is dense
    double *GP = S + pm * pm + pm;      // G0 P (p0 x p) with a dense right factor; then R1^-1
    double *Rp = lds, *rdiag = lds + BIG_PACKED;   // R1 packed by columns, 1 / diag(R1)
    const double *sigma = (ds->it & 1) ? a.sig1 : a.sig0;
    for (int i = threadIdx.x; i < p; i += NT) sP[i] = (i < rs) ? sigma[i] : (a.sigma2 ? a.sigma2[i - rs] : 1.0);
    __syncthreads();
    if (a.use_vt) {
        // P = blkdiag(Sigma_r, Vt): GP = G0 P, then G1 = P^T GP into S
        for (int idx = threadIdx.x; idx < p0 * p; idx += NT) {
            const int i = idx % p0, b = idx / p0;
            double v;
            if (b < rs) {
                v = a.G[i + b * pm] * sP[b];
            } else {
                v = 0.0;
                for (int l = 0; l < p0 - rs; ++l) v += a.G[i + (rs + l) * pm] * a.Vt[l + (b - rs) * pm];
            }
            GP[i + b * p0] = v;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < p * p; idx += NT) {
            const int i = idx % p, j = idx / p;
            double v;
            if (i < rs) {
                v = sP[i] * GP[i + j * p0];
            } else {
                v = 0.0;
                for (int l = 0; l < p0 - rs; ++l) v += a.Vt[l + (i - rs) * pm] * GP[(rs + l) + j * p0];
            }
            S[idx] = v;
        }
        __syncthreads();
    }
    // G1 = P^T G0 P, read where the Cholesky needs it
    // (two forms, chosen outside the factorisation, so that its loads are
    // straight-line code and stay in flight together)
    auto g1d = [&](int i, int j) -> double { return a.G[i + j * pm] * (sP[i] * sP[j]); };
    auto g1v = [&](int i, int j) -> double { return S[i + j * p]; };
    auto g1 = [&](int i, int j) -> double { return a.use_vt ? g1v(i, j) : g1d(i, j); };
    double tr = (threadIdx.x < p) ? g1(threadIdx.x, threadIdx.x) : 0.0;
    tr = wave_sum(tr);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = tr;
    __syncthreads();
    double trace = 0.0;
    for (int q = 0; q < NT / 64; ++q) trace += sred[q];
    // R1 into Rp; a failed pivot is retried once with the diagonal shifted by
    // p u tr(G1)
    int fail = isfinite(trace) ? 0 : 2;
    for (int attempt = 0; attempt < 2 && fail != 2; ++attempt) {
        const double shift = attempt ? (double)p * a.urnd * trace : 0.0;
        const double thr = attempt ? 0.0 : a.urnd * trace * 1e-3;
        auto st = [&](int r, int c, double v) {
            Rp[c * (c + 1) / 2 + r] = v;
            if (r == c) rdiag[c] = 1.0 / v;
        };
        if (a.use_vt)
            fail = big_chol(p, thr, [&](int i, int j) { return g1v(i, j) + ((i == j) ? shift : 0.0); }, st);
        else
            fail = big_chol(p, thr, [&](int i, int j) { return g1d(i, j) + ((i == j) ? shift : 0.0); }, st);
        if (fail != 1) break;
        if (attempt == 0 && threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)FLAG_SHIFT);
    }
    if (fail) {
        if (threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)((fail & 2) ? FLAG_NONFINITE : FLAG_NOTPD));
        for (int q = threadIdx.x; q < p * (p + 1) / 2; q += NT) {
            const int c = packed_col(q);
            Rp[q] = (q - c * (c + 1) / 2 == c) ? 1.0 : 0.0;
        }
        for (int i = threadIdx.x; i < p; i += NT) rdiag[i] = 1.0;
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < pm * pm; idx += NT) {
        const int i = idx % pm, j = idx / pm;
        a.R1[idx] = (i <= j && j < p) ? Rp[j * (j + 1) / 2 + i] : 0.0;
    }
    // T1 = P R1^-1 (p0 x p, zero-padded to pmax x pmax); without a right
    // factor P is diagonal and k_wide_trsm<0> forms T1 on the matrix cores
    // from R1 and the inverses of its diagonal blocks
    if (!a.use_vt) {
        diag_inv16(p, [&](int i, int k) { return Rp[k * (k + 1) / 2 + i]; }, a.ws + big_dinv_offset(pm));
    } else {
        double *Xi = GP;   // R1^-1 (the G0 P product is no longer needed)
        big_trinv_solve(Rp, rdiag, p, [&](int i, int j, double x) { Xi[i + j * p] = x; });
        for (int idx = threadIdx.x; idx < pm * pm; idx += NT) {
            const int i = idx % pm, j = idx / pm;
            double v = 0.0;
            if (i < p0 && j < p) {
                if (i < rs) {
                    v = sP[i] * Xi[i + j * p];
                } else {
                    for (int l = rs; l <= j; ++l) v += a.Vt[(i - rs) + (l - rs) * pm] * Xi[l + j * p];
                }
            }
            store_c(a.Tc, a.prec, idx, v);
        }
    }
    }
}

template <bool BIG>
__global__ __launch_bounds__(512) void k_chol_first(SmallArgs a)
{
    chol_first_body<BIG>(a);
}

// ---------------------------------------------------------------------------
// Triangular solves of a wide merge on the matrix cores, X = R^-1 B for the
// upper-triangular p x p factor R (M = 0: R1 (a.R1, ld pmax), B = I, into Tc
// as T1 = diag(sP) X, zero outside p x p; M = 1: R2 (S1, ld p), B = U_R (S3,
// p x r'), into the leading p x r' block of Tc as Z2).  Blocked back
// substitution over 16 x 16 tiles: wave w of workgroup b owns the column
// tile J = 4 b + w of X and, for the row tiles I from the last up,
//   X(I, J) = D_I (B(I, J) - sum_{K > I} R(I, K) X(K, J)),
// D_I the inverse of the diagonal block (BIG_DINV_DOUBLES at
// big_dinv_offset, written by the Cholesky kernel), each product a chain of
// v_mfma_f64_16x16x4.  The solved tiles stay in registers: the FP64
// accumulator layout (rows l / 16 + 4 v) is the layout of the B operand's
// four k-chunks.  R's upper tiles and the D_I are staged in LDS in the
// A-operand layout (tile (I, K) at (K (K + 1) / 2 + I) 256, chunk s, lane).
// ---------------------------------------------------------------------------
constexpr int TRSM_NT = EIG_NMAX / 16;                          // row tiles of the widest merge
constexpr int TRSM_TILES = TRSM_NT * (TRSM_NT + 1) / 2;
constexpr size_t TRSM_LDS = (size_t)(TRSM_TILES + TRSM_NT) * 256 * sizeof(double);
constexpr int TRSM_BATCH = 32;                                   // staging loads in flight per thread

// (NTH threads: NTH / 64 column tiles per workgroup; blk the workgroup's
// index among those doing this solve; sP: LDS for the column weights, M = 0)
template <int M, int NTH>
__device__ __forceinline__ void wide_trsm_body(const SmallArgs &a, int blk, double *lds, double *sP)
{
    const DevState *ds = a.ds;
    const int p = ds->p, pm = a.pmax;
    const int ncol = (M == 0) ? p : ds->rnew;
    const int nt = (p + 15) >> 4;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int J = (NTH / 64) * blk + w;
    const double *Rm = (M == 0) ? a.R1 : a.ws;
    const int ldr = (M == 0) ? pm : p;
    const double *dinv = a.ws + big_dinv_offset(pm);
    // (Ts: the upper tiles of the first nt tile columns, packed; Ds right after them)
    if (M == 0) {
        const int rs = ds->rs;
        const double *sigma = (ds->it & 1) ? a.sig1 : a.sig0;
        for (int i = threadIdx.x; i < p; i += NTH) sP[i] = (i < rs) ? sigma[i] : (a.sigma2 ? a.sigma2[i - rs] : 1.0);
    }
    // stage R's upper tiles, then the D_I: thread e takes entry e of every
    // (NTH / 256)-th tile from its first, TRSM_BATCH tiles (loads in flight)
    // at a time
    constexpr int TS = NTH / 256;   // tiles per pass
    const int ntri = nt * (nt + 1) / 2;
    const int e = threadIdx.x & 255, toff = threadIdx.x >> 8;
    const int erow = e & 15, ecol = 4 * (e >> 6) + ((e >> 4) & 3);   // (m, k) of entry e in the operand layout
    int tI = 0, tK = 0;                                               // tile (I, K) of t = t0 + toff
    for (int q = 0; q < toff; ++q)
        if (++tI > tK) {
            ++tK;
            tI = 0;
        }
    for (int t0 = 0; t0 < ntri + nt; t0 += TS * TRSM_BATCH) {
        double v[TRSM_BATCH];
        int I = tI, K = tK;
#pragma unroll
        for (int u = 0; u < TRSM_BATCH; ++u) {
            const int t = t0 + TS * u + toff;
            // (no branch around the load: a load inside a divergent branch is
            // waited for there, and the batch would not be in flight together)
            const int row = 16 * I + erow, col = 16 * K + ecol;
            const bool tri = t < ntri, dg = !tri && t < ntri + nt;
            const bool ok = tri && row < p && col < p && row <= col;
            const double *src = tri ? Rm : dinv;
            const size_t off = ok ? row + (size_t)col * ldr : (dg ? (size_t)256 * (t - ntri) + e : 0);
            const double ld = src[off];
            const double x = (ok || dg) ? ld : 0.0;
#pragma unroll
            for (int q = 0; q < TS; ++q)
                if (++I > K) {
                    ++K;
                    I = 0;
                }
            v[u] = x;
        }
        tI = I;
        tK = K;
#pragma unroll
        for (int u = 0; u < TRSM_BATCH; ++u) {
            const int t = t0 + TS * u + toff;
            if (t < ntri + nt) lds[256 * t + e] = v[u];
        }
    }
    __syncthreads();
    if (16 * J >= pm) return;
    const int jc = 16 * J + (l & 15);   // this lane's column of X
    double X[TRSM_NT][4];
#pragma unroll
    for (int I = 0; I < TRSM_NT; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * I + (l >> 4) + 4 * v;
            if (M == 0)
                X[I][v] = (row == jc && row < p) ? 1.0 : 0.0;
            else
                X[I][v] = (row < p && jc < ncol) ? a.ws[2 * (size_t)p * p + row + (size_t)jc * p] : 0.0;
        }
    if (16 * J < ncol) {
#pragma unroll
        for (int I = TRSM_NT - 1; I >= 0; --I) {
            if (I >= nt || (M == 0 && I > J)) continue;
            v4d acc = {X[I][0], X[I][1], X[I][2], X[I][3]};
#pragma unroll
            for (int K = I + 1; K < TRSM_NT; ++K) {
                if (K >= nt || (M == 0 && K > J)) continue;
                const double *ta = lds + (K * (K + 1) / 2 + I) * 256 + l;
#pragma unroll
                for (int s = 0; s < 4; ++s) acc = mfma16x16x4(-ta[64 * s], X[K][s], acc);
            }
            v4d x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 4; ++s) x = mfma16x16x4(lds[256 * (ntri + I) + 64 * s + l], acc[s], x);
#pragma unroll
            for (int v = 0; v < 4; ++v) X[I][v] = x[v];
        }
    }
    // out: T1 over all of pmax x pmax (zero outside p x p and below the
    // diagonal tiles), Z2 on its leading p x r' block
#pragma unroll
    for (int I = 0; I < TRSM_NT; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * I + (l >> 4) + 4 * v;
            if (M == 0) {
                if (row < pm && jc < pm)
                    store_c(a.Tc, a.prec, row + (size_t)jc * pm,
                            (row < p && jc < p && I <= J) ? sP[row] * X[I][v] : 0.0);
            } else if (row < p && jc < ncol) {
                store_c(a.Tc, a.prec, row + (size_t)jc * pm, X[I][v]);
            }
        }
}

template <int M>
__global__ __launch_bounds__(256) void k_wide_trsm(SmallArgs a)
{
    extern __shared__ double lds[];
    __shared__ double sP[EIG_NMAX];
    if (merge_halted(a.ds)) return;
    wide_trsm_body<M, 256>(a, blockIdx.x, lds, sP);
}

// Batched: one workgroup per matrix (blockIdx.y), stopped matrices skipped.
__global__ __launch_bounds__(512) void k_chol_first_b(const SmallArgs *__restrict__ arr)
{
    const SmallArgs a = arr[blockIdx.y];
    if (a.ds->done) return;
    chol_first_body<false>(a);
}

hipError_t launch_chol_first(const SmallArgs &a, hipStream_t st)
{
    const bool big = a.pmax > SMALL_LDS_P;
    const size_t lds = big ? (size_t)(BIG_PACKED + EIG_NMAX) * sizeof(double) : chol_first_lds_rl(a.pmax);
    static bool attr[2] = {false, false};
    const void *fn = big ? (const void *)k_chol_first<true> : (const void *)k_chol_first<false>;
    if (!attr[big]) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_limit(big));
        if (e != hipSuccess) return e;
        attr[big] = true;
    }
    static bool attr_t1 = false;
    if (big && !a.use_vt && !attr_t1) {
        hipError_t e = hipFuncSetAttribute((const void *)k_wide_trsm<0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)TRSM_LDS);
        if (e != hipSuccess) return e;
        attr_t1 = true;
    }
    ProfScope ps(POD_K_CHOL, st);
    if (big) {
        hipLaunchKernelGGL(k_chol_first<true>, dim3(1), dim3(NT), lds, st, a);
        if (!a.use_vt)
            hipLaunchKernelGGL(k_wide_trsm<0>, dim3((unsigned)((a.pmax + 63) / 64)), dim3(256), TRSM_LDS, st, a);
    } else {
        hipLaunchKernelGGL(k_chol_first<false>, dim3(1), dim3(NT), lds, st, a);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CholeskyQR pass 2 and the small SVD of the merge:
//   R2 = chol(G2) (G2 = Y^T Y), R = R2 R1 (upper triangular: the paper's E up
//   to an orthogonal left factor), R R^T = U_R Lambda U_R^T by the symmetric
//   eigensolver, Sigma_R = sqrt(Lambda), rank guard
//   r' = min(r, #{lambda_i > max((p u)^2, p u_64) lambda_1}) (the sigma-domain
//   guard sigma_i > p u sigma_1, floored at the resolution of the FP64
//   eigenvalues), Z2 = R2^-1 U_R(:, 0:r') in the compute type for
//   U_new = Y Z2, Sigma_new = Sigma_R(0:r').
// Convergence (Alg. 1): the first k columns of M = [U Sigma | C] span the old
// modes, and M = Q R with R upper triangular, so in the basis Q the old
// subspace is span(e_1..e_k) and the new one span(U_R(:, 0:k)).  The sines of
// the principal angles are the singular values of B = U_R(k:p, 0:k); the
// largest is the square root of the largest eigenvalue of B^T B.  The mode
// criterion compares R(:, i)/|R(:, i)| with U_R(:, i) one by one.
// ---------------------------------------------------------------------------
// Register-resident form for p <= 64 (pod_rl.h).  LDS: bufA holds R2, then
// H = R R^T, then the eigenvectors Y; bufB holds R, then the reflectors of the
// tridiagonalisation, then B^T B and its reflectors; Xs holds R2^-T.
// The convergence sine of the merge: the largest sine of the principal angles
// between the leading kk directions before and after it, from the first kk
// columns of U_R (Y: p x >= kk, ld p, in LDS).  With U_R
// orthogonal, span(U_old) = span(e_0..e_kk-1) in the merge basis and the
// sines are the singular values of B = U_R(kk:p, 0:kk): sin^2 = lambda_max
// of B^T B.  POD_CRIT_MODE instead takes the largest residual of each new
// direction against the matching scaled column of R (a.work).  Every thread
// calls this; NaN for kk = 0.
__device__ __forceinline__ double merge_sin_rl(const SmallArgs &a, const double *Y, int p, int kk, double *bufB,
                                               double *Pp, double *sd, double *se, double *stau, double *ssde,
                                               double *ssin, double *sred)
{
    double sin_max = __builtin_nan("");
    if (kk > 0) {
        if (a.criterion == POD_CRIT_MODE) {
            double mx = 0.0;
            if (threadIdx.x < 64) {
                for (int i = 0; i < kk; ++i) {
                    double nr = 0.0, dt = 0.0;
                    for (int q = threadIdx.x; q < p; q += 64) {
                        const double x = a.work[q + i * p];
                        nr += x * x;
                        dt += x * Y[q + i * p];
                    }
                    nr = wave_sum(nr);
                    dt = wave_sum(dt);
                    const double inv = 1.0 / sqrt(nr);
                    double res = 0.0;
                    for (int q = threadIdx.x; q < p; q += 64) {
                        const double dd = Y[q + i * p] - a.work[q + i * p] * inv * (dt * inv);
                        res += dd * dd;
                    }
                    res = wave_sum(res);
                    mx = fmax(mx, sqrt(res));
                }
            }
            if (threadIdx.x == 0) sred[0] = mx;
            __syncthreads();
            sin_max = sred[0];
            __syncthreads();
        } else {
            const int br = p - kk;
            if (br <= 0) {
                sin_max = 0.0;
            } else {
                // F = B^T B (kk x kk), B = U_R(kk:p, 0:kk)
                rl_mm64([&](int i, int q) { return (i < kk && q < br) ? Y[kk + q + i * p] : 0.0; },
                        [&](int q, int j) { return (q < br && j < kk) ? Y[kk + q + j * p] : 0.0; },
                        [&](int i, int j, double v) { bufB[i * RL_LD + j] = v; });
                __syncthreads();
                double r[8];
                rl_load_rows(r, bufB);
                __syncthreads();
                rl_tridiag(r, kk, sd, se, stau, bufB, Pp);
                bisect_top_rl(tri_regs(sd, se, kk, ssde), kk, 1, ssin);
                sin_max = sqrt(fmax(ssin[0], 0.0));
            }
        }
    }
    return sin_max;
}

__device__ __forceinline__ void svd_merge_rl(const SmallArgs &a)
{
    extern __shared__ double lds[];
    __shared__ double sd[SMALL_LDS_P], se[SMALL_LDS_P], stau[SMALL_LDS_P], sev[SMALL_LDS_P], ssin[2], sred[8],
        ssde[TRI_SDE];
    __shared__ __align__(8) int scl[EIG_NMAX + 8];
    __shared__ int sfl[8];
    DevState *ds = a.ds;
    if (merge_halted(ds)) return;
    const int p = ds->p, rs = ds->rs;
    const int it0 = ds->it;   // read before thread 0 advances it at the end
    const int pm = a.pmax;
    const int w = rl_wave(), l = rl_lane();
    double *bufA = lds;
    double *bufB = bufA + 64 * RL_LD;
    double *Xs = bufB + 64 * RL_LD;
    double *Pp = Xs + 64 * RL_LD;    // 8 x 64
    double *lu = Pp + 512;           // INVIT_LDS
    // ---- pass-2 Cholesky R2 and R2^-T
    double g[8], r[8];
    rl_load_sym_chol(g, a.G, pm, p);
    const double trace = wave_sum((l < p) ? a.G[l + l * pm] : 0.0);
    int fail = 1;
    if (isfinite(trace)) {
#pragma unroll
        for (int k = 0; k < 8; ++k) r[k] = g[k];
        fail = rl_cholinv(r, p, a.urnd * trace * 1e-3, bufA, Xs, sfl);
    }
    if (fail) {
        const double shift = (double)p * a.urnd * (isfinite(trace) ? trace : 1.0);
        if (threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)FLAG_SHIFT);
        fail = 1;
        if (isfinite(trace)) {
#pragma unroll
            for (int k = 0; k < 8; ++k) r[k] = g[k] + ((l == rl_chol_row(w, k) && l < p) ? shift : 0.0);
            fail = rl_cholinv(r, p, 0.0, bufA, Xs, sfl);
        }
        if (fail) {
            if (threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)(isfinite(trace) ? FLAG_NOTPD : FLAG_NONFINITE));
            rl_identity(p, bufA, Xs);
        }
    }
    // ---- R = R2 R1 (both upper triangular) into bufB
    rl_mm64([&](int i, int k) { return bufA[i * RL_LD + k]; },
            [&](int k, int j) { return (k < p && j < p) ? a.R1[k + j * pm] : 0.0; },
            [&](int i, int j, double v) { bufB[i * RL_LD + j] = v; });
    __syncthreads();
    // the merge factor R, kept for the adjoint (ld pm, zero-padded)
    for (int idx = threadIdx.x; idx < pm * pm; idx += NT) {
        const int i = idx % pm, j = idx / pm;
        a.R2[idx] = (i < p && j < p) ? bufB[i * RL_LD + j] : 0.0;
    }
    const int kk0 = (a.k < rs) ? a.k : rs;
    if (a.criterion == POD_CRIT_MODE && kk0 > 0)
        for (int idx = threadIdx.x; idx < p * kk0; idx += NT) a.work[idx] = bufB[(idx % p) * RL_LD + idx / p];
    // ---- H = R R^T into bufA, then into registers
    rl_mm64([&](int i, int q) { return bufB[i * RL_LD + q]; },
            [&](int q, int j) { return bufB[j * RL_LD + q]; },
            [&](int i, int j, double v) { bufA[i * RL_LD + j] = v; });
    __syncthreads();
    rl_load_rows(r, bufA);
    __syncthreads();
    // ---- eigen-decomposition of H
    rl_tridiag(r, p, sd, se, stau, bufB, Pp);
    const int nv = (a.r < p) ? a.r : p;
    const TriRegs tt = tri_regs(sd, se, p, ssde);
    bisect_top_rl(tt, p, nv, sev);
    const double u64 = 1.1102230246251565e-16;
    const double g1 = (double)p * a.urnd;
    const double thr = fmax(g1 * g1, (double)p * u64) * fmax(sev[0], 0.0);
    const int nz = count_above_rl(tt, p, thr);
    const int rnew = (sev[0] > 0.0) ? ((nv < nz) ? nv : nz) : 0;
    double *Y = bufA;
    tri_invit_rl(tt, p, sev, rnew, Y, lu, scl);
    rl_backtransform(bufB, stau, p, Y, rnew);
    // Y now holds U_R(:, 0:rnew) (p x rnew, ld p)
    // ---- convergence angle
    const int kk = (kk0 < rnew) ? kk0 : rnew;
    const double sin_max = merge_sin_rl(a, Y, p, kk, bufB, Pp, sd, se, stau, ssde, ssin, sred);
    // ---- Z2 = R2^-1 U_R(:, 0:rnew) in the compute type: Z2^T(c, i) = sum_m Y(m, c) R2^-T(m, i)
    rl_mm64([&](int c, int q) { return (c < rnew && q < p) ? Y[q + c * p] : 0.0; },
            [&](int q, int i) { return Xs[q * RL_LD + i]; },
            [&](int c, int i, double v) {
                if (c < pm && i < pm) store_c(a.Tc, a.prec, i + c * pm, v);
            });
    // ---- Sigma_new(i) = |U_R(:, i)^T R| (the rows of U_R^T R = Sigma_R V_R^T):
    // accurate to about p u sigma_1 where sqrt(lambda_i) loses p u sigma_1^2 / sigma_i
    __syncthreads();
    rl_mm64([&](int i, int q) { return (i < rnew && q < p) ? Y[q + i * p] : 0.0; },
            [&](int q, int j) { return (q < p && j < p) ? a.R2[q + j * pm] : 0.0; },
            [&](int i, int j, double v) { bufB[i * RL_LD + j] = v; });
    __syncthreads();
    double *sigma_new = (it0 & 1) ? a.sig0 : a.sig1;
    for (int i = threadIdx.x; i < a.r; i += NT) {
        double v = 0.0;
        if (i < rnew)
            for (int j = 0; j < p; ++j) v = fma(bufB[i * RL_LD + j], bufB[i * RL_LD + j], v);
        sigma_new[i] = sqrt(v);
    }
    if (threadIdx.x == 0) {
        ds->rnew = rnew;
        ds->sin_theta = sin_max;
        ds->rs = rnew;
        ds->it = it0 + 1;
        ds->g = 0;
    }
}

// ---------------------------------------------------------------------------
// Wide merges (64 < p <= 160): the small stage of Alg. 2 as a chain of
// kernels over the workspace ws (S1 = R2, S2 = H, S3 = R then U_R, each
// p x p, ld p), so that the products and the triangular solves spread over
// many workgroups and only the inherently sequential factorisations
// (Cholesky, tridiagonalisation, eigenvectors) keep one workgroup:
//   k_wide_chol2   G2 = R2^T R2 (one workgroup)
//   k_wide_mm<0>   R = R2 R1 (one 16 x 16 tile per workgroup)
//   k_wide_mm<1>   H = R R^T
//   k_wide_eig     the top r' eigenpairs of H (U_R) (one workgroup); sets rnew
//   k_wide_tail    side by side: Z2 = R2^-1 U_R into Tc (blocked, on the
//                  matrix cores), Sigma_new(i) = |U_R(:, i)^T R| and the
//                  convergence sine (one workgroup each); then the merge
//                  count and rank advance
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_wide_chol2(SmallArgs a)
{
    __shared__ double sred[NT / 64];
    __shared__ double sdg[TRSM_NT * 256];   // the diagonal 16 x 16 blocks of R2 (column-major), for their inverses
    DevState *ds = a.ds;
    if (merge_halted(ds)) return;
    const int p = ds->p;
    const int pm = a.pmax;
    double *S1 = a.ws;
    // G2 = R2^T R2 into S1, read from G; a failed pivot is retried once with
    // the diagonal shifted by p u tr(G2)
    double tr = (threadIdx.x < p) ? a.G[threadIdx.x + threadIdx.x * pm] : 0.0;
    tr = wave_sum(tr);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = tr;
    __syncthreads();
    double trace = 0.0;
    for (int q = 0; q < NT / 64; ++q) trace += sred[q];
    int fail = isfinite(trace) ? 0 : 2;
    for (int attempt = 0; attempt < 2 && fail != 2; ++attempt) {
        const double shift = attempt ? (double)p * a.urnd * trace : 0.0;
        const double thr = attempt ? 0.0 : a.urnd * trace * 1e-3;
        fail = big_chol(
            p, thr, [&](int i, int j) { return a.G[i + j * pm] + ((i == j) ? shift : 0.0); },
            [&](int r, int c, double v) {
                S1[r + c * p] = v;
                if (c > r) S1[c + r * p] = 0.0;
                if ((r >> 4) == (c >> 4)) sdg[256 * (r >> 4) + 16 * (c & 15) + (r & 15)] = v;
            });
        if (fail != 1) break;
        if (attempt == 0 && threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)FLAG_SHIFT);
    }
    if (fail) {
        if (threadIdx.x == 0) atomicOr(&ds->flags, (int32_t)((fail & 2) ? FLAG_NONFINITE : FLAG_NOTPD));
        for (int idx = threadIdx.x; idx < p * p; idx += NT) S1[idx] = (idx % p == idx / p) ? 1.0 : 0.0;
        for (int idx = threadIdx.x; idx < TRSM_NT * 256; idx += NT)
            sdg[idx] = ((idx & 15) == ((idx >> 4) & 15)) ? 1.0 : 0.0;
    }
    __syncthreads();
    diag_inv16(p, [&](int i, int k) { return sdg[256 * (i >> 4) + 16 * (k & 15) + (i & 15)]; },
               a.ws + big_dinv_offset(pm));
}

// R = R2 R1 (M = 0; both upper triangular: tile (I, J) sums k in
// [16 I, 16 J + 16)), kept in R2 for the singular values and, for the mode
// criterion, its first min(k, r_s) columns in work; H = R R^T (M = 1: upper
// tiles, mirrored; tile (I, J) sums k from 16 max(I, J)).  Grid: the tiles
// of pmax x pmax; tiles outside p x p return at once.
template <int M>
__global__ __launch_bounds__(64) void k_wide_mm(SmallArgs a)
{
    const DevState *ds = a.ds;
    if (merge_halted(ds)) return;
    const int p = ds->p, rs = ds->rs, pm = a.pmax;
    const int nt = (p + 15) >> 4;
    const int ti = (int)blockIdx.x % TRSM_NT, tj = (int)blockIdx.x / TRSM_NT;
    if (ti >= nt || tj >= nt) return;
    double *S1 = a.ws, *S2 = S1 + p * p, *S3 = S1 + 2 * p * p;
    if (M == 0) {
        const int kk0 = (a.k < rs) ? a.k : rs;
        const bool keep = a.criterion == POD_CRIT_MODE;
        mm_tile_all<EIG_NMAX / 16>(
            ti, tj, 16 * ti, 16 * tj + 16, [&](int i, int k) { return (i < p && k < p) ? S1[i + k * p] : 0.0; },
            [&](int k, int j) { return (k < p && j < p) ? a.R1[k + j * pm] : 0.0; },
            [&](int i, int j, double v) {
                if (i < p && j < p) {
                    S3[i + j * p] = v;
                    a.R2[i + j * pm] = v;
                    if (keep && j < kk0) a.work[i + j * p] = v;
                }
            });
    } else {
        if (ti > tj) return;
        mm_tile_all<EIG_NMAX / 16>(
            ti, tj, 16 * ((ti > tj) ? ti : tj), 16 * nt,
            [&](int i, int k) { return (i < p && k < p) ? S3[i + k * p] : 0.0; },
            [&](int k, int j) { return (k < p && j < p) ? S3[j + k * p] : 0.0; },
            [&](int i, int j, double v) {
                if (i < p && j < p) {
                    S2[i + j * p] = v;
                    S2[j + i * p] = v;
                }
            });
    }
}

// The top r' = min(r, p, #{lambda_i > max((p u)^2, p u64) lambda_1})
// eigenpairs of H (S2): tridiagonalisation, multisection, inverse iteration,
// back-transformation into S3 (p x r').  Sets ds->rnew.
__global__ __launch_bounds__(512) void k_wide_eig(SmallArgs a)
{
    extern __shared__ double lds[];
    __shared__ double sd[EIG_NMAX], se[EIG_NMAX], stau[EIG_NMAX], sev[EIG_NMAX];
    __shared__ __align__(8) int scl[EIG_NMAX + 8];
    DevState *ds = a.ds;
    if (merge_halted(ds)) return;
    const int p = ds->p;
    const int pm = a.pmax;
    double *S2 = a.ws + p * p;       // H -> reflectors
    double *S3 = a.ws + 2 * p * p;   // eigenvectors U_R (p x r')
    big_tridiag(S2, p, sd, se, stau);
    const int nv = (a.r < p) ? a.r : p;
    const BigTri bt = big_tri(sd, se, p, lds);   // (the dynamic LDS is free until the convergence test)
    big_bisect_top(bt, p, nv, sev);
    const double u64 = 1.1102230246251565e-16;
    const double g1 = (double)p * a.urnd;
    const double thr = fmax(g1 * g1, (double)p * u64) * fmax(sev[0], 0.0);
    const int nz = p - big_sturm(bt, p, thr);
    const int rnew = (sev[0] > 0.0) ? ((nv < nz) ? nv : nz) : 0;
    big_invit(sd, se, p, sev, rnew, S3, a.ws + 3 * pm * pm + pm, lds, scl);
    big_backtransform(S2, stau, p, S3, rnew);
    // S3 now holds U_R(:, 0:rnew) (p x rnew, ld p); the convergence sines
    // follow in k_wide_tail
    if (threadIdx.x == 0) ds->rnew = rnew;
}

// Sigma_new(i) = |row i of W = U_R^T R| (i < r'; zero for r' <= i < r), R
// upper triangular in R2 (ld pmax): the tiles of W dealt to the 8 waves, each
// wave summing the squares of its tiles' rows into its own partials, the
// partials added in wave order.  Then the merge count and rank advance.
constexpr int SIG_NT = 512;
// (part: SIG_NT / 64 x EIG_NMAX doubles of LDS)
__device__ __forceinline__ void wide_sig_body(const SmallArgs &a, double *part)
{
    const DevState *ds = a.ds;
    const int p = ds->p, rnew = ds->rnew, it0 = ds->it, pm = a.pmax;
    const double *S3 = a.ws + 2 * p * p;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int idx = threadIdx.x; idx < (SIG_NT / 64) * EIG_NMAX; idx += SIG_NT) part[idx] = 0.0;
    __syncthreads();
    const int nti = (rnew + 15) >> 4, ntj = (p + 15) >> 4;
    for (int tile = w; tile < nti * ntj; tile += SIG_NT / 64) {
        const int ti = tile / ntj, tj = tile % ntj;
        mm_tile_all<EIG_NMAX / 16>(
            ti, tj, 0, 16 * tj + 16, [&](int i, int k) { return (i < rnew && k < p) ? S3[k + i * p] : 0.0; },
            [&](int k, int j) { return (k < p && j < p) ? a.R2[k + j * pm] : 0.0; },
            [&](int i, int j, double v) {
                // the 16 lanes of a row group hold the 16 columns of its rows
                const double sq = group_reduce<16, OpSum>(v * v);
                if ((l & 15) == 0 && i < EIG_NMAX) part[w * EIG_NMAX + i] += sq;
                (void)j;
            });
    }
    __syncthreads();
    double *sigma_new = (it0 & 1) ? a.sig0 : a.sig1;
    for (int i = threadIdx.x; i < a.r; i += SIG_NT) {
        double v = 0.0;
        if (i < rnew)
            for (int q = 0; q < SIG_NT / 64; ++q) v += part[q * EIG_NMAX + i];
        sigma_new[i] = sqrt(v);
    }
}

// The convergence sine of the merge (Sec. "Convergence", largest principal
// angle between the leading k modes before and after it) from U_R (S3) and,
// for the mode criterion, the first columns of R (work).  Every thread gets
// the value.  (lds: 64 RL_LD + 512 + TRI_SDE doubles of LDS)
__device__ __forceinline__ double wide_sines(const SmallArgs &a, double *lds)
{
    __shared__ double sd[EIG_NMAX], se[EIG_NMAX], stau[EIG_NMAX], se2[EIG_NMAX], spv[EIG_NMAX], ssc[8], ssin[2];
    __shared__ double sred[NT / 64];
    const DevState *ds = a.ds;
    const int p = ds->p, rs = ds->rs, rnew = ds->rnew;
    double *S2 = a.ws + p * p;       // free: B^T B for k > 64
    const double *S3 = a.ws + 2 * p * p;
    const int kk0 = (a.k < rs) ? a.k : rs;
    const int kk = (kk0 < rnew) ? kk0 : rnew;
    double sin_max = __builtin_nan("");
    if (kk > 0) {
        if (a.criterion == POD_CRIT_MODE) {
            double mx = 0.0;
            if (threadIdx.x < 64) {
                for (int i = 0; i < kk; ++i) {
                    double nr = 0.0, dt = 0.0;
                    for (int r = threadIdx.x; r < p; r += 64) {
                        const double x = a.work[r + i * p];
                        nr += x * x;
                        dt += x * S3[r + i * p];
                    }
                    nr = wave_sum(nr);
                    dt = wave_sum(dt);
                    const double inv = 1.0 / sqrt(nr);
                    double res = 0.0;
                    for (int r = threadIdx.x; r < p; r += 64) {
                        const double d = S3[r + i * p] - a.work[r + i * p] * inv * (dt * inv);
                        res += d * d;
                    }
                    res = wave_sum(res);
                    mx = fmax(mx, sqrt(res));
                }
            }
            if (threadIdx.x == 0) sred[0] = mx;
            __syncthreads();
            sin_max = sred[0];
            __syncthreads();
        } else {
            const int br = p - kk;
            if (br <= 0) {
                sin_max = 0.0;
            } else if (kk <= 64) {
                // F = B^T B (kk x kk), B = U_R(kk:p, 0:kk), on the matrix cores into a
                // zero-padded 64 x 64 LDS matrix; register-resident eigensolver
                double *bufB = lds, *Pp = lds + 64 * RL_LD, *ssde = Pp + 512;
                for (int idx = threadIdx.x; idx < 64 * RL_LD; idx += NT) bufB[idx] = 0.0;
                __syncthreads();
                big_mm(kk, false,
                       [&](int i, int q) { return (i < kk && q < br) ? S3[kk + q + i * p] : 0.0; },
                       [&](int q, int j) { return (q < br && j < kk) ? S3[kk + q + j * p] : 0.0; },
                       [&](int i, int j, double v) {
                           if (i < kk && j < kk) bufB[i * RL_LD + j] = v;
                       },
                       [&](int ti, int tj, int &k0, int &k1) { (void)ti; (void)tj; k0 = 0; k1 = (br + 15) & ~15; });
                __syncthreads();
                double r[8];
                rl_load_rows(r, bufB);
                __syncthreads();
                rl_tridiag(r, kk, sd, se, stau, bufB, Pp);
                bisect_top_rl(tri_regs(sd, se, kk, ssde), kk, 1, ssin);
                sin_max = sqrt(fmax(ssin[0], 0.0));
            } else {
                // F = B^T B, B = U_R(kk:p, 0:kk)
                for (int idx = threadIdx.x; idx < kk * kk; idx += NT) {
                    const int i = idx % kk, j = idx / kk;
                    double s = 0.0;
                    for (int r = kk; r < p; ++r) s += S3[r + i * p] * S3[r + j * p];
                    S2[i + j * kk] = s;
                }
                __syncthreads();
                tridiag(S2, kk, sd, se, stau, spv, ssc);
                bisect_top(sd, se, kk, 1, ssin, se2, ssc);
                sin_max = sqrt(fmax(ssin[0], 0.0));
            }
        }
    }
    return sin_max;
}

// The tail of a wide merge in one launch of NT-thread workgroups, whose parts
// depend only on U_R and the factors and so run side by side: workgroups
// [0, ntr) solve Z2 = R2^-1 U_R (k_wide_trsm<1>, NT / 64 column tiles each),
// workgroup ntr computes Sigma_new, workgroup ntr + 1 the convergence sine.
// The last workgroup to finish (a counter in the device state, reset by it)
// advances the merge count and rank.
__global__ __launch_bounds__(NT) void k_wide_tail(SmallArgs a, int ntr)
{
    extern __shared__ double lds[];
    DevState *ds = a.ds;
    if (merge_halted(ds)) return;
    const int blk = blockIdx.x;
    if (blk < ntr) {
        wide_trsm_body<1, NT>(a, blk, lds, nullptr);
    } else if (blk == ntr) {
        wide_sig_body(a, lds);
    } else {
        const double sn = wide_sines(a, lds);
        if (threadIdx.x == 0) ds->sin_theta = sn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const int prev = atomicAdd(&ds->tail_done, 1);
        if (prev == (int)gridDim.x - 1) {
            __threadfence();
            const int it0 = ds->it;
            ds->rs = ds->rnew;
            ds->it = it0 + 1;
            ds->g = 0;
            ds->tail_done = 0;
        }
    }
}

__device__ __forceinline__ void svd_merge_body(const SmallArgs &a) { svd_merge_rl(a); }

__global__ __launch_bounds__(512) void k_svd_merge(SmallArgs a)
{
    svd_merge_body(a);
}
// Batched: one workgroup per matrix (blockIdx.y), stopped matrices skipped.
__global__ __launch_bounds__(512) void k_svd_merge_b(const SmallArgs *__restrict__ arr)
{
    const SmallArgs a = arr[blockIdx.y];
    if (a.ds->done) return;
    svd_merge_body(a);
}

hipError_t launch_svd_merge(const SmallArgs &a, hipStream_t st)
{
    const bool big = a.pmax > SMALL_LDS_P;
    if (!big) {
        static bool attr = false;
        if (!attr) {
            hipError_t e = hipFuncSetAttribute((const void *)k_svd_merge, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)svd_merge_lds_rl(SMALL_LDS_P));
            if (e != hipSuccess) return e;
            attr = true;
        }
        ProfScope ps(POD_K_SVD, st);
        hipLaunchKernelGGL(k_svd_merge, dim3(1), dim3(NT), svd_merge_lds_rl(a.pmax), st, a);
        return hipGetLastError();
    }
    // wide merges: the eigensolver's convergence eigenproblem (kk <= 64) and
    // the multisection tables in dynamic LDS
    const size_t lds = (size_t)max(64 * RL_LD + 512 + TRI_SDE, BIG_PACKED) * sizeof(double);
    static bool attr_big = false;
    if (!attr_big) {
        hipError_t e = hipFuncSetAttribute((const void *)k_wide_eig, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_limit(true));
        if (e != hipSuccess) return e;
        attr_big = true;
    }
    static bool attr_z2 = false;
    if (!attr_z2) {
        hipError_t e = hipFuncSetAttribute((const void *)k_wide_tail, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)TRSM_LDS);
        if (e != hipSuccess) return e;
        attr_z2 = true;
    }
    const unsigned tiles = (unsigned)(TRSM_NT * TRSM_NT);
    ProfScope ps(POD_K_SVD, st);
    hipLaunchKernelGGL(k_wide_chol2, dim3(1), dim3(NT), 0, st, a);
    hipLaunchKernelGGL(k_wide_mm<0>, dim3(tiles), dim3(64), 0, st, a);
    hipLaunchKernelGGL(k_wide_mm<1>, dim3(tiles), dim3(64), 0, st, a);
    hipLaunchKernelGGL(k_wide_eig, dim3(1), dim3(NT), lds, st, a);
    const int ntr = (max(a.r, 1) + 16 * (NT / 64) - 1) / (16 * (NT / 64));   // trsm workgroups
    hipLaunchKernelGGL(k_wide_tail, dim3((unsigned)(ntr + 2)), dim3(NT), TRSM_LDS, st, a, ntr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz of the final step on B = U^T A (r x n, ld r):
//   k_rr_gram: G_B = B B^T over chunks of RR_CHUNK columns (one workgroup
//     each, the chunk staged in LDS), partials part[chunk] (upper triangle);
//   k_rr_small: the partials summed in chunk order, eigen-decomposition
//     G_B = U_B Lambda U_B^T (tridiagonalisation, bisection, inverse
//     iteration), U_B(:, 0:kv) (kv = k + 1 when r > k: sigma_{k+1} for the
//     quality measure) and U_B(:, 0:k) in the compute type;
//   k_rr_sig: per chunk and pair index i, sum over its columns c of
//     (B^T U_B)(c, i)^2; k_rr_sig_sum adds the chunks in order:
//     Sigma_B(i) = |B^T U_B(:, i)|, accurate to about r u sigma_1, where
//     sqrt(lambda_i) would lose r u sigma_1^2 / sigma_i.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rr_gram(const double *__restrict__ B, int64_t n, int32_t r,
                                                 double *__restrict__ part)
{
    extern __shared__ double bs[];   // RR_CHUNK x r (column c at bs + c r)
    const int64_t c0 = (int64_t)blockIdx.x * RR_CHUNK;
    const int nc = (n - c0 < RR_CHUNK) ? (int)(n - c0) : RR_CHUNK;
    for (int idx = threadIdx.x; idx < nc * r; idx += 256) bs[idx] = B[c0 * r + idx];
    __syncthreads();
    double *pb = part + (int64_t)blockIdx.x * r * r;
    for (int idx = threadIdx.x; idx < r * r; idx += 256) {
        const int i = idx % r, j = idx / r;
        if (i > j) continue;
        double s = 0.0;
        for (int c = 0; c < nc; ++c) s = fma(bs[i + c * r], bs[j + c * r], s);
        pb[idx] = s;
    }
}

__global__ __launch_bounds__(256) void k_rr_sig(const double *__restrict__ B, int64_t n, int32_t r, int32_t kv,
                                                const double *__restrict__ UB, double *__restrict__ part)
{
    extern __shared__ double bs[];   // RR_CHUNK x r, then RR_CHUNK x 64 squares
    double *sq = bs + RR_CHUNK * r;
    const int64_t c0 = (int64_t)blockIdx.x * RR_CHUNK;
    const int nc = (n - c0 < RR_CHUNK) ? (int)(n - c0) : RR_CHUNK;
    for (int idx = threadIdx.x; idx < nc * r; idx += 256) bs[idx] = B[c0 * r + idx];
    __syncthreads();
    double *pb = part + (int64_t)blockIdx.x * kv;
    for (int i0 = 0; i0 < kv; i0 += 64) {
        // thread (c, l): t = (B^T U_B)(c0 + c, i0 + l)
        for (int idx = threadIdx.x; idx < RR_CHUNK * 64; idx += 256) {
            const int c = idx / 64, l = idx % 64, i = i0 + l;
            double t = 0.0;
            if (c < nc && i < kv)
                for (int j = 0; j < r; ++j) t = fma(bs[j + c * r], UB[j + (int64_t)i * r], t);
            sq[idx] = t * t;
        }
        __syncthreads();
        if (threadIdx.x < 64 && i0 + threadIdx.x < kv) {
            double v = 0.0;
            for (int c = 0; c < nc; ++c) v += sq[c * 64 + threadIdx.x];
            pb[i0 + threadIdx.x] = v;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_rr_sig_sum(const double *__restrict__ part, int32_t nch, int32_t kv,
                                                    double *__restrict__ sig)
{
    for (int i = threadIdx.x; i < kv; i += 256) {
        double v = 0.0;
        for (int b = 0; b < nch; ++b) v += part[(int64_t)b * kv + i];
        sig[i] = sqrt(v);
    }
}

template <bool BIG>
__global__ __launch_bounds__(512) void k_rr_small(RRArgs a)
{
    extern __shared__ double lds[];
    __shared__ double sd[EIG_NMAX], se[EIG_NMAX], stau[EIG_NMAX], se2[EIG_NMAX], spv[EIG_NMAX], sev[EIG_NMAX],
        sdots[EIG_NMAX], ssc[8];
    __shared__ __align__(8) int scl[EIG_NMAX + 8];
    const int r = a.r, k = a.k;
    double *S = BIG ? a.ws : lds; // G_B -> reflectors
    double *Y = S + r * r;        // eigenvectors (r x kv)
    double *lu = BIG ? lds : Y + r * r;  // eig_lu_doubles(r)
    // G_B: the chunk partials summed in chunk order (upper triangle, mirrored)
    const int nch = (int)((a.n + RR_CHUNK - 1) / RR_CHUNK);
    for (int idx = threadIdx.x; idx < r * r; idx += NT) {
        const int i = idx % r, j = idx / r;
        if (i > j) continue;
        double s = 0.0;
        for (int b = 0; b < nch; ++b) s += a.part[(int64_t)b * r * r + idx];
        S[i + j * r] = s;
        S[j + i * r] = s;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < r * r; idx += NT) a.GB[idx] = S[idx];
    tridiag(S, r, sd, se, stau, spv, ssc);
    const int kv = (k < r) ? k + 1 : k;
    bisect_top(sd, se, r, kv, sev, se2, ssc);
    tri_invit(sd, se, r, sev, kv, Y, lu, scl);
    tridiag_backtransform(S, stau, r, Y, kv, sdots);
    for (int idx = threadIdx.x; idx < r * kv; idx += NT) a.UB[idx] = Y[idx];
    for (int idx = threadIdx.x; idx < r * k; idx += NT) store_c(a.Zc, a.prec, idx, Y[idx]);
}

hipError_t launch_rr_small(const RRArgs &a, hipStream_t st)
{
    const bool big = a.r > SMALL_LDS_P;
    const size_t lds = big ? ((size_t)(eig_lu_doubles(a.r)) * sizeof(double)) : ((size_t)(2 * a.r * a.r + eig_lu_doubles(a.r)) * sizeof(double));
    static bool attr[2] = {false, false};
    const void *fn = big ? (const void *)k_rr_small<true> : (const void *)k_rr_small<false>;
    if (!attr[big]) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_limit(big));
        if (e != hipSuccess) return e;
        attr[big] = true;
    }
    static bool attr_chunk = false;
    if (!attr_chunk) {
        // chunk staging beyond the default 64 KiB of dynamic LDS (r up to 160)
        hipError_t e = hipFuncSetAttribute((const void *)k_rr_gram, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           RR_CHUNK * 160 * (int)sizeof(double));
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_rr_sig, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    RR_CHUNK * (160 + 64) * (int)sizeof(double));
        if (e != hipSuccess) return e;
        attr_chunk = true;
    }
    ProfScope ps(POD_K_RR, st);
    const unsigned nch = (unsigned)((a.n + RR_CHUNK - 1) / RR_CHUNK);
    hipLaunchKernelGGL(k_rr_gram, dim3(nch), dim3(256), (size_t)RR_CHUNK * a.r * sizeof(double), st, a.B, a.n, a.r,
                       a.part);
    if (big)
        hipLaunchKernelGGL(k_rr_small<true>, dim3(1), dim3(NT), lds, st, a);
    else
        hipLaunchKernelGGL(k_rr_small<false>, dim3(1), dim3(NT), lds, st, a);
    const int kv = (a.k < a.r) ? a.k + 1 : a.k;
    hipLaunchKernelGGL(k_rr_sig, dim3(nch), dim3(256), (size_t)RR_CHUNK * (a.r + 64) * sizeof(double), st, a.B, a.n,
                       a.r, kv, a.UB, a.part);
    hipLaunchKernelGGL(k_rr_sig_sum, dim3(1), dim3(256), 0, st, a.part, (int32_t)nch, kv, a.sig);
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

// ---------------------------------------------------------------------------
// Right factor of the new block (GET UPDATE of Alg. 1).  Mode 0 (rows
// sampled): W = diag(sqrt(t_hat / (w q))) D(I_r, :) with q_i = w_i / Omega
// (SAMPLE AND SCALE UNIQUE ROWS), G_B = W^T W.  Mode 1 (block truncated to
// its leading directions): G_B = D^T D, the D-block of the pass-1 Gram.
// Eigen-decomposition G_B = V Lambda V^T (descending); Vt = V(:, 0:ru) with
// ru = min(r_lim, g, h, #{lambda_i > g u lambda_1}).  The merge then takes
// C = D Vt: P = blkdiag(Sigma, Vt) in the CholeskyQR passes.
// ---------------------------------------------------------------------------
template <bool BIG>
__global__ __launch_bounds__(512) void k_block_eig(BlockEigArgs a)
{
    extern __shared__ double lds[];
    __shared__ double sd[EIG_NMAX], se[EIG_NMAX], stau[EIG_NMAX], se2[EIG_NMAX], spv[EIG_NMAX], sev[EIG_NMAX],
        sdots[EIG_NMAX], ssc[8];
    __shared__ __align__(8) int scl[EIG_NMAX + 8];
    DevState *ds = a.ds;
    if (merge_halted(ds)) return;
    const int g = ds->g, rs = ds->rs;
    const int pm = a.pmax;
    double *S = BIG ? a.ws : lds; // G_B (g x g) -> reflectors
    double *Y = S + pm * pm;      // eigenvectors (g x ru)
    double *lu = BIG ? lds : Y + pm * pm;  // eig_lu_doubles(g)
    const int h = (a.mode == 0) ? ds->h : g;
    if (g == 0 || h == 0) {
        if (threadIdx.x == 0) {
            ds->ru = 0;
            ds->p = rs;
        }
        return;
    }
    if (a.mode == 0) {
        const double Om = (double)ds->wrow_tot;
        for (int idx = threadIdx.x; idx < g * g; idx += NT) {
            const int i = idx % g, j = idx / g;
            if (i > j) continue;
            const int64_t ci = a.cols[i], cj = a.cols[j];
            double s = 0.0;
            for (int rr = 0; rr < h; ++rr) {
                const int64_t row = a.rows[rr];
                const double q = (double)a.wr[row] / Om;
                const double sc = sqrt((double)a.rcnt[rr] / ((double)a.w * q));
                double di, dj;
                if (a.a_dtype == POD_F64) {
                    di = reinterpret_cast<const double *>(a.A)[ci * a.lda + row];
                    dj = reinterpret_cast<const double *>(a.A)[cj * a.lda + row];
                } else {
                    di = (double)reinterpret_cast<const float *>(a.A)[ci * a.lda + row];
                    dj = (double)reinterpret_cast<const float *>(a.A)[cj * a.lda + row];
                }
                if (a.cscale) {
                    di *= a.cscale[i];
                    dj *= a.cscale[j];
                }
                s += (sc * di) * (sc * dj);
            }
            S[i + j * g] = s;
            S[j + i * g] = s;
        }
        if (a.scales)
            for (int rr = threadIdx.x; rr < h; rr += NT) {
                const double q = (double)a.wr[a.rows[rr]] / Om;
                a.scales[rr] = sqrt((double)a.rcnt[rr] / ((double)a.w * q));
            }
    } else {
        for (int idx = threadIdx.x; idx < g * g; idx += NT) {
            const int i = idx % g, j = idx / g;
            double v = a.G[(rs + i) + (rs + j) * pm];
            if (a.cscale) v = (a.cscale[i] * v) * a.cscale[j];
            S[idx] = v;
        }
    }
    __syncthreads();
    // trace of G_B (= |W|_F^2 of the one-shot CTSVD rule), in index order
    if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int i = 0; i < g; ++i) tr += S[i + i * g];
        ssc[7] = tr;
    }
    __syncthreads();
    const double trace = ssc[7];
    __syncthreads();
    tridiag(S, g, sd, se, stau, spv, ssc);
    int nv = (a.r_lim < g) ? a.r_lim : g;
    if (nv > h) nv = h;
    bisect_top(sd, se, g, nv, sev, se2, ssc);
    const double thr = (a.crit == 1) ? a.gamma * trace : (double)g * 1.1102230246251565e-16 * fmax(sev[0], 0.0);
    const int nz = count_above(sd, se2, g, thr, ssc[2], scl);
    const int ru = (sev[0] > 0.0) ? ((nv < nz) ? nv : nz) : 0;
    tri_invit(sd, se, g, sev, ru, Y, lu, scl);
    tridiag_backtransform(S, stau, g, Y, ru, sdots);
    for (int idx = threadIdx.x; idx < g * ru; idx += NT) {
        const int i = idx % g, j = idx / g;
        a.Vt[i + j * pm] = Y[i + j * g];
    }
    if (a.evals)
        for (int i = threadIdx.x; i < ru; i += NT) a.evals[i] = sev[i];
    if (threadIdx.x == 0) {
        ds->ru = ru;
        ds->p = rs + ru;
    }
}

// ---------------------------------------------------------------------------
// Reverse pass of a row-sampled merge (p <= 64, one workgroup): G = W^T W with
// W = diag(s) A(rows, cols), summed as the forward's block eigensolver sums
// it, then all g eigenpairs (descending) by the same routines; the first ru
// eigenvectors take the signs of the forward's right factor vt.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_adj_rows_eig(AdjRowsArgs a)
{
    extern __shared__ double lds[];
    __shared__ double sd[EIG_NMAX], se[EIG_NMAX], stau[EIG_NMAX], se2[EIG_NMAX], spv[EIG_NMAX], sev[EIG_NMAX],
        sdots[EIG_NMAX], ssc[8];
    __shared__ __align__(8) int scl[EIG_NMAX + 8];
    const int g = a.g, h = a.h, pm = a.pm;
    double *S = lds, *Y = S + pm * pm, *lu = Y + pm * pm;
    for (int idx = threadIdx.x; idx < g * g; idx += NT) {
        const int i = idx % g, j = idx / g;
        if (i > j) continue;
        const int64_t ci = a.cols[i], cj = a.cols[j];
        double sum = 0.0;
        for (int rr = 0; rr < h; ++rr) {
            const int64_t row = a.rows[rr];
            const double sc = a.scales[rr];
            double di, dj;
            if (a.a_dtype == POD_F64) {
                di = reinterpret_cast<const double *>(a.A)[ci * a.lda + row];
                dj = reinterpret_cast<const double *>(a.A)[cj * a.lda + row];
            } else {
                di = (double)reinterpret_cast<const float *>(a.A)[ci * a.lda + row];
                dj = (double)reinterpret_cast<const float *>(a.A)[cj * a.lda + row];
            }
            sum += (sc * di) * (sc * dj);
        }
        S[i + j * g] = sum;
        S[j + i * g] = sum;
    }
    __syncthreads();
    tridiag(S, g, sd, se, stau, spv, ssc);
    bisect_top(sd, se, g, g, sev, se2, ssc);
    tri_invit(sd, se, g, sev, g, Y, lu, scl);
    tridiag_backtransform(S, stau, g, Y, g, sdots);
    // signs of the first ru columns: those of the forward's factor
    for (int j = threadIdx.x >> 6; j < g; j += NT / 64) {
        double d = 0.0;
        if (j < a.ru)
            for (int i = threadIdx.x & 63; i < g; i += 64) d += Y[i + j * g] * a.vt[i + j * pm];
        d = wave_sum(d);
        const double sg = (d < 0.0) ? -1.0 : 1.0;
        for (int i = threadIdx.x & 63; i < g; i += 64) a.vfull[i + j * pm] = sg * Y[i + j * g];
    }
    for (int i = threadIdx.x; i < g; i += NT) a.lam[i] = sev[i];
}

hipError_t launch_adj_rows_eig(const AdjRowsArgs &a, hipStream_t st)
{
    if (a.pm > SMALL_LDS_P || a.g > a.pm) return hipErrorInvalidValue;
    const size_t lds = (size_t)(2 * a.pm * a.pm + eig_lu_doubles(a.pm)) * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_adj_rows_eig, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_limit(false));
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_adj_rows_eig, dim3(1), dim3(NT), lds, st, a);
    return hipGetLastError();
}

// dA(rows[q], cols[j]) += 2 s_q^2 sum_l A(rows[q], cols[l]) Gbar(l, j): one
// thread per (q, j); the (row, column) pairs are distinct.
template <typename TC>
__global__ __launch_bounds__(256) void k_adj_rows_update(AdjRowsArgs a)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= a.h * a.g) return;
    const int q = idx % a.h, j = idx / a.h;
    const int64_t row = a.rows[q];
    double v = 0.0;
    for (int l = 0; l < a.g; ++l) {
        const int64_t cl = a.cols[l];
        const double x = (a.a_dtype == POD_F64) ? reinterpret_cast<const double *>(a.A)[cl * a.lda + row]
                                                : (double)reinterpret_cast<const float *>(a.A)[cl * a.lda + row];
        v = fma(x, a.gbar[l + j * a.pm], v);
    }
    const double sc = a.scales[q];
    TC *d = reinterpret_cast<TC *>(a.dA) + (int64_t)a.cols[j] * a.ldd + row;
    *d += (TC)(2.0 * sc * sc * v);
}

hipError_t launch_adj_rows_update(const AdjRowsArgs &a, hipStream_t st)
{
    const int n = a.h * a.g;
    if (n <= 0) return hipSuccess;
    if (a.prec == POD_F64)
        hipLaunchKernelGGL(k_adj_rows_update<double>, dim3((n + 255) / 256), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_adj_rows_update<float>, dim3((n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_block_eig(const BlockEigArgs &a, hipStream_t st)
{
    const bool big = a.pmax > SMALL_LDS_P;
    const size_t lds = big ? ((size_t)(eig_lu_doubles(a.pmax)) * sizeof(double)) : ((size_t)(2 * a.pmax * a.pmax + eig_lu_doubles(a.pmax)) * sizeof(double));
    static bool attr[2] = {false, false};
    const void *fn = big ? (const void *)k_block_eig<true> : (const void *)k_block_eig<false>;
    if (!attr[big]) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_limit(big));
        if (e != hipSuccess) return e;
        attr[big] = true;
    }
    ProfScope ps(POD_K_DRAW, st);
    if (big)
        hipLaunchKernelGGL(k_block_eig<true>, dim3(1), dim3(NT), lds, st, a);
    else
        hipLaunchKernelGGL(k_block_eig<false>, dim3(1), dim3(NT), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_chol_first_b(const SmallArgs *arr, int32_t count, int32_t pmax_max, hipStream_t st)
{
    if (pmax_max > SMALL_LDS_P || count < 1) return hipErrorInvalidValue;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_chol_first_b, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_limit(false));
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_chol_first_b, dim3(1, (unsigned)count), dim3(NT),
                       chol_first_lds_rl(pmax_max), st, arr);
    return hipGetLastError();
}

hipError_t launch_svd_merge_b(const SmallArgs *arr, int32_t count, int32_t pmax_max, hipStream_t st)
{
    if (pmax_max > SMALL_LDS_P || count < 1) return hipErrorInvalidValue;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_svd_merge_b, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)svd_merge_lds_rl(SMALL_LDS_P));
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_svd_merge_b, dim3(1, (unsigned)count), dim3(NT),
                       svd_merge_lds_rl(pmax_max), st, arr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reverse pass through one merge (adjoint of BLOCK MERGE, Alg. 2).  Forward:
// M = X0 P (X0 = [U_{t-1} | A(:, I_t)], P = diag(Sigma_{t-1}, I)), M = Q R,
// R = U_R S V^T, outputs U_t = Q U_R(:, 0:rz), Sigma_t = S(0:rz).  With the
// output adjoints (Ubar, sbar) the adjoint of M is (thin-SVD adjoint,
// Townsend 2016, V-bar = 0, guarded coupling F)
//   Mbar = U K V^T + (I - U U^T) Ubar S_r^-1 V_r^T,   U = Q U_R,
//   K = (F o (J - J^T)) S + diag(sbar),   J = U^T Ubar.
// Everything reduces to small matrices: with Z = Q^T Ubar = R^-T P (X0^T Ubar)
// and Vs = V S = R^T U_R,
//   Mbar = Q W1 + Ubar W2,  W1 = U_R [(F o (J - J^T)) Vs^T + diag(sbar) V_r^T] - Z S_r^-2 Vs_r^T,
//   W2 = S_r^-2 Vs_r^T,
// and the adjoint of X0 is X0bar = Mbar P = [X0 | Ubar] Wt with
// Wt = [P R^-1 W1 P ; W2 P].  Its first rs columns are Ubar_{t-1}; the rest
// belong to A(:, I_t).  sbar_{t-1,i} = U_{t-1}(:, i)^T Mbar(:, i) comes from the
// Gram of [X0 | Ubar].  The eigen-decomposition of R R^T is recomputed here.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void adj_small_body(const AdjArgs &a);

__global__ __launch_bounds__(512) void k_adj_small(AdjArgs a)
{
    adj_small_body(a);
}

// Batched: one workgroup per matrix (blockIdx.x).
__global__ __launch_bounds__(512) void k_adj_small_b(const AdjArgs *__restrict__ arr)
{
    const AdjArgs a = arr[blockIdx.x];
    adj_small_body(a);
}

__device__ __forceinline__ void adj_small_body(const AdjArgs &a)
{
    extern __shared__ double lds[];
    __shared__ double sd[EIG_NMAX], se[EIG_NMAX], stau[EIG_NMAX], spv[EIG_NMAX], sev[EIG_NMAX], sS[EIG_NMAX],
        sP[EIG_NMAX];
    __shared__ __align__(8) int scl[EIG_NMAX + 8];
    // p: columns of M = X0 P (the merge factor R is p x p); p0: columns of X0.
    // Column-only merges: P = diag(Sigma, I), p0 = p.  Row-sampled merges:
    // P = blkdiag(Sigma, V_u) with V_u = a.vt (g x ru).
    const bool rowm = a.vt != nullptr;
    const int rs = a.rs, p = a.rs + (rowm ? a.ru : a.g), p0 = a.rs + a.g, rz = a.rz, pm = a.pm, pb = a.pb;
    const int t = threadIdx.x;
    double *H = lds;                 // R R^T (p x p, ld p), then the reflectors (64 x RL_LD)
    double *Y = H + 64 * RL_LD;      // eigenvectors (p x p, ld p)
    double *Pp = Y + 64 * 64;        // 8 x 64
    double *lu = Pp + 512;           // INVIT_LDS
    __shared__ double ssde[TRI_SDE];
    const int q2 = pm * pm;
    double *wR = a.ws, *wRi = wR + q2, *wUR = wRi + q2, *wV = wUR + q2, *wZ = wV + q2, *wJ = wZ + q2, *wK = wJ + q2,
           *wN = wK + q2, *wW = wN + q2, *wT = wW + q2, *wP = wT + q2, *wQ = wP + q2;
    // P (p0 x p, ld p0) of a row-sampled merge
    if (rowm)
        for (int idx = t; idx < p0 * p; idx += NT) {
            const int i = idx % p0, j = idx / p0;
            double v = 0.0;
            if (i < rs && j < rs) v = (i == j) ? a.sig[i] : 0.0;
            else if (i >= rs && j >= rs) v = a.vt[(i - rs) + (j - rs) * pm];
            wP[idx] = v;
        }
    for (int idx = t; idx < p * p; idx += NT) {
        const int i = idx % p, j = idx / p;
        const double v = a.R[i + j * pm];
        wR[idx] = v;
        wRi[idx] = v;
    }
    for (int i = t; i < p; i += NT) sP[i] = (i < rs) ? a.sig[i] : 1.0;
    __syncthreads();
    for (int idx = t; idx < p * p; idx += NT) {
        const int i = idx % p, j = idx / p;
        const int l0 = (i > j) ? i : j;
        double s = 0.0;
        for (int l = l0; l < p; ++l) s += wR[i + l * p] * wR[j + l * p];
        H[idx] = s;
    }
    __syncthreads();
    trinv_upper<false>(wR, p, wRi, spv);
    // the eigensolver of the forward merge (same start vectors, so the same signs of U_R)
    {
        double r[8];
        rl_load_sym(r, H, p, p);
        __syncthreads();
        rl_tridiag(r, p, sd, se, stau, H, Pp);
    }
    const TriRegs tt = tri_regs(sd, se, p, ssde);
    bisect_top_rl(tt, p, p, sev);
    tri_invit_rl(tt, p, sev, p, Y, lu, scl);
    rl_backtransform(H, stau, p, Y, p);
    for (int i = t; i < p; i += NT) sS[i] = sqrt(fmax(sev[i], 0.0));
    for (int idx = t; idx < p * p; idx += NT) wUR[idx] = Y[idx];
    __syncthreads();
    // Vs = R^T U_R;  Z = R^-T (P X0^T Ubar)
    for (int idx = t; idx < p * p; idx += NT) {
        const int i = idx % p, j = idx / p;
        double s = 0.0;
        for (int l = 0; l <= i; ++l) s += wR[l + i * p] * wUR[l + j * p];
        wV[idx] = s;
    }
    if (!rowm) {
        for (int idx = t; idx < p * rz; idx += NT) {
            const int i = idx % p, j = idx / p;
            double s = 0.0;
            for (int l = 0; l <= i; ++l) s += wRi[l + i * p] * sP[l] * a.Gext[l + (p + j) * pb];
            wZ[i + j * p] = s;
        }
    } else {
        // Q = P^T X0^T Ubar (p x rz), then Z = R^-T Q
        for (int idx = t; idx < p * rz; idx += NT) {
            const int i = idx % p, j = idx / p;
            double s = 0.0;
            for (int l = 0; l < p0; ++l) s += wP[l + i * p0] * a.Gext[l + (p0 + j) * pb];
            wQ[i + j * p] = s;
        }
        __syncthreads();
        for (int idx = t; idx < p * rz; idx += NT) {
            const int i = idx % p, j = idx / p;
            double s = 0.0;
            for (int l = 0; l <= i; ++l) s += wRi[l + i * p] * wQ[l + j * p];
            wZ[i + j * p] = s;
        }
    }
    __syncthreads();
    // J = U_R^T Z (p x rz)
    for (int idx = t; idx < p * rz; idx += NT) {
        const int i = idx % p, j = idx / p;
        double s = 0.0;
        for (int l = 0; l < p; ++l) s += wUR[l + i * p] * wZ[l + j * p];
        wJ[i + j * p] = s;
    }
    __syncthreads();
    // K~ = F o (J - J^T)  (J zero beyond column rz)
    {
        const double l1 = sS[0] * sS[0];
        const double gl = a.eta * l1;
        for (int idx = t; idx < p * p; idx += NT) {
            const int i = idx % p, j = idx / p;
            double v = 0.0;
            if (i != j) {
                const double d = sS[j] * sS[j] - sS[i] * sS[i];
                const double f = d / (d * d + gl * gl);
                const double jij = (j < rz) ? wJ[i + j * p] : 0.0;
                const double jji = (i < rz) ? wJ[j + i * p] : 0.0;
                v = f * (jij - jji);
            }
            wK[idx] = v;
        }
    }
    __syncthreads();
    // N = K~ Vs^T + diag(sbar) V_r^T   (V_r = Vs_r S_r^-1)
    for (int idx = t; idx < p * p; idx += NT) {
        const int i = idx % p, c = idx / p;
        double s = 0.0;
        for (int j = 0; j < p; ++j) s += wK[i + j * p] * wV[c + j * p];
        if (i < rz) s += a.sbar_in[i] / sS[i] * wV[c + i * p];
        wN[idx] = s;
    }
    __syncthreads();
    // W1 = U_R N - Z S_r^-2 Vs_r^T
    for (int idx = t; idx < p * p; idx += NT) {
        const int r0 = idx % p, c = idx / p;
        double s = 0.0;
        for (int i = 0; i < p; ++i) s += wUR[r0 + i * p] * wN[i + c * p];
        for (int j = 0; j < rz; ++j) s -= wZ[r0 + j * p] * wV[c + j * p] / (sS[j] * sS[j]);
        wW[idx] = s;
    }
    __syncthreads();
    // T = P R^-1 W1 (the factor of Mbar on X0; p0 x p, ld p0)
    if (!rowm) {
        for (int idx = t; idx < p * p; idx += NT) {
            const int r0 = idx % p, c = idx / p;
            double s = 0.0;
            for (int l = r0; l < p; ++l) s += wRi[r0 + l * p] * wW[l + c * p];
            wT[idx] = sP[r0] * s;
        }
    } else {
        for (int idx = t; idx < p * p; idx += NT) {
            const int r0 = idx % p, c = idx / p;
            double s = 0.0;
            for (int l = r0; l < p; ++l) s += wRi[r0 + l * p] * wW[l + c * p];
            wQ[idx] = s;
        }
        __syncthreads();
        for (int idx = t; idx < p0 * p; idx += NT) {
            const int r0 = idx % p0, c = idx / p0;
            double s = 0.0;
            for (int l = 0; l < p; ++l) s += wP[r0 + l * p0] * wQ[l + c * p];
            wT[idx] = s;
        }
    }
    __syncthreads();
    if (!rowm) {
        // Wt = [T P ; W2 P]
        for (int idx = t; idx < (p + rz) * p; idx += NT) {
            const int row = idx % (p + rz), c = idx / (p + rz);
            double v;
            if (row < p) v = wT[row + c * p] * sP[c];
            else v = wV[c + (row - p) * p] / (sS[row - p] * sS[row - p]) * sP[c];
            store_c(a.Wt, a.prec, row + (int64_t)c * pb, v);
        }
        // sbar_{t-1,i} = [X0^T X0 T + X0^T Ubar W2]_{ii}
        for (int i = t; i < rs; i += NT) {
            double s = 0.0;
            for (int l = 0; l < p; ++l) s += a.Gext[i + l * pb] * wT[l + i * p];
            for (int j = 0; j < rz; ++j) s += a.Gext[i + (p + j) * pb] * wV[i + j * p] / (sS[j] * sS[j]);
            a.sbar_out[i] = s;
        }
        return;
    }
    // row-sampled merge: Wt = [T P^T ; W2 P^T] ((p0 + rz) x p0), W2(j, l) = Vs(l, j) / s_j^2
    for (int idx = t; idx < (p0 + rz) * p0; idx += NT) {
        const int row = idx % (p0 + rz), c = idx / (p0 + rz);
        double v = 0.0;
        if (row < p0)
            for (int l = 0; l < p; ++l) v += wT[row + l * p0] * wP[c + l * p0];
        else
            for (int l = 0; l < p; ++l) v += wV[l + (row - p0) * p] / (sS[row - p0] * sS[row - p0]) * wP[c + l * p0];
        store_c(a.Wt, a.prec, row + (int64_t)c * pb, v);
    }
    for (int i = t; i < rs; i += NT) {
        double s = 0.0;
        for (int l = 0; l < p0; ++l) s += a.Gext[i + l * pb] * wT[l + i * p0];
        for (int j = 0; j < rz; ++j) s += a.Gext[i + (p0 + j) * pb] * wV[i + j * p] / (sS[j] * sS[j]);
        a.sbar_out[i] = s;
    }
    // adjoint of V_u: Vbar = [X0^T Mbar](rs:p0, rs:p), X0^T Mbar = Gext(0:p0, :) [T ; W2]
    const int g = a.g, ru = a.ru;
    if (ru == 0) {   // no retained direction: V_u is empty and so is its adjoint
        for (int idx = t; idx < g * g; idx += NT) a.gbar[(idx % g) + (idx / g) * pm] = 0.0;
        return;
    }
    double *wVb = wJ, *wKg = wK, *wG = wN;
    for (int idx = t; idx < g * ru; idx += NT) {
        const int i = idx % g, b = idx / g;
        const int row = rs + i, col = rs + b;
        double s = 0.0;
        for (int l = 0; l < p0; ++l) s += a.Gext[row + l * pb] * wT[l + col * p0];
        for (int j = 0; j < rz; ++j) s += a.Gext[row + (p0 + j) * pb] * wV[col + j * p] / (sS[j] * sS[j]);
        wVb[i + b * g] = s;
    }
    __syncthreads();
    // K(i, j) = (v_i^T Vbar_j) / (lambda_j - lambda_i) (i != j, j < ru; eta guard), G-bar = V K V^T
    {
        const double gl = a.eta * fabs(a.lam[0]);
        for (int idx = t; idx < g * g; idx += NT) {
            const int i = idx % g, j = idx / g;
            double v = 0.0;
            if (i != j && j < ru) {
                double dt = 0.0;
                for (int l = 0; l < g; ++l) dt += a.vfull[l + i * pm] * wVb[l + j * g];
                const double d = a.lam[j] - a.lam[i];
                v = (d == 0.0) ? 0.0 : dt * (d / (d * d + gl * gl));
            }
            wKg[idx] = v;
        }
    }
    __syncthreads();
    for (int idx = t; idx < g * g; idx += NT) {   // V K
        const int i = idx % g, j = idx / g;
        double s = 0.0;
        for (int l = 0; l < g; ++l) s += a.vfull[i + l * pm] * wKg[l + j * g];
        wG[idx] = s;
    }
    __syncthreads();
    for (int idx = t; idx < g * g; idx += NT) {   // (V K) V^T
        const int i = idx % g, j = idx / g;
        double s = 0.0;
        for (int l = 0; l < g; ++l) s += wG[i + l * g] * a.vfull[j + l * pm];
        wKg[idx] = s;
    }
    __syncthreads();
    for (int idx = t; idx < g * g; idx += NT) {
        const int i = idx % g, j = idx / g;
        a.gbar[i + j * pm] = 0.5 * (wKg[i + j * g] + wKg[j + i * g]);
    }
}

hipError_t launch_adj_small(const AdjArgs &a, hipStream_t st)
{
    const int p = a.rs + a.g;
    if (a.pm > SMALL_LDS_P || p > a.pm) return hipErrorInvalidValue;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_adj_small, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_limit(false));
        if (e != hipSuccess) return e;
        attr = true;
    }
    const size_t lds = (size_t)(64 * RL_LD + 64 * 64 + 512 + INVIT_LDS) * sizeof(double);
    hipLaunchKernelGGL(k_adj_small, dim3(1), dim3(NT), lds, st, a);
    return hipGetLastError();
}

// Every entry must satisfy launch_adj_small's bounds (checked by the caller).
hipError_t launch_adj_small_b(const AdjArgs *arr, int32_t count, hipStream_t st)
{
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_adj_small_b, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_limit(false));
        if (e != hipSuccess) return e;
        attr = true;
    }
    const size_t lds = (size_t)(64 * RL_LD + 64 * 64 + 512 + INVIT_LDS) * sizeof(double);
    hipLaunchKernelGGL(k_adj_small_b, dim3((unsigned)count), dim3(NT), lds, st, arr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The small adjoint of a wide merge (SMALL_LDS_P < pmax, p <= 160; column
// draws): the steps and arithmetic of adj_small_body with P = diag(Sigma, I),
// split over launches.  k_adj_wide_eig (one workgroup) recomputes the full
// eigen-decomposition R R^T = U_R S^2 U_R^T with the forward merge's
// eigensolver (same start vectors, so the same signs of U_R) and R^-1; then
// each product of the adjoint is one launch with one output element per
// thread over as many workgroups as it has elements (the operands are L2
// resident).  All matrices in the workspace have leading dimension p.
// ---------------------------------------------------------------------------
struct AdjWideWs {
    double *R, *H, *UR, *W, *Ri, *V, *Z, *J, *K, *N, *Wm, *T, *s, *sp;
};

__device__ __forceinline__ AdjWideWs adj_wide_ws(double *ws, int pm)
{
    const size_t q = (size_t)pm * pm;
    AdjWideWs w;
    w.R = ws;
    w.H = ws + q;                  // R R^T, then the reflectors
    w.UR = ws + 2 * q;             // eigenvectors (all p)
    w.W = ws + 3 * q + pm;         // inverse-iteration scratch (BIG_INVIT_DOUBLES)
    double *b = w.W + BIG_INVIT_DOUBLES;
    w.Ri = b;                      // R^-1
    w.V = b + q;                   // Vs = R^T U_R
    w.Z = b + 2 * q;               // R^-T P X0^T Ubar (p x rz)
    w.J = b + 3 * q;               // U_R^T Z (p x rz)
    w.K = b + 4 * q;               // F o (J - J^T)
    w.N = b + 5 * q;
    w.Wm = b + 6 * q;              // W1
    w.T = b + 7 * q;               // P R^-1 W1
    w.s = b + 8 * q;               // singular values of R (p)
    w.sp = w.s + pm;               // diagonal of P (p)
    return w;
}

static_assert(BIG_TRI_SDE <= BIG_PACKED && EIG_NMAX * 64 <= BIG_PACKED, "the wide adjoint's dynamic LDS");

__global__ __launch_bounds__(512) void k_adj_wide_eig(AdjArgs a)
{
    extern __shared__ double lds[];
    __shared__ double sd[EIG_NMAX], se[EIG_NMAX], stau[EIG_NMAX], sev[EIG_NMAX], stmp[EIG_NMAX];
    __shared__ __align__(8) int scl[EIG_NMAX + 8];
    const int p = a.rs + a.g;
    const AdjWideWs w = adj_wide_ws(a.ws, a.pm);
    for (int idx = threadIdx.x; idx < p * p; idx += NT) {
        const int i = idx % p, j = idx / p;
        w.R[idx] = (i <= j) ? a.R[i + (size_t)j * a.pm] : 0.0;
    }
    __syncthreads();
    // H = R R^T on the matrix cores: tile (I, J) sums k from 16 max(I, J)
    big_mm(
        p, false, [&](int i, int k) { return (i < p && k < p) ? w.R[i + k * p] : 0.0; },
        [&](int k, int j) { return (j < p && k < p) ? w.R[j + k * p] : 0.0; },
        [&](int i, int j, double v) {
            if (i < p && j < p) w.H[i + j * p] = v;
        },
        [&](int ti, int tj, int &k0, int &k1) {
            k0 = 16 * ((ti > tj) ? ti : tj);
            (void)k1;
        });
    __syncthreads();
    big_tridiag(w.H, p, sd, se, stau);
    const BigTri bt = big_tri(sd, se, p, lds);
    big_bisect_top(bt, p, p, sev);
    big_invit(sd, se, p, sev, p, w.UR, w.W, lds, scl);
    big_backtransform(w.H, stau, p, w.UR, p);
    for (int i = threadIdx.x; i < p; i += NT) {
        w.s[i] = sqrt(fmax(sev[i], 0.0));
        w.sp[i] = (i < a.rs) ? a.sig[i] : 1.0;
    }
    trinv_upper<true>(w.R, p, w.Ri, stmp);
}

template <int STEP> __global__ __launch_bounds__(256) void k_adj_wide_step(AdjArgs a)
{
    const int rs = a.rs, p = a.rs + a.g, rz = a.rz, pb = a.pb;
    const AdjWideWs w = adj_wide_ws(a.ws, a.pm);
    const int idx = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (STEP == 0) {
        if (idx < p * p) {   // Vs = R^T U_R
            const int i = idx % p, j = idx / p;
            double s = 0.0;
            for (int l = 0; l <= i; ++l) s += w.R[l + i * p] * w.UR[l + j * p];
            w.V[idx] = s;
        } else if (idx < p * p + p * rz) {   // Z = R^-T P X0^T Ubar
            const int e = idx - p * p, i = e % p, j = e / p;
            double s = 0.0;
            for (int l = 0; l <= i; ++l) s += w.Ri[l + i * p] * w.sp[l] * a.Gext[l + (size_t)(p + j) * pb];
            w.Z[i + j * p] = s;
        }
    } else if (STEP == 1) {   // J = U_R^T Z
        if (idx < p * rz) {
            const int i = idx % p, j = idx / p;
            double s = 0.0;
            for (int l = 0; l < p; ++l) s += w.UR[l + i * p] * w.Z[l + j * p];
            w.J[i + j * p] = s;
        }
    } else if (STEP == 2) {   // K~ = F o (J - J^T), J zero beyond column rz
        if (idx < p * p) {
            const int i = idx % p, j = idx / p;
            const double gl = a.eta * w.s[0] * w.s[0];
            double v = 0.0;
            if (i != j) {
                const double d = w.s[j] * w.s[j] - w.s[i] * w.s[i];
                const double f = d / (d * d + gl * gl);
                const double jij = (j < rz) ? w.J[i + j * p] : 0.0;
                const double jji = (i < rz) ? w.J[j + i * p] : 0.0;
                v = f * (jij - jji);
            }
            w.K[idx] = v;
        }
    } else if (STEP == 3) {   // N = K~ Vs^T + diag(sbar) V_r^T
        if (idx < p * p) {
            const int i = idx % p, c = idx / p;
            double s = 0.0;
            for (int j = 0; j < p; ++j) s += w.K[i + j * p] * w.V[c + j * p];
            if (i < rz) s += a.sbar_in[i] / w.s[i] * w.V[c + i * p];
            w.N[idx] = s;
        }
    } else if (STEP == 4) {   // W1 = U_R N - Z S_r^-2 Vs_r^T
        if (idx < p * p) {
            const int r0 = idx % p, c = idx / p;
            double s = 0.0;
            for (int i = 0; i < p; ++i) s += w.UR[r0 + i * p] * w.N[i + c * p];
            for (int j = 0; j < rz; ++j) s -= w.Z[r0 + j * p] * w.V[c + j * p] / (w.s[j] * w.s[j]);
            w.Wm[idx] = s;
        }
    } else if (STEP == 5) {   // T = P R^-1 W1
        if (idx < p * p) {
            const int r0 = idx % p, c = idx / p;
            double s = 0.0;
            for (int l = r0; l < p; ++l) s += w.Ri[r0 + l * p] * w.Wm[l + c * p];
            w.T[idx] = w.sp[r0] * s;
        }
    } else {
        if (idx < (p + rz) * p) {   // Wt = [T P ; W2 P]
            const int row = idx % (p + rz), c = idx / (p + rz);
            double v;
            if (row < p) v = w.T[row + c * p] * w.sp[c];
            else v = w.V[c + (row - p) * p] / (w.s[row - p] * w.s[row - p]) * w.sp[c];
            store_c(a.Wt, a.prec, row + (int64_t)c * pb, v);
        } else if (idx < (p + rz) * p + rs) {   // sbar_{t-1,i} = [X0^T X0 T + X0^T Ubar W2]_{ii}
            const int i = idx - (p + rz) * p;
            double s = 0.0;
            for (int l = 0; l < p; ++l) s += a.Gext[i + (size_t)l * pb] * w.T[l + i * p];
            for (int j = 0; j < rz; ++j) s += a.Gext[i + (size_t)(p + j) * pb] * w.V[i + j * p] / (w.s[j] * w.s[j]);
            a.sbar_out[i] = s;
        }
    }
}

hipError_t launch_adj_wide(const AdjArgs &a, hipStream_t st)
{
    const int p = a.rs + a.g;
    if (a.vt || p > EIG_NMAX || p > a.pm || a.rz < 0 || a.rz > p || p + a.rz > a.pb) return hipErrorInvalidValue;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_adj_wide_eig, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_limit(true));
        if (e != hipSuccess) return e;
        attr = true;
    }
    if (p < 1) return hipSuccess;
    auto grid = [](int n) { return dim3((unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1)); };
    const int pp = p * p, prz = p * a.rz;
    hipLaunchKernelGGL(k_adj_wide_eig, dim3(1), dim3(NT), (size_t)BIG_PACKED * sizeof(double), st, a);
    hipLaunchKernelGGL(k_adj_wide_step<0>, grid(pp + prz), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_adj_wide_step<1>, grid(prz), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_adj_wide_step<2>, grid(pp), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_adj_wide_step<3>, grid(pp), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_adj_wide_step<4>, grid(pp), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_adj_wide_step<5>, grid(pp), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_adj_wide_step<6>, grid((p + a.rz) * p + a.rs), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace pod

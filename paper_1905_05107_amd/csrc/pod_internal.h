// pod_internal.h -- shared device/host declarations of the gfx950 ISMA library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pod.h"

namespace pod {

// Device-resident progress of one context.  Kernels read sizes from here so
// that one iteration (sample -> merge) runs without a host round trip.
struct DevState {
    int32_t it;         // merges done so far (= iteration index of the next draw)
    int32_t rs;         // columns of the current basis U
    int32_t g;          // distinct columns of the pending draw
    int32_t h;          // distinct rows of the pending draw
    int32_t ru;         // columns of the update block after its right factor
    int32_t p0;         // rs + g: columns of the gathered block X0 = [U | A(:, I_c)]
    int32_t p;          // rs + ru: columns of M = X0 P
    int32_t rnew;       // rank after the pending merge
    int32_t exhausted;  // no drawable column at the last draw
    int32_t flags;      // bit0 shifted Cholesky, bit1 non-finite, bit2 Jacobi limit, bit3 zero row weights,
                        // bit4 Cholesky breakdown after the shifted retry
    int32_t sweeps;     // Jacobi sweeps of the last merge
    int32_t col_log_len;// entries used in the column log
    int32_t s_empty;    // no drawable column left after the last draw
    int32_t sweeps_total; // Jacobi sweeps summed over merges
    int32_t done;       // batched or device-driven runs: this run stopped (merge-time kernels skip)
    int32_t tail_done;  // workgroups of the wide merge's tail kernel finished (0 between launches)
    double sin_theta;   // last convergence sine (NaN until the second merge)
    uint64_t wtot;      // total column weight of the last draw
    uint64_t wrow_tot;  // total row weight of the last row draw
};

enum : int32_t { FLAG_SHIFT = 1, FLAG_NONFINITE = 2, FLAG_NOCONV = 4, FLAG_ZERO_ROWS = 8, FLAG_NOTPD = 16 };
// Flags that end a run (the merged state is no longer meaningful).
constexpr int32_t FLAG_FATAL = FLAG_NONFINITE | FLAG_NOTPD;

// The merge-time kernels do nothing when the pending draw found S exhausted
// or the run has stopped (`done`, set on the device by the stop test of a
// batched or device-driven run).
__device__ __forceinline__ bool merge_halted(const DevState *ds) { return ds->exhausted || ds->done; }

// ---------------------------------------------------------------- Philox-4x64-10
// Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11: ten rounds of two 64x64->128 multiplies with a Weyl key schedule.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t lo0 = 0xD2E7470EE14C6C93ULL * c[0];
        const uint64_t hi0 = __umul64hi(0xD2E7470EE14C6C93ULL, c[0]);
        const uint64_t lo1 = 0xCA5A826395121157ULL * c[2];
        const uint64_t hi1 = __umul64hi(0xCA5A826395121157ULL, c[2]);
        const uint64_t n0 = hi1 ^ c[1] ^ k0;
        const uint64_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
}

// ---------------------------------------------------------------- MFMA wrappers
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<double> { typedef v4d type; };
template <> struct Acc<float> { typedef v4f type; };

// D(16x16) += A(16x4) * B(4x16).  Lane l supplies A[l%16][l/16] and
// B[l/16][l%16].  Its four results are D[acc_row<T>(l, v)][l%16], v = 0..3:
// rows 4*(l/16)+v for the FP32 instruction, rows l/16 + 4v for the FP64 one.
template <typename T> __device__ __forceinline__ int acc_row(int lane, int v);
template <> __device__ __forceinline__ int acc_row<float>(int lane, int v) { return 4 * (lane >> 4) + v; }
template <> __device__ __forceinline__ int acc_row<double>(int lane, int v) { return (lane >> 4) + 4 * v; }
__device__ __forceinline__ v4d mfma16x16x4(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16x16x4(float a, float b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

}  // namespace pod

// ---------------------------------------------------------------- host launchers
namespace pod {

// Brackets one launch with HIP events when its kernel class is being profiled.
struct ProfScope {
    ProfScope(int kclass, hipStream_t st);
    ~ProfScope();
    bool on;
    hipStream_t st;
};

hipError_t launch_col_sqnorms(const void *A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, double *nu,
                              hipStream_t st);
// Row centring of A in place; scratch holds center_splits(m) * m doubles.
int32_t center_splits(int64_t m);
hipError_t launch_center_rows(void *A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda, double *scratch,
                              hipStream_t st);
hipError_t launch_quantize(const double *v, int64_t len, uint64_t *w, DevState *ds, int32_t guard, hipStream_t st);

struct DrawArgs {
    const uint64_t *wq;   // weights of the draw (n): L2N, or ORT from the second iteration
    const uint64_t *wq_left; // weights that decide whether S keeps a drawable column (nullable: wq)
    uint8_t *inS;         // membership of S (n)
    int64_t n;
    int32_t c;
    int32_t unf;          // uniform weights over S from the second iteration
    uint64_t seed, block;
    int32_t *cols;        // out: distinct columns (c)
    int32_t *ccnt;        // out: multiplicities (c)
    int32_t *col_log;     // out: appended distinct columns (n)
    int32_t *ccnt_log;    // out: their multiplicities (n)
    int32_t *col_log_off; // out: offsets per merge (max_iter + 1)
    int32_t max_iter;
    const int32_t *forced;// replayed columns and their counts (forced + 1024) (nullable)
    int32_t forced_g;
    DevState *ds;
};
hipError_t launch_draw_cols(const DrawArgs &a, hipStream_t st);
hipError_t launch_draw_cols_b(const DrawArgs *arr, int32_t count, hipStream_t st);
hipError_t launch_run_done(DevState *ds, int32_t max_iter, double tol, int32_t stop_conv, double *sin_log,
                           int32_t log_cap, hipStream_t st);
hipError_t launch_batch_done(DevState *const *dss, const int32_t *max_iter, const double *sin_tol, int32_t count,
                             int32_t *ndone, hipStream_t st);

// Row squared norms of the gathered block D = A(:, cols[0..g)) (rows of D in
// ascending column order, FP64 fma chain), g read from the device state.
hipError_t launch_row_sqnorms(const void *A, int32_t a_dtype, int64_t m, int64_t lda, const int32_t *cols,
                              const void *U0, const void *U1, int32_t u_prec, int32_t k_ls, const DevState *ds,
                              double *rho, hipStream_t st, const double *cscale = nullptr);
struct RowDrawArgs {
    const uint64_t *wr;    // row weights (m)
    int64_t m;
    int32_t w;             // draws
    uint64_t seed, block;
    int32_t *rows;         // out: distinct rows (w)
    int32_t *rcnt;         // out: multiplicities (w)
    int32_t *row_log;      // out: per merge, w entries
    int32_t *rcnt_log;
    int32_t max_iter;
    const int32_t *forced;   // replayed rows and their counts (forced + 1024) (nullable)
    int32_t forced_h;
    DevState *ds;
};
hipError_t launch_draw_rows(const RowDrawArgs &a, hipStream_t st);
// Device state for a merge with an external basis of rb columns (Alg. 3):
// the first one becomes the state (rs = min(rb, r)); later ones are the new
// block, gathered through cols = 0..rb-1.
hipError_t launch_basis_state(DevState *ds, int32_t rb, int32_t r, int32_t first, int32_t *cols, hipStream_t st);

struct GemmDesc {
    int32_t prec;         // POD_F64, POD_F32 or POD_BF16_REFINE (FP32 compute type, split-BF16 matrix cores)
    int32_t a_dtype;      // storage of A
    int64_t m;
    const void *U;        // basis (compute type), ld = m
    const void *U1;       // nullable; when set the basis is U1 if the device merge count is odd, else U
    const void *A;
    int64_t lda;
    const int32_t *cols;
    const void *Y;        // contiguous m x P source (compute type), ld = m (when gather == 0)
    int32_t gather;       // 1: source is X0 = [U | A(:, cols)], 0: Y
    int32_t guard;        // 1: skip when the pending draw found S exhausted
    const void *Z;        // nullable: gathered source extended to [U | A(:, cols) | Z] (compute type, ld m),
                          // the A block being ds->g columns wide
    void *tsplit = nullptr;  // POD_BF16_REFINE: workspace for the split right factor of the tall
                             // transform (TSPLIT_BYTES)
};
// Workspace of the split right factor: three bf16 terms of a 160 x 160 factor.
constexpr size_t TSPLIT_BYTES = 3 * 160 * 160 * 2;
// Partial Grams of the first `P` (device count) columns of the source, P <= pmax.
// Kernels launched with guard = 1 do nothing when the pending draw found S exhausted.
hipError_t launch_gram_partial(const GemmDesc &d, const DevState *ds, int32_t which_p, int32_t pmax, double *part,
                               int32_t nblk, hipStream_t st);
hipError_t launch_gram_reduce_sel(const double *part, int32_t nblk, int32_t pmax, const DevState *ds,
                                  int32_t which_p, double *G, hipStream_t st);
// Y (m x pout, ld m) = source (m x pin) * T (pin x pout, ld ldt); counts from the device state.
// With Yout1 set, the output is Yout1 if the device merge count is odd, else Yout.
// tri: T is upper triangular (T(k, j) = 0 for k > j); the zero tiles are skipped.
hipError_t launch_gemm_tall(const GemmDesc &d, const DevState *ds, int32_t which_in, int32_t which_out,
                            int32_t pin_max, int32_t pout_max, const void *T, int32_t ldt, void *Yout, void *Yout1,
                            hipStream_t st, int32_t tri = 0);

// Per-matrix arguments of the batched launches (device arrays, one entry per
// matrix; blockIdx.y selects the entry).
struct GramArgs {
    GemmDesc d;
    const DevState *ds;
    int32_t which_p, pmax, nblk, vec;
    double *part;
    double *G;
};
struct TallArgs {
    GemmDesc d;
    const DevState *ds;
    int32_t sel_in, sel_out, pin_max, pout_max;  // pin_max / pout_max: multiples of 16
    const void *T;
    int32_t ldt, vec, nb;
    int32_t tri;           // T upper triangular (launch_gemm_tall)
    void *Yout, *Yout1;
};
// Batched launches (pmax <= 64 for every matrix; prec uniform).
hipError_t launch_gram_partial_b(const GramArgs *arr, int32_t count, int32_t max_nblk, int32_t pmax_max, int32_t prec,
                                 hipStream_t st);
hipError_t launch_gram_reduce_b(const GramArgs *arr, int32_t count, int32_t pmax_max, hipStream_t st);
hipError_t launch_gemm_tall_b(const TallArgs *arr, int32_t count, int32_t max_nb, int32_t pi_max, int32_t po_max,
                              int32_t prec, hipStream_t st);
// Host checks of one matrix's arguments
int32_t gemm_vec_ok(const GemmDesc &d);
int32_t tall_blocks(int64_t m);

// Y = source T as launch_gemm_tall (no parity selection), except that output
// column split + j is added to D(:, cmap[j]) (ld ldd) instead of being stored.
hipError_t launch_gemm_tall_scatter(const GemmDesc &d, const DevState *ds, int32_t which_in, int32_t which_out,
                                    int32_t pin_max, int32_t pout_max, const void *T, int32_t ldt, void *Yout,
                                    int32_t split, const int32_t *cmap, void *D, int64_t ldd, hipStream_t st);

// Merge widths up to this run the register-resident small kernels.
constexpr int SMALL_LDS_P = 64;
// Device scratch of the inverse iteration of wide merges (p > SMALL_LDS_P):
// six arrays of 160 rows for 64 lanes.
constexpr size_t BIG_INVIT_DOUBLES = (size_t)6 * 160 * 64;
// inverses of the 16 x 16 diagonal blocks of a wide merge's triangular factor
constexpr size_t BIG_DINV_DOUBLES = (size_t)(160 / 16) * 256;
__host__ __device__ constexpr size_t big_dinv_offset(int pmax)
{
    return (size_t)3 * pmax * pmax + pmax + BIG_INVIT_DOUBLES;
}

struct SmallArgs {
    DevState *ds;
    const double *Vt;      // right factor of the new block (g x ru, ld pmax) when use_vt
    int32_t use_vt;
    double *sig0, *sig1;   // Sigma pair: current = sig[it & 1], the merge writes sig[(it + 1) & 1]
    const double *sigma2;  // weights of the new block's columns (nullable: 1)
    const double *G;       // reduced Gram (pmax x pmax, ld pmax)
    double *R1;            // (pmax x pmax)
    double *R2;            // (pmax x pmax) receives the merge factor R = R2 R1
    void *Tc;              // transform in compute type (pmax x pmax, ld pmax)
    double *work;          // scratch (pmax x pmax)
    double *ws;            // matrices of the kernel when pmax > 64 (3 pmax^2 + pmax)
    int32_t pmax;
    int32_t r, k;
    int32_t prec;
    int32_t criterion;
    double urnd;           // unit roundoff of the merge arithmetic
};
hipError_t launch_chol_first(const SmallArgs &a, hipStream_t st);

// Right factor of the new block: the top right singular directions of the
// scaled row sample W (mode 0, SAMPLE AND SCALE UNIQUE ROWS) or of D itself
// through the D-block of the pass-1 Gram (mode 1, truncated block update):
// eigen-decomposition of W^T W (resp. D^T D), Vt = its top ru eigenvectors,
// ru = min(r_lim, g, h, #{lambda_i > g u lambda_1}); sets ds->ru and ds->p.
struct BlockEigArgs {
    int32_t mode;
    int32_t a_dtype;
    const void *A;
    int64_t lda, m;
    const int32_t *cols, *rows, *rcnt;
    int32_t w;
    const uint64_t *wr;
    const double *G;       // pass-1 Gram (mode 1), pmax x pmax
    int32_t pmax;
    int32_t r_lim;
    double *Vt;            // out, g x ru (ld pmax)
    double *ws;            // matrices of the kernel when pmax > 64 (2 pmax^2)
    DevState *ds;
    // one-shot sampled SVDs (Appendix A): column scales of the block (nullable),
    // the kept eigenvalues (nullable), and the rule for ru: 0 the rank rule
    // above, 1 ru = min(r_lim, max{r : lambda_r >= gamma trace(G_B)})
    const double *cscale = nullptr;
    double *evals = nullptr;
    int32_t crit = 0;
    double *scales = nullptr;  // out (mode 0, nullable): the h row scales sqrt(t_hat / (w q))
    double gamma = 0.0;
};
hipError_t launch_block_eig(const BlockEigArgs &a, hipStream_t st);
hipError_t launch_svd_merge(const SmallArgs &a, hipStream_t st);
hipError_t launch_chol_first_b(const SmallArgs *arr, int32_t count, int32_t pmax_max, hipStream_t st);
hipError_t launch_svd_merge_b(const SmallArgs *arr, int32_t count, int32_t pmax_max, hipStream_t st);

// One step of the reverse pass through merge t (adjoint of its truncated
// thin SVD, see k_adj_small).
struct AdjArgs {
    const double *Gext;    // Gram of [U_{t-1} | A(:, I_t) | Ubar_t] (ld pb)
    int32_t pb;
    const double *R;       // merge factor of merge t (ld pm)
    int32_t pm;
    const double *sig;     // Sigma_{t-1} (rs)
    const double *sbar_in; // adjoint of Sigma_t (rz)
    double *sbar_out;      // adjoint of Sigma_{t-1} (rs)
    void *Wt;              // out: ((p + rz) x p, ld pb, compute type)
    int32_t prec;
    double *ws;            // 12 pm^2 doubles (adj_wide_ws_doubles(pm) for wide merges)
    int32_t rs, g, rz;
    double eta;            // gap guard
    // row-sampled merge (vt set): P = blkdiag(Sigma, V_u), V_u = vt (g x ru, ld pm);
    // vfull / lam the full eigenbasis (g x g, ld pm) and eigenvalues of G = W^T W;
    // gbar receives the symmetric adjoint of G (g x g, ld pm)
    const double *vt = nullptr;
    int32_t ru = 0;
    const double *vfull = nullptr, *lam = nullptr;
    double *gbar = nullptr;
};
hipError_t launch_adj_small(const AdjArgs &a, hipStream_t st);
// The same step for merges wider than SMALL_LDS_P (p <= 160, column draws
// only): the eigen-decomposition of R R^T and R^-1 in one workgroup, then the
// small products one launch each over many workgroups.  Workspace (ws):
// adj_wide_ws_doubles(pm) doubles.
hipError_t launch_adj_wide(const AdjArgs &a, hipStream_t st);
__host__ __device__ constexpr size_t adj_wide_ws_doubles(int pm)
{
    return (size_t)11 * pm * pm + (size_t)3 * pm + BIG_INVIT_DOUBLES;
}
// Reverse pass of a row-sampled merge: G = W^T W (W = diag(s) A(rows, cols)),
// its full eigen-decomposition (descending) into vfull (g x g, ld pm) and lam,
// the first ru columns signed like vt; then, after the small adjoint,
// dA(rows, cols) += 2 diag(s)^2 A(rows, cols) Gbar.
struct AdjRowsArgs {
    const void *A;
    int32_t a_dtype;
    int64_t lda;
    const int32_t *cols, *rows;
    const double *scales;
    const double *vt;
    int32_t g, h, ru, pm;
    double *vfull, *lam;
    const double *gbar;
    void *dA;              // m x n gradient (compute type), ld ldd
    int64_t ldd;
    int32_t prec;
};
hipError_t launch_adj_rows_eig(const AdjRowsArgs &a, hipStream_t st);
hipError_t launch_adj_rows_update(const AdjRowsArgs &a, hipStream_t st);
// Batched reverse-pass launches (one entry per matrix, blockIdx selects it).
hipError_t launch_adj_small_b(const AdjArgs *arr, int32_t count, hipStream_t st);
struct ScatterArgs {       // one launch_gemm_tall_scatter of the reverse pass (P <= 64)
    GemmDesc d;
    const DevState *ds;
    int32_t which_in, which_out;
    const void *T;
    int32_t ldt;
    void *Yout;
    int32_t split;
    const int32_t *cmap;
    void *D;
    int64_t ldd;
    int32_t vec, nb;
};
hipError_t launch_gemm_tall_scatter_b(const ScatterArgs *arr, int32_t count, int32_t max_nb, int32_t pi_max,
                                      int32_t po_max, int32_t prec, hipStream_t st);
// Reverse pass of the loss gradient: its first part for one run, and the
// merge-chain part of many runs together (same stream; p + r <= 64).
pod_status loss_enqueue(pod_ctx *ctx, void *dA, double *loss);
pod_status reverse_merges_batch(pod_ctx *const *ctxs, int32_t count, void *const *dA, hipStream_t st);

struct ProjArgs {
    int32_t prec, a_dtype;
    int64_t m, n, lda;
    const void *U;        // basis m x r (compute type)
    const void *U1 = nullptr;      // with ds set: the basis is U1 when the merge count is odd
    const DevState *ds = nullptr;  // set: the live columns are ds->rs (<= r); nothing is done on the
                                   // first iteration or once the run has stopped
    const void *A;
    int32_t r;
    double *Bpart;        // partial B (nsplit x r x n)
    int32_t nsplit;
    double *B;            // r x n
};
hipError_t launch_project_partial(const ProjArgs &a, hipStream_t st);
hipError_t launch_project_reduce(const ProjArgs &a, hipStream_t st);
// ORT column weights of GET UPDATE from the second iteration: for j in S,
// rho_j = nu_j - |U^T a_j|^2 (B = U^T A, r x n, ld r; the live rows ds->rs),
// zero when at most floor_rel nu_j; zero outside S; rho = nu on the first
// iteration.
hipError_t launch_ort_resid(const double *nu, const double *B, int32_t r, int64_t n, const uint8_t *inS,
                            double floor_rel, const DevState *ds, double *rho, hipStream_t st);
struct RRArgs {
    const double *B;      // r x n
    int64_t n;
    int32_t r, k;
    double *part;         // scratch of the chunked sums: rr_part_doubles(n, r)
    double *GB;           // r x r
    double *UB;           // r x r (out, ld r)
    double *sig;          // r (out)
    void *Zc;             // U_B in compute type (r x k, ld r)
    double *ws;           // matrices of the kernel when r > 64 (2 r^2)
    int32_t prec;
    DevState *ds;
};
// Columns of B per workgroup of the chunked Rayleigh-Ritz sums, and the
// scratch they need (Gram partials, then the sigma partials).
constexpr int RR_CHUNK = 64;
inline size_t rr_part_doubles(int64_t n, int32_t r)
{
    return (size_t)((n + RR_CHUNK - 1) / RR_CHUNK) * (size_t)r * (size_t)r;
}
// G_B = B B^T (chunked partials, summed in chunk order), its
// eigen-decomposition, then Sigma_B(i) = |B^T U_B(:, i)| (chunked, in order).
hipError_t launch_rr_small(const RRArgs &a, hipStream_t st);
hipError_t launch_rr_v(const double *B, int64_t n, int32_t r, int32_t k, const double *UB, const double *sig,
                       int32_t prec, void *V, hipStream_t st);
hipError_t launch_sign_fix(int32_t prec, void *U, int64_t m, int32_t k, void *V, int64_t n, double *cv, int64_t *ci,
                           hipStream_t st);

}  // namespace pod

// pod_gemm.hip -- the tall-skinny contractions of the merge and of the final
// projection on gfx950 matrix cores (v_mfma_*_16x16x4 in FP64 or FP32).
//
//   gram partials   G = X^T X over row blocks     (CholeskyQR passes, Alg. 2)
//   tall transform  Y = X T                        (Q1 = X0 T1, U_new = Y Z2)
//   projection      B = U^T A                      (final step of Alg. 1)
//
// X is either the gathered block X0 = [U | A(:, I_c)] -- the sampled columns
// are streamed straight from A into LDS, never materialised -- or a
// contiguous m x p workspace.  Row blocks are staged through LDS in
// column-major order (rows contiguous) with an odd padded stride, so the
// 16 lanes that read one MFMA operand row hit distinct banks.  Partial sums
// are FP64 and reduced in a fixed order (deterministic results).
#include "pod_internal.h"

namespace pod {

constexpr int RB = 32;       // rows per LDS stage
constexpr int LDSR = RB + 1; // padded stride (elements) of one staged column

template <typename TC> struct SrcT {
    const TC *U;          // basis, ld = m
    const void *A;        // snapshot matrix
    int64_t lda;
    const int32_t *cols;
    const TC *Y;          // contiguous source, ld = m
    int32_t gather;
    int32_t a_f64;        // A stored in FP64
    int32_t rs;           // columns of U in X0
    int32_t guard;        // skip when the pending draw found S exhausted
};

template <typename TC>
__device__ __forceinline__ TC src_load(const SrcT<TC> &s, int64_t m, int c, int64_t row)
{
    if (!s.gather) return s.Y[(int64_t)c * m + row];
    if (c < s.rs) return s.U[(int64_t)c * m + row];
    const int64_t j = s.cols[c - s.rs];
    if (s.a_f64) return (TC)(reinterpret_cast<const double *>(s.A)[j * s.lda + row]);
    return (TC)(reinterpret_cast<const float *>(s.A)[j * s.lda + row]);
}

__device__ __forceinline__ int sel_count(const DevState *ds, int sel)
{
    if (sel >= 0) return sel;
    switch (sel) {
    case -1: return ds->p0;
    case -2: return ds->p;
    case -3: return ds->rnew;
    default: return ds->rs;
    }
}

// Stage rows [r0, r0 + RB) x columns [0, P) of the source into Xs (column c at
// Xs + c * LDSR); rows past m and columns past P are zero.
template <typename TC>
__device__ __forceinline__ void stage_rows(const SrcT<TC> &s, int64_t m, int64_t r0, int P, int PP, TC *Xs)
{
    for (int idx = threadIdx.x; idx < PP * RB; idx += 256) {
        const int c = idx / RB, rr = idx % RB;
        const int64_t row = r0 + rr;
        TC v = (TC)0;
        if (c < P && row < m) v = src_load<TC>(s, m, c, row);
        Xs[c * LDSR + rr] = v;
    }
}

// ---------------------------------------------------------------------------
// Partial Grams.  Workgroup b owns rows [m b / nblk, m (b+1) / nblk); each of
// its 4 waves accumulates a fixed set of the upper-triangular 16x16 tiles
// (I <= J) over the staged rows.  The tile is written (and mirrored) to
// part[b] (pmax x pmax, FP64); tiles outside P x P stay untouched and are
// ignored by the reduction.
// ---------------------------------------------------------------------------
constexpr int MAXPW = 3;  // tiles per wave for pmax <= 64 (10 tiles / 4 waves)

template <typename TC>
__global__ __launch_bounds__(256) void k_gram_partial(SrcT<TC> s, int64_t m, const DevState *ds, int which_p,
                                                      int pmax, double *__restrict__ part, int nblk)
{
    typedef typename Acc<TC>::type AccT;
    extern __shared__ unsigned char lds_raw[];
    TC *Xs = reinterpret_cast<TC *>(lds_raw);
    if (s.guard && ds->exhausted) return;
    const int P = sel_count(ds, which_p);
    s.rs = ds->rs;
    const int PP = (P + 15) & ~15;
    const int NT16 = PP / 16;
    const int npairs = NT16 * (NT16 + 1) / 2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t b = blockIdx.x;
    const int64_t r0 = (m * b) / nblk, r1 = (m * (b + 1)) / nblk;
    int tI[MAXPW], tJ[MAXPW];
#pragma unroll
    for (int q = 0; q < MAXPW; ++q) {
        int pr = wv + 4 * q, I = 0;
        tI[q] = -1;
        tJ[q] = -1;
        if (pr < npairs) {
            while (pr >= NT16 - I) {
                pr -= NT16 - I;
                ++I;
            }
            tI[q] = I;
            tJ[q] = I + pr;
        }
    }
    AccT acc[MAXPW];
#pragma unroll
    for (int q = 0; q < MAXPW; ++q) acc[q] = AccT{0, 0, 0, 0};
    for (int64_t rb = r0; rb < r1; rb += RB) {
        __syncthreads();
        // rows past r1 belong to the next workgroup: mask them
        const int64_t lim = (rb + RB < r1) ? rb + RB : r1;
        for (int idx = threadIdx.x; idx < PP * RB; idx += 256) {
            const int c = idx / RB, rr = idx % RB;
            const int64_t row = rb + rr;
            TC v = (TC)0;
            if (c < P && row < lim) v = src_load<TC>(s, m, c, row);
            Xs[c * LDSR + rr] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < MAXPW; ++q) {
            if (tI[q] >= 0) {
                const TC *xa = Xs + (tI[q] * 16 + (lane & 15)) * LDSR + (lane >> 4);
                const TC *xb = Xs + (tJ[q] * 16 + (lane & 15)) * LDSR + (lane >> 4);
#pragma unroll
                for (int k4 = 0; k4 < RB; k4 += 4) acc[q] = mfma16x16x4(xa[k4], xb[k4], acc[q]);
            }
        }
    }
    double *pb = part + b * (int64_t)pmax * pmax;
#pragma unroll
    for (int q = 0; q < MAXPW; ++q) {
        if (tI[q] < 0) continue;
        const int j = tJ[q] * 16 + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = tI[q] * 16 + acc_row<TC>(lane, v);
            const double x = (double)acc[q][v];
            if (tI[q] == tJ[q]) {
                if (i <= j) {
                    pb[i + (int64_t)j * pmax] = x;
                    pb[j + (int64_t)i * pmax] = x;
                }
            } else {
                pb[i + (int64_t)j * pmax] = x;
                pb[j + (int64_t)i * pmax] = x;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_gram_reduce(const double *__restrict__ part, int nblk, int pmax,
                                                     const DevState *ds, int which_p, double *__restrict__ G)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= pmax * pmax || ds->exhausted) return;
    const int P = sel_count(ds, which_p);
    const int i = idx % pmax, j = idx / pmax;
    double s = 0.0;
    if (i < P && j < P)
        for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * pmax * pmax + idx];
    G[idx] = s;
}

template <typename TC> static SrcT<TC> make_src(const GemmDesc &d)
{
    SrcT<TC> s;
    s.U = reinterpret_cast<const TC *>(d.U);
    s.A = d.A;
    s.lda = d.lda;
    s.cols = d.cols;
    s.Y = reinterpret_cast<const TC *>(d.Y);
    s.gather = d.gather;
    s.a_f64 = (d.a_dtype == POD_F64);
    s.rs = 0;
    s.guard = d.guard;
    return s;
}

hipError_t launch_gram_partial(const GemmDesc &d, const DevState *ds, int32_t which_p, int32_t pmax, double *part,
                               int32_t nblk, hipStream_t st)
{
    if (pmax > 64) return hipErrorInvalidValue;
    if (d.prec == POD_F64) {
        const size_t lds = (size_t)pmax * LDSR * sizeof(double);
        hipLaunchKernelGGL(k_gram_partial<double>, dim3(nblk), dim3(256), lds, st, make_src<double>(d), d.m, ds,
                           which_p, pmax, part, nblk);
    } else {
        const size_t lds = (size_t)pmax * LDSR * sizeof(float);
        hipLaunchKernelGGL(k_gram_partial<float>, dim3(nblk), dim3(256), lds, st, make_src<float>(d), d.m, ds,
                           which_p, pmax, part, nblk);
    }
    return hipGetLastError();
}

hipError_t launch_gram_reduce_sel(const double *part, int32_t nblk, int32_t pmax, const DevState *ds,
                                  int32_t which_p, double *G, hipStream_t st)
{
    hipLaunchKernelGGL(k_gram_reduce, dim3((pmax * pmax + 255) / 256), dim3(256), 0, st, part, nblk, pmax, ds,
                       which_p, G);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tall transform Y = X T (m x pout) with T pin x pout (ld ldt, compute type).
// Each workgroup stages RB rows of X and all of T in LDS and produces the
// RB x pout block of Y as Y^T tiles = T^T X^T, so that each lane's four
// results are consecutive-row entries of one output column.
// ---------------------------------------------------------------------------
template <typename TC>
__global__ __launch_bounds__(256) void k_gemm_tall(SrcT<TC> s, int64_t m, const DevState *ds, int sel_in,
                                                   int sel_out, int pmax_in, int pmax_out, const TC *__restrict__ T,
                                                   int ldt, TC *__restrict__ Yout)
{
    typedef typename Acc<TC>::type AccT;
    extern __shared__ unsigned char lds_raw[];
    if (s.guard && ds->exhausted) return;
    const int pin = sel_count(ds, sel_in), pout = sel_count(ds, sel_out);
    s.rs = ds->rs;
    const int PI = (pin + 15) & ~15, PO = (pout + 15) & ~15;
    TC *Xs = reinterpret_cast<TC *>(lds_raw);        // PI x LDSR
    TC *Ts = Xs + pmax_in * LDSR;                    // PI x PO, row k at Ts + k * PO
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * RB;
    for (int idx = threadIdx.x; idx < PI * PO; idx += 256) {
        const int k = idx / PO, j = idx % PO;
        Ts[idx] = (k < pin && j < pout) ? T[k + (int64_t)j * ldt] : (TC)0;
    }
    stage_rows<TC>(s, m, r0, pin, PI, Xs);
    __syncthreads();
    // tiles: (row block rbk in 0..RB/16) x (col block jc in 0..PO/16)
    const int ntile = (RB / 16) * (PO / 16);
    for (int tile = wv; tile < ntile; tile += 4) {
        const int rbk = tile % (RB / 16), jc = tile / (RB / 16);
        AccT acc = AccT{0, 0, 0, 0};
        const TC *ta = Ts + (lane >> 4) * PO + jc * 16 + (lane & 15);
        const TC *xb = Xs + (lane >> 4) * LDSR + rbk * 16 + (lane & 15);
        for (int k4 = 0; k4 < PI; k4 += 4) acc = mfma16x16x4(ta[k4 * PO], xb[k4 * LDSR], acc);
        const int64_t row = r0 + rbk * 16 + (lane & 15);
        if (row < m) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = jc * 16 + acc_row<TC>(lane, v);
                if (col < pout) Yout[(int64_t)col * m + row] = acc[v];
            }
        }
    }
}

hipError_t launch_gemm_tall(const GemmDesc &d, const DevState *ds, int32_t which_in, int32_t which_out,
                            int32_t pin_max, int32_t pout_max, const void *T, int32_t ldt, void *Yout,
                            hipStream_t st)
{
    if (pin_max > 64 || pout_max > 64) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)((d.m + RB - 1) / RB);
    const int PI = (pin_max + 15) & ~15, PO = (pout_max + 15) & ~15;
    if (d.prec == POD_F64) {
        const size_t lds = (size_t)(PI * LDSR + PI * PO) * sizeof(double);
        hipLaunchKernelGGL(k_gemm_tall<double>, dim3(nb), dim3(256), lds, st, make_src<double>(d), d.m, ds,
                           which_in, which_out, PI, PO, (const double *)T, ldt, (double *)Yout);
    } else {
        const size_t lds = (size_t)(PI * LDSR + PI * PO) * sizeof(float);
        hipLaunchKernelGGL(k_gemm_tall<float>, dim3(nb), dim3(256), lds, st, make_src<float>(d), d.m, ds,
                           which_in, which_out, PI, PO, (const float *)T, ldt, (float *)Yout);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Projection B = U^T A (r x n), one pass over A.  Workgroup (split, column
// block of 64) covers rows [m s / nsplit, m (s+1) / nsplit) of 64 columns of
// A; wave w owns 16 of those columns and all ceil(r/16) mode tiles.  The
// linear block index is remapped so that all column blocks of one row split
// run on the same XCD (workgroups are dealt round-robin to the 8 XCDs), where
// they share that split's rows of U in L2.
// ---------------------------------------------------------------------------
constexpr int PCB = 64;  // columns of A per workgroup

template <typename TC, typename TA>
__global__ __launch_bounds__(256) void k_project_partial(const TC *__restrict__ U, const TA *__restrict__ A,
                                                         int64_t m, int64_t n, int64_t lda, int r, int nsplit,
                                                         int ncb, double *__restrict__ Bpart)
{
    typedef typename Acc<TC>::type AccT;
    extern __shared__ unsigned char lds_raw[];
    const int RP = (r + 15) & ~15;
    TC *As = reinterpret_cast<TC *>(lds_raw);   // PCB x LDSR
    TC *Us = As + PCB * LDSR;                   // RP x LDSR
    // XCD-aware remap of the linear workgroup id
    const int total = nsplit * ncb;
    const int id = blockIdx.x;
    int sidx, cb;
    if (total % 8 == 0 && nsplit % 8 == 0) {
        const int xcd = id % 8, local = id / 8;   // local in [0, total/8)
        const int spx = nsplit / 8;               // splits per XCD
        sidx = xcd * spx + local / ncb;
        cb = local % ncb;
    } else {
        sidx = id / ncb;
        cb = id % ncb;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r0 = (m * sidx) / nsplit, r1 = (m * (sidx + 1)) / nsplit;
    const int64_t c0 = (int64_t)cb * PCB;
    constexpr int MT = 4;  // r <= 64
    AccT acc[MT];
#pragma unroll
    for (int q = 0; q < MT; ++q) acc[q] = AccT{0, 0, 0, 0};
    for (int64_t rb = r0; rb < r1; rb += RB) {
        __syncthreads();
        const int64_t lim = (rb + RB < r1) ? rb + RB : r1;
        for (int idx = threadIdx.x; idx < PCB * RB; idx += 256) {
            const int c = idx / RB, rr = idx % RB;
            const int64_t row = rb + rr, col = c0 + c;
            As[c * LDSR + rr] = (row < lim && col < n) ? (TC)A[col * lda + row] : (TC)0;
        }
        for (int idx = threadIdx.x; idx < RP * RB; idx += 256) {
            const int c = idx / RB, rr = idx % RB;
            const int64_t row = rb + rr;
            Us[c * LDSR + rr] = (row < lim && c < r) ? U[(int64_t)c * m + row] : (TC)0;
        }
        __syncthreads();
        const TC *xb = As + (wv * 16 + (lane & 15)) * LDSR + (lane >> 4);
#pragma unroll
        for (int q = 0; q < MT; ++q) {
            if (q * 16 < RP) {
                const TC *ua = Us + (q * 16 + (lane & 15)) * LDSR + (lane >> 4);
#pragma unroll
                for (int k4 = 0; k4 < RB; k4 += 4) acc[q] = mfma16x16x4(ua[k4], xb[k4], acc[q]);
            }
        }
    }
    const int64_t col = c0 + wv * 16 + (lane & 15);
    if (col < n) {
#pragma unroll
        for (int q = 0; q < MT; ++q) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int mode = q * 16 + acc_row<TC>(lane, v);
                if (mode < r) Bpart[(int64_t)sidx * r * n + col * r + mode] = (double)acc[q][v];
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_project_reduce(const double *__restrict__ Bpart, int64_t rn, int nsplit,
                                                        double *__restrict__ B)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= rn) return;
    double s = 0.0;
    for (int q = 0; q < nsplit; ++q) s += Bpart[(int64_t)q * rn + idx];
    B[idx] = s;
}

hipError_t launch_project_partial(const ProjArgs &a, hipStream_t st)
{
    if (a.r > 64) return hipErrorInvalidValue;
    const int ncb = (int)((a.n + PCB - 1) / PCB);
    const int RP = (a.r + 15) & ~15;
    const unsigned total = (unsigned)(a.nsplit * ncb);
    if (a.prec == POD_F64) {
        const size_t lds = (size_t)(PCB + RP) * LDSR * sizeof(double);
        if (a.a_dtype == POD_F64)
            hipLaunchKernelGGL((k_project_partial<double, double>), dim3(total), dim3(256), lds, st,
                               (const double *)a.U, (const double *)a.A, a.m, a.n, a.lda, a.r, a.nsplit, ncb,
                               a.Bpart);
        else
            hipLaunchKernelGGL((k_project_partial<double, float>), dim3(total), dim3(256), lds, st,
                               (const double *)a.U, (const float *)a.A, a.m, a.n, a.lda, a.r, a.nsplit, ncb,
                               a.Bpart);
    } else {
        const size_t lds = (size_t)(PCB + RP) * LDSR * sizeof(float);
        if (a.a_dtype == POD_F64) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_project_partial<float, float>), dim3(total), dim3(256), lds, st, (const float *)a.U,
                           (const float *)a.A, a.m, a.n, a.lda, a.r, a.nsplit, ncb, a.Bpart);
    }
    return hipGetLastError();
}

hipError_t launch_project_reduce(const ProjArgs &a, hipStream_t st)
{
    const int64_t rn = (int64_t)a.r * a.n;
    hipLaunchKernelGGL(k_project_reduce, dim3((unsigned)((rn + 255) / 256)), dim3(256), 0, st, a.Bpart, rn,
                       a.nsplit, a.B);
    return hipGetLastError();
}

}  // namespace pod

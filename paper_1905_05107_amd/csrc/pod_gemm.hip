// pod_gemm.hip -- the tall-skinny contractions of the merge and of the final
// projection on gfx950 matrix cores (v_mfma_*_16x16x4 in FP64 or FP32).
//
//   gram partials   G = X^T X over row blocks     (CholeskyQR passes, Alg. 2)
//   tall transform  Y = X T                        (Q1 = X0 T1, U_new = Y Z2)
//   projection      B = U^T A                      (final step of Alg. 1)
//
// X is either the gathered block X0 = [U | A(:, I_c)] -- the sampled columns
// are streamed straight from A into LDS, never materialised -- or a
// contiguous m x p workspace.  Rows are staged through LDS in 32-row stages,
// column-major with an odd padded stride (the 16 lanes that read one MFMA
// operand row hit distinct banks).  Stages are loaded as 16-byte vectors
// into registers one stage ahead of the MFMA work on the current stage.
// Partial sums are FP64 and reduced in a fixed order (deterministic results).
#include <algorithm>

#include "pod_internal.h"

namespace pod {

constexpr int RB = 32;       // rows per LDS stage
constexpr int LDSR = RB + 1; // padded stride (elements) of one staged column
constexpr int GRP = RB / 4;  // 4-row groups per staged column
constexpr int TALL_ST = 8;                 // row stages per workgroup of the tall transforms
constexpr int TALL_ST_WIDE = 16;           // the same for inputs wider than 64 (T staged once per 16 stages)
constexpr size_t TALL_T_LDS = 112 * 1024;  // largest T staged in LDS
constexpr int TALL_DYN_LDS = 160 * 1024;   // dynamic LDS limit of the tall kernels

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const f64x2 gf64x2;

template <typename TC> struct SrcT {
    const TC *U;          // basis, ld = m
    const TC *U1;         // second basis buffer (nullable): used when the merge count is odd
    const void *A;        // snapshot matrix
    int64_t lda;
    const int32_t *cols;
    const TC *Y;          // contiguous source, ld = m
    int32_t gather;
    int32_t a_f64;        // A stored in FP64
    int32_t rs;           // columns of U in X0
    int32_t guard;        // skip when the pending draw found S exhausted
    const TC *Z;          // third block of a gathered source (nullable)
    int32_t g;            // columns of the A block when Z is set
};

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

// Address and storage type of one source column.
struct ColPtr {
    const void *p;
    int f64;   // element is double
};
template <typename TC> __device__ __forceinline__ ColPtr col_ptr(const SrcT<TC> &s, int64_t m, int c)
{
    ColPtr r;
    if (!s.gather) {
        r.p = s.Y + (int64_t)c * m;
        r.f64 = sizeof(TC) == 8;
    } else if (c < s.rs) {
        r.p = s.U + (int64_t)c * m;
        r.f64 = sizeof(TC) == 8;
    } else if (s.Z && c >= s.rs + s.g) {
        r.p = s.Z + (int64_t)(c - s.rs - s.g) * m;
        r.f64 = sizeof(TC) == 8;
    } else {
        const int64_t j = s.cols[c - s.rs];
        if (s.a_f64) {
            r.p = reinterpret_cast<const double *>(s.A) + j * s.lda;
            r.f64 = 1;
        } else {
            r.p = reinterpret_cast<const float *>(s.A) + j * s.lda;
            r.f64 = 0;
        }
    }
    return r;
}

// Four consecutive rows [row, row + 4) of a column, converted to TC; vector
// loads when the group is in range and the column is 16-byte aligned.
template <typename TC>
__device__ __forceinline__ void load4(const ColPtr &cp, int64_t row, int64_t lim, bool vec, TC out[4])
{
    if (cp.f64) {
        const double *p = reinterpret_cast<const double *>(cp.p) + row;
        if (vec && row + 4 <= lim) {
            const f64x2 a = *reinterpret_cast<const f64x2 *>(p);
            const f64x2 b = *reinterpret_cast<const f64x2 *>(p + 2);
            out[0] = (TC)a[0];
            out[1] = (TC)a[1];
            out[2] = (TC)b[0];
            out[3] = (TC)b[1];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) out[q] = (row + q < lim) ? (TC)p[q] : (TC)0;
        }
    } else {
        const float *p = reinterpret_cast<const float *>(cp.p) + row;
        if (vec && row + 4 <= lim) {
            const f32x4 a = *reinterpret_cast<const f32x4 *>(p);
            out[0] = (TC)a[0];
            out[1] = (TC)a[1];
            out[2] = (TC)a[2];
            out[3] = (TC)a[3];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) out[q] = (row + q < lim) ? (TC)p[q] : (TC)0;
        }
    }
}

// A register-held stage: item `it` of thread t is (column, 4-row group)
// = ((t + 256 it) / GRP, (t + 256 it) % GRP).  prepare() fixes the column
// start of every item once (the columns do not change between stages); when
// every column is 16-byte aligned, a full stage is then loaded with plain
// vector loads (FP32 columns of A widened to FP64 on the FP64 path), so the
// loads of the stages in flight are not waited for until their store.  Items
// beyond the P columns point at column 0 and are replaced by zeros at the
// store.
template <typename TC, int ITEMS, int NTH = 256> struct Stage {
    TC v[ITEMS][4];
    const TC *base[ITEMS];
    uint32_t f32col;   // bit it: item it reads an FP32 column while TC is double
    bool fast;

    __device__ __forceinline__ void prepare(const SrcT<TC> &s, int64_t m, int P, bool vec)
    {
        fast = vec;
        f32col = 0;
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int idx = threadIdx.x + NTH * it;
            const int c = idx / GRP;
            const ColPtr cp = col_ptr<TC>(s, m, (c < P) ? c : 0);
            base[it] = reinterpret_cast<const TC *>(cp.p);
            if (sizeof(TC) == 8 && !cp.f64) f32col |= 1u << it;
        }
    }

    // a full stage on the fast path (prepare() set fast, rb + RB <= m): vector
    // loads only.  On the FP64 path every item issues the same two 16-byte
    // loads with no branch (an FP32 item's second one repeats its first), and
    // an FP32 item's four floats stay as raw bits in v[it][0..1] until
    // store_all widens them: a value used inside a divergent branch would be
    // waited for there, and with it every load issued before it, the next
    // stages' prefetches included.
    __device__ __forceinline__ void load_full(int64_t rb)
    {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int g = (threadIdx.x + NTH * it) % GRP;
            const TC *q = base[it] + rb + 4 * g;
            if (sizeof(TC) == 8) {
                const bool f32 = (f32col >> it) & 1u;
                const char *b = reinterpret_cast<const char *>(base[it]);
                const char *q0 = b + (f32 ? 4 : 8) * (rb + 4 * g);
                const char *q1 = f32 ? q0 : q0 + 16;
                const f64x2 a = *reinterpret_cast<const gf64x2 *>((uintptr_t)q0);
                const f64x2 c = *reinterpret_cast<const gf64x2 *>((uintptr_t)q1);
                v[it][0] = a[0];
                v[it][1] = a[1];
                v[it][2] = c[0];
                v[it][3] = c[1];
            } else if (sizeof(TC) == 4) {
                const f32x4 a = *reinterpret_cast<const f32x4 *>(q);
                v[it][0] = a[0];
                v[it][1] = a[1];
                v[it][2] = a[2];
                v[it][3] = a[3];
            } else {
                const f64x2 a = *reinterpret_cast<const f64x2 *>(q);
                const f64x2 b = *reinterpret_cast<const f64x2 *>(q + 2);
                v[it][0] = a[0];
                v[it][1] = a[1];
                v[it][2] = b[0];
                v[it][3] = b[1];
            }
        }
    }

    __device__ __forceinline__ void load(const SrcT<TC> &s, int64_t m, int64_t rb, int P, bool vec)
    {
        if (fast && rb + RB <= m) {
            load_full(rb);
            return;
        }
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int idx = threadIdx.x + NTH * it;
            const int c = idx / GRP, g = idx % GRP;
            if (c < P) {
                const ColPtr cp = col_ptr<TC>(s, m, c);
                load4<TC>(cp, rb + 4 * g, m, vec, v[it]);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) v[it][q] = (TC)0;
            }
        }
    }
    // P: live columns (items beyond are written as zeros), PP: padded width
    __device__ __forceinline__ void store(TC *Xs, int PP, int P) const
    {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int idx = threadIdx.x + NTH * it;
            const int c = idx / GRP, g = idx % GRP;
            if (c < PP) {
                const bool live = c < P;
#pragma unroll
                for (int q = 0; q < 4; ++q) Xs[c * LDSR + 4 * g + q] = live ? v[it][q] : (TC)0;
            }
        }
    }
    // every item written (the LDS stage holds all ITEMS * NTH / GRP columns):
    // no branch between the loads and the stores
    __device__ __forceinline__ void store_all(TC *Xs, int P) const
    {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int idx = threadIdx.x + NTH * it;
            const int c = idx / GRP, g = idx % GRP;
            const bool live = c < P;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                TC x = v[it][q];
                if (sizeof(TC) == 8) {
                    // (an FP32 item: float q in half q & 1 of v[it][q >> 1])
                    const uint64_t w = (uint64_t)__double_as_longlong((double)v[it][q >> 1]);
                    const float f = __uint_as_float((uint32_t)((q & 1) ? (w >> 32) : w));
                    x = ((f32col >> it) & 1u) ? (TC)f : x;
                }
                Xs[c * LDSR + 4 * g + q] = live ? x : (TC)0;
            }
        }
    }
};

// 16-byte loads are legal for every column of the source.
template <typename TC> static bool vec_ok(const SrcT<TC> &s, int64_t m)
{
    const size_t esz = sizeof(TC);
    bool ok = ((m * esz) % 16 == 0);
    if (s.gather) {
        ok = ok && ((uintptr_t)s.U % 16 == 0) && ((uintptr_t)s.U1 % 16 == 0) && ((uintptr_t)s.Z % 16 == 0);
        const size_t ae = s.a_f64 ? 8 : 4;
        ok = ok && ((uintptr_t)s.A % 16 == 0) && ((s.lda * ae) % 16 == 0);
    } else {
        ok = ok && ((uintptr_t)s.Y % 16 == 0);
    }
    return ok;
}

template <typename TC> __host__ __device__ SrcT<TC> make_src(const GemmDesc &d)
{
    SrcT<TC> s;
    s.U = reinterpret_cast<const TC *>(d.U);
    s.U1 = reinterpret_cast<const TC *>(d.U1);
    s.Z = reinterpret_cast<const TC *>(d.Z);
    s.g = 0;
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

// ---------------------------------------------------------------------------
// Partial Grams.  Workgroup b owns stages [ns b / nblk, ns (b+1) / nblk) of
// the ns = ceil(m / 32) row stages; each of its NWV waves accumulates a fixed
// set of the upper-triangular 16x16 tiles (I <= J).  The tile is written (and
// mirrored) to part[b] (pmax x pmax, FP64); the reduction reads only P x P.
// ---------------------------------------------------------------------------
// Width classes of the staged kernels: pmax <= 64 (a stage is 64 columns x 8
// groups = 2 items per thread of 256) and pmax <= 160 (5 items per thread of
// 256).  The wide Gram runs 8 waves per workgroup (55 tiles: 7 per wave; 3
// items per thread of 512), whose accumulator and stage sets leave room for
// two waves per SIMD.
constexpr int ITEMS64 = 2;
constexpr int ITEMS160 = 5;
constexpr int MAXPW160_8 = 7, ITEMS160_8 = 3;
constexpr int PMAX_WIDE = 160;
// The reverse pass's Gram of [U | A(:, I) | Ubar] and its transform from that
// block reach p + r <= 208 columns (13 tiles: 91 tile pairs, 12 per wave of 8;
// 4 items per thread of 512 stage 256 columns); its transform runs on the
// register-operand tall kernel (scatter mode, 80-column groups of T in LDS).
constexpr int PMAX_ADJ = 208;
constexpr int MAXPW208_8 = 12, ITEMS208_8 = 4;

template <typename TC, int MAXPW, int ITEMS, int NWV = 4>
__device__ __forceinline__ void gram_partial_body(SrcT<TC> s, int64_t m, const DevState *ds, int which_p, int pmax,
                                                  double *__restrict__ part, int nblk, int vec, int bid)
{
    typedef typename Acc<TC>::type AccT;
    extern __shared__ unsigned char lds_raw[];
    TC *Xs = reinterpret_cast<TC *>(lds_raw);
    if (s.guard && merge_halted(ds)) return;
    const int P = sel_count(ds, which_p);
    s.rs = ds->rs;
    s.g = ds->g;
    if (s.U1 && (ds->it & 1)) s.U = s.U1;
    const int PP = (P + 15) & ~15;
    const int NT16 = PP / 16;
    const int npairs = NT16 * (NT16 + 1) / 2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nst = (m + RB - 1) / RB;
    const int64_t s0 = (nst * bid) / nblk, s1 = (nst * (bid + 1)) / nblk;
    int tI[MAXPW], tJ[MAXPW];
#pragma unroll
    for (int q = 0; q < MAXPW; ++q) {
        int pr = wv + NWV * q, I = 0;
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
    // two register stages in flight: the loads of stages sg+1 and sg+2 overlap
    // the MFMA work on stage sg
    // tiles in groups of four whose products alternate (independent chains:
    // a product that waits for the one before it on the same tile stalls the
    // matrix core); each tile still sums its k in order.  A wave's live tiles
    // are a prefix of its slots.
    auto compute = [&]() {
#pragma unroll
        for (int q0 = 0; q0 < MAXPW; q0 += 4) {
            if (q0 + 3 < MAXPW && tI[q0 + 3] >= 0) {
                const TC *xa[4], *xb[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    xa[u] = Xs + (tI[q0 + u] * 16 + (lane & 15)) * LDSR + (lane >> 4);
                    xb[u] = Xs + (tJ[q0 + u] * 16 + (lane & 15)) * LDSR + (lane >> 4);
                }
#pragma unroll
                for (int k4 = 0; k4 < RB; k4 += 4)
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc[q0 + u] = mfma16x16x4(xa[u][k4], xb[u][k4], acc[q0 + u]);
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int q = q0 + u;
                    if (q < MAXPW && tI[q] >= 0) {
                        const TC *xa = Xs + (tI[q] * 16 + (lane & 15)) * LDSR + (lane >> 4);
                        const TC *xb = Xs + (tJ[q] * 16 + (lane & 15)) * LDSR + (lane >> 4);
#pragma unroll
                        for (int k4 = 0; k4 < RB; k4 += 4) acc[q] = mfma16x16x4(xa[k4], xb[k4], acc[q]);
                    }
                }
            }
        }
    };
    Stage<TC, ITEMS, 64 * NWV> sa, sb;
    sa.prepare(s, m, P, vec);
    sb.fast = sa.fast;
    sb.f32col = sa.f32col;
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) sb.base[it] = sa.base[it];
    // full stages [s0, e) on the fast path: two register stages in flight (the
    // loads of stages sg+1 and sg+2 overlap the MFMA work on stage sg; the
    // prefetch index is clamped so every iteration issues the same loads)
    const int64_t full_end = m / RB;   // stages entirely inside [0, m)
    const int64_t e = sa.fast ? ((s1 < full_end) ? s1 : ((full_end > s0) ? full_end : s0)) : s0;
    if (e > s0) {
        const int64_t last = e - 1;
        sa.load_full(s0 * RB);
        sb.load_full(((s0 + 1 < last) ? s0 + 1 : last) * RB);
        int64_t sg = s0;
        for (; sg + 1 < e; sg += 2) {
            __syncthreads();
            sa.store_all(Xs, P);
            __syncthreads();
            sa.load_full(((sg + 2 < last) ? sg + 2 : last) * RB);
            compute();
            __syncthreads();
            sb.store_all(Xs, P);
            __syncthreads();
            sb.load_full(((sg + 3 < last) ? sg + 3 : last) * RB);
            compute();
        }
        if (sg < e) {
            __syncthreads();
            sa.store_all(Xs, P);
            __syncthreads();
            compute();
        }
    }
    // remaining stages (a partial last stage, or every stage off the fast path)
    for (int64_t sg = e; sg < s1; ++sg) {
        sa.load(s, m, sg * RB, P, vec);
        __syncthreads();
        sa.store(Xs, PP, P);
        __syncthreads();
        compute();
    }
    double *pb = part + (int64_t)bid * pmax * pmax;
#pragma unroll
    for (int q = 0; q < MAXPW; ++q) {
        if (tI[q] < 0) continue;
        const int j = tJ[q] * 16 + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = tI[q] * 16 + acc_row<TC>(lane, v);
            const double x = (double)acc[q][v];
            if (tI[q] < tJ[q] || i <= j) {
                pb[i + (int64_t)j * pmax] = x;
                pb[j + (int64_t)i * pmax] = x;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Partial Grams for P <= 64 straight from registers.  Lane (i, k) =
// (l % 16, l / 16) of a wave loads rows 4k .. 4k+3 of a 16-row group, as one
// 16-byte vector per column tile t, from column 16 t + i.  MFMA step j takes
// row 4k + j as the k-th row of a 4-row slice (a Gram sums over its rows in
// any order), so the A and B operands of tile (I, J) are the lanes' own values
// of tiles I and J: no LDS staging and no barrier in the row loop.  Waves take
// interleaved groups with two groups loaded ahead; the four wave partials of
// a workgroup are summed in FP64 through LDS in a fixed order and written as
// the tile pairs I <= J of part[b] (both triangles).
// ---------------------------------------------------------------------------
constexpr int GD_LDS = 4 * 5 * 4 * 64 * 8;   // wave partials of five tile pairs, FP64
constexpr int GD_NB = 3;                      // register groups per wave

template <typename TC> struct Vec4;
template <> struct Vec4<float> {
    __device__ static void load(const float *p, float v[4])
    {
        const f32x4 a = *reinterpret_cast<const f32x4 *>(p);
        v[0] = a[0];
        v[1] = a[1];
        v[2] = a[2];
        v[3] = a[3];
    }
};
template <> struct Vec4<double> {
    __device__ static void load(const double *p, double v[4])
    {
        const f64x2 a = *reinterpret_cast<const f64x2 *>(p);
        const f64x2 b = *reinterpret_cast<const f64x2 *>(p + 2);
        v[0] = a[0];
        v[1] = a[1];
        v[2] = b[0];
        v[3] = b[1];
    }
};

template <typename TC, int NWV>
__device__ __forceinline__ void gram_direct_body(SrcT<TC> s, int64_t m, const DevState *ds, int which_p, int pmax,
                                                 double *__restrict__ part, int nblk, int vec, int bid)
{
    typedef typename Acc<TC>::type AccT;
    extern __shared__ unsigned char lds_raw[];
    double *red = reinterpret_cast<double *>(lds_raw);
    if (s.guard && merge_halted(ds)) return;
    const int P = sel_count(ds, which_p);
    s.rs = ds->rs;
    s.g = ds->g;
    if (s.U1 && (ds->it & 1)) s.U = s.U1;
    const int NT = (P + 15) >> 4;   // column tiles, <= 4
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ci = lane & 15, kr = 4 * (lane >> 4);
    // the lane's column of every tile (tiles past P read column 0, zeroed below)
    ColPtr cp[4];
    bool live[4];
    bool same = true;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int c = 16 * t + ci;
        live[t] = c < P;
        cp[t] = col_ptr<TC>(s, m, live[t] ? c : 0);
        same = same && (cp[t].f64 == (sizeof(TC) == 8 ? 1 : 0));
    }
    // fast path: every column in the compute type and 16-byte aligned (uniform)
    const bool fast = vec && __all(same);
    // groups of 16 rows, grid-strided over the waves: group W + i NW for wave W
    // (at each step the grid reads one contiguous span of every column)
    const int64_t ngr = (m + 15) >> 4, nfull = m >> 4;   // groups; those entirely inside [0, m)
    const int64_t W = (int64_t)bid * NWV + wv, NW = (int64_t)nblk * NWV;
    AccT acc[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) acc[q] = AccT{0, 0, 0, 0};
    auto mma = [&](const TC (&v)[4][4]) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int q = 0;
#pragma unroll
            for (int I = 0; I < 4; ++I)
#pragma unroll
                for (int J = I; J < 4; ++J, ++q)
                    if (J < NT) acc[q] = mfma16x16x4(v[I][j], v[J][j], acc[q]);
        }
    };
    auto load_fast = [&](int64_t gr, TC (&v)[4][4]) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            Vec4<TC>::load(reinterpret_cast<const TC *>(cp[t].p) + gr * 16 + kr, v[t]);
#pragma unroll
            for (int q = 0; q < 4; ++q) v[t][q] = live[t] ? v[t][q] : (TC)0;
        }
    };
    int64_t gstart = W;
    if (fast && gstart < nfull) {
        // GD_NB register groups: loads GD_NB - 1 groups ahead (indices clamped to
        // the wave's last full group, so every iteration issues the same loads)
        const int64_t lastg = gstart + ((nfull - 1 - gstart) / NW) * NW;
        TC vr[GD_NB][4][4];
#pragma unroll
        for (int b = 0; b < GD_NB - 1; ++b) load_fast((gstart + NW * b < lastg) ? gstart + NW * b : lastg, vr[b]);
        // (the loads are issued outside the branch that skips the products of
        // groups past the wave's last: a load inside a branch is waited for
        // where the branch ends, and the prefetch with it)
        for (int64_t gr = gstart;; gr += NW * GD_NB) {
#pragma unroll
            for (int b = 0; b < GD_NB; ++b) {
                const int64_t ld = gr + NW * (b + GD_NB - 1);
                load_fast((ld < lastg) ? ld : lastg, vr[(b + GD_NB - 1) % GD_NB]);
                if (gr + NW * b <= lastg) mma(vr[b]);
            }
            if (gr + NW * GD_NB > lastg) break;
        }
        gstart = lastg + NW;   // the wave's groups past the full ones
    }
    // the rest (a partial last group, or every group off the fast path)
    for (int64_t gr = gstart; gr < ngr; gr += NW) {
        TC v[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            load4<TC>(cp[t], gr * 16 + kr, m, vec, v[t]);
#pragma unroll
            for (int q = 0; q < 4; ++q) v[t][q] = live[t] ? v[t][q] : (TC)0;
        }
        mma(v);
    }
    // sum the wave partials in FP64 (waves in order), CP tile pairs at a time
    // (CP = 5 for 4 waves, 2 for 8: at most 40 KiB of LDS)
    constexpr int CP = (NWV == 4) ? 5 : 2;
    double *pb = part + (int64_t)bid * pmax * pmax;
#pragma unroll
    for (int half = 0; half < 10 / CP; ++half) {
        if (half) __syncthreads();
#pragma unroll
        for (int q5 = 0; q5 < CP; ++q5)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[((wv * CP + q5) * 4 + v) * 64 + lane] = (double)acc[CP * half + q5][v];
        __syncthreads();
        for (int o = threadIdx.x; o < CP * 256; o += NWV * 64) {
            const int q5 = o >> 8, v = (o >> 6) & 3, ln = o & 63;
            const int q = CP * half + q5;
            // pair q -> (I, J), I <= J
            const int I = (q < 4) ? 0 : (q < 7) ? 1 : (q < 9) ? 2 : 3;
            const int J = I + q - ((q < 4) ? 0 : (q < 7) ? 4 : (q < 9) ? 7 : 9);
            if (J >= NT) continue;
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < NWV; ++w) sum += red[((w * CP + q5) * 4 + v) * 64 + ln];
            const int i = 16 * I + acc_row<TC>(ln, v), j = 16 * J + (ln & 15);
            if (I < J || i <= j) {
                pb[i + (int64_t)j * pmax] = sum;
                pb[j + (int64_t)i * pmax] = sum;
            }
        }
    }
}

template <typename TC, int MAXPW, int ITEMS, int NWV>
__global__ __launch_bounds__(64 * NWV) void k_gram_partial(SrcT<TC> s, int64_t m, const DevState *ds, int which_p,
                                                      int pmax, double *__restrict__ part, int nblk, int vec)
{
    gram_partial_body<TC, MAXPW, ITEMS, NWV>(s, m, ds, which_p, pmax, part, nblk, vec, blockIdx.x);
}

// 8 waves per workgroup (two per SIMD at one workgroup per CU).
template <typename TC>
__global__ __launch_bounds__(512) void k_gram_direct(SrcT<TC> s, int64_t m, const DevState *ds, int which_p, int pmax,
                                                     double *__restrict__ part, int nblk, int vec)
{
    gram_direct_body<TC, 8>(s, m, ds, which_p, pmax, part, nblk, vec, blockIdx.x);
}

// Batched (P <= 64): matrix blockIdx.y, its own block count; stopped matrices skipped.
template <typename TC>
__global__ __launch_bounds__(512) void k_gram_direct_b(const GramArgs *__restrict__ arr)
{
    const GramArgs &a = arr[blockIdx.y];
    if ((int)blockIdx.x >= a.nblk || a.ds->done) return;
    gram_direct_body<TC, 8>(make_src<TC>(a.d), a.d.m, a.ds, a.which_p, a.pmax, a.part, a.nblk, a.vec, blockIdx.x);
}

// Fixed-order reduction of the partial Grams: workgroup w owns 64 entries;
// its 4 waves each add a contiguous quarter of the partials in order, and the
// four quarter sums are added in order.
// G = sum of the nblk partials, 64 entries per workgroup, the partials split
// over GR_W waves (memory parallelism), wave sums combined in wave order
// (deterministic).  Only the upper triangle is summed; it is mirrored.
constexpr int GR_W = 16;
__device__ __forceinline__ void gram_reduce_body(const double *__restrict__ part, int nblk, int pmax,
                                                 const DevState *ds, int which_p, double *__restrict__ G, int bid)
{
    __shared__ double sq[GR_W][64];
    if (merge_halted(ds)) return;
    const int P = sel_count(ds, which_p);
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int idx = bid * 64 + lane;
    const int i = idx % pmax, j = idx / pmax;
    const bool live = idx < pmax * pmax && i < P && j < P && i <= j;
    const int b0 = (nblk * wv) / GR_W, b1 = (nblk * (wv + 1)) / GR_W;
    double s = 0.0;
    if (live) {
        // four independent accumulators keep four loads in flight; fixed order
        const int64_t st = (int64_t)pmax * pmax;
        const double *pp = part + idx;
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        int b = b0;
        for (; b + 4 <= b1; b += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] += pp[(int64_t)(b + u) * st];
        }
        for (; b < b1; ++b) a[0] += pp[(int64_t)b * st];
        s = (a[0] + a[1]) + (a[2] + a[3]);
    }
    sq[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && idx < pmax * pmax && i <= j) {
        double g = 0.0;
        if (live) {
#pragma unroll
            for (int w = 0; w < GR_W; ++w) g += sq[w][lane];
        }
        G[idx] = g;
        G[j + (int64_t)i * pmax] = g;
    }
}

__global__ __launch_bounds__(64 * GR_W) void k_gram_reduce(const double *__restrict__ part, int nblk, int pmax,
                                                     const DevState *ds, int which_p, double *__restrict__ G)
{
    gram_reduce_body(part, nblk, pmax, ds, which_p, G, blockIdx.x);
}

__global__ __launch_bounds__(64 * GR_W) void k_gram_reduce_b(const GramArgs *__restrict__ arr)
{
    const GramArgs &a = arr[blockIdx.y];
    if ((int)blockIdx.x * 64 >= a.pmax * a.pmax || a.ds->done) return;
    gram_reduce_body(a.part, a.nblk, a.pmax, a.ds, a.which_p, a.G, blockIdx.x);
}


// ---------------------------------------------------------------------------
// BF16 matrix cores with a three-term split (POD_BF16_REFINE).  Each FP32
// operand x is written as x = h + d + l with h = bf16(x), d = bf16(x - h),
// l = bf16(x - h - d) (round to nearest even; both differences are exact in
// FP32, and the three terms carry the 24 significand bits of x).  A product
// x y is taken as hh' + hd' + dh' + hl' + lh' + dd' on
// v_mfma_f32_16x16x32_bf16: each bf16 product is exact and the sum is
// accumulated in FP32; the dropped terms dl' + ld' + ll' are below 2^-23 |x y|,
// the size of one FP32 rounding.  The Grams, Q1 = X0 T1 and U_new = Q1 Z2 thus
// keep FP32 accuracy (a plain BF16 rounding of X0 would move the span of the
// merge by about 2^-9 sigma_1 / gap) on 6/16 of the FP32 matrix-core cycles.
//
// Operands of the 16x16x32 instruction: lane l supplies A[l % 16][8 (l / 16) + t]
// and B[8 (l / 16) + t][l % 16], t = 0..7, as eight packed bf16; its four
// results are D[4 (l / 16) + v][l % 16] (acc_row<float>).
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split3(float x, __bf16 &h, __bf16 &d, __bf16 &l)
{
    h = (__bf16)x;
    const float r1 = x - (float)h;
    d = (__bf16)r1;
    l = (__bf16)(r1 - (float)d);
}

__device__ __forceinline__ v4f mfma_bf16(const bf16x8 &a, const bf16x8 &b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// c += (ah + ad + al)(bh + bd + bl) without the three smallest cross terms
__device__ __forceinline__ v4f mfma_split(const bf16x8 &ah, const bf16x8 &ad, const bf16x8 &al, const bf16x8 &bh,
                                          const bf16x8 &bd, const bf16x8 &bl, v4f c)
{
    c = mfma_bf16(ad, bd, c);
    c = mfma_bf16(al, bh, c);
    c = mfma_bf16(ah, bl, c);
    c = mfma_bf16(ad, bh, c);
    c = mfma_bf16(ah, bd, c);
    return mfma_bf16(ah, bh, c);
}

// tile pairs per round of the final LDS reduction, and that reduction's LDS
// (4 waves x CH pairs x 256 FP64 values, within the 64 KiB default)
constexpr int gram_bf16_direct_ch(int bt) { return (bt * (bt + 1) / 2 + 7) / 8; }
constexpr size_t gram_bf16_direct_lds(int bt) { return (size_t)4 * gram_bf16_direct_ch(bt) * 4 * 64 * sizeof(double); }

// Partial Grams on the split operands straight from registers (the layout of
// gram_direct_body with 32-row groups): lane (i, k) = (l % 16, l / 16) of a
// wave loads rows 8k .. 8k+7 of a 32-row group from column 16 t + i of every
// column tile t, splits them into three bf16x8 terms, and MFMA step (I, J)
// takes the lane's own terms of tiles I and J -- no LDS staging and no
// barrier in the row loop.  Groups are grid-strided over the waves, one group
// loaded ahead; the four wave partials of a workgroup are summed in FP64
// through LDS in a fixed order, CH tile pairs at a time.
template <int BT>
__device__ __forceinline__ void gram_bf16_direct_body(SrcT<float> s, int64_t m, const DevState *ds, int which_p,
                                                      int pmax, double *__restrict__ part, int nblk, int vec,
                                                      int bid)
{
    constexpr int NPAIR = BT * (BT + 1) / 2;
    constexpr int CH = gram_bf16_direct_ch(BT);   // pairs per LDS reduction round
    extern __shared__ unsigned char lds_raw[];
    double *red = reinterpret_cast<double *>(lds_raw);   // 4 waves x CH pairs x 4 x 64
    if (s.guard && merge_halted(ds)) return;
    const int P = sel_count(ds, which_p);
    s.rs = ds->rs;
    s.g = ds->g;
    if (s.U1 && (ds->it & 1)) s.U = s.U1;
    const int NT16 = (P + 15) >> 4;
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ci = lane & 15, kr = 8 * (lane >> 4);
    const float *cpt[BT];
    bool live[BT];
    bool same = true;
#pragma unroll
    for (int t = 0; t < BT; ++t) {
        const int c = 16 * t + ci;
        live[t] = c < P;
        const ColPtr cp = col_ptr<float>(s, m, live[t] ? c : 0);
        cpt[t] = reinterpret_cast<const float *>(cp.p);
        same = same && (cp.f64 == 0);
    }
    const bool fast = vec && __all(same);
    const int64_t ngr = (m + 31) >> 5, nfull = m >> 5;
    const int64_t W = (int64_t)bid * 4 + wv, NW = (int64_t)nblk * 4;
    v4f acc[NPAIR];
#pragma unroll
    for (int q = 0; q < NPAIR; ++q) acc[q] = v4f{0, 0, 0, 0};
    auto split = [&](const float (&v)[BT][8], bf16x8 (&oh)[BT], bf16x8 (&od)[BT], bf16x8 (&ol)[BT]) {
#pragma unroll
        for (int t = 0; t < BT; ++t) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                __bf16 a0, a1, a2;
                split3(v[t][q], a0, a1, a2);
                oh[t][q] = a0;
                od[t][q] = a1;
                ol[t][q] = a2;
            }
        }
    };
    auto mma = [&](const bf16x8 (&oh)[BT], const bf16x8 (&od)[BT], const bf16x8 (&ol)[BT]) {
        int q = 0;
#pragma unroll
        for (int I = 0; I < BT; ++I)
#pragma unroll
            for (int J = I; J < BT; ++J, ++q)
                if (J < NT16) acc[q] = mfma_split(oh[I], od[I], ol[I], oh[J], od[J], ol[J], acc[q]);
    };
    auto load_fast = [&](int64_t gr, float (&v)[BT][8]) {
#pragma unroll
        for (int t = 0; t < BT; ++t) {
            const float *p = cpt[t] + gr * 32 + kr;
            const f32x4 a = *reinterpret_cast<const f32x4 *>(p);
            const f32x4 b = *reinterpret_cast<const f32x4 *>(p + 4);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                v[t][q] = live[t] ? a[q] : 0.0f;
                v[t][4 + q] = live[t] ? b[q] : 0.0f;
            }
        }
    };
    int64_t gstart = W;
    if (fast && gstart < nfull) {
        // one group in flight: a group is split into its terms, then the raw
        // registers take the next group's loads (index clamped to the wave's last
        // full group) while the matrix cores work on the terms
        const int64_t lastg = gstart + ((nfull - 1 - gstart) / NW) * NW;
        float vr[BT][8];
        load_fast(gstart, vr);
        for (int64_t gr = gstart;; gr += NW) {
            bf16x8 oh[BT], od[BT], ol[BT];
            split(vr, oh, od, ol);
            const int64_t nx = gr + NW;
            load_fast((nx < lastg) ? nx : lastg, vr);
            mma(oh, od, ol);
            if (gr >= lastg) break;
        }
        gstart = lastg + NW;
    }
    for (int64_t gr = gstart; gr < ngr; gr += NW) {
        float v[BT][8];
#pragma unroll
        for (int t = 0; t < BT; ++t) {
            const ColPtr cp = col_ptr<float>(s, m, live[t] ? 16 * t + ci : 0);
            float a[4], b[4];
            load4<float>(cp, gr * 32 + kr, m, vec, a);
            load4<float>(cp, gr * 32 + kr + 4, m, vec, b);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                v[t][q] = live[t] ? a[q] : 0.0f;
                v[t][4 + q] = live[t] ? b[q] : 0.0f;
            }
        }
        bf16x8 oh[BT], od[BT], ol[BT];
        split(v, oh, od, ol);
        mma(oh, od, ol);
    }
    // sum the four wave partials in FP64 (waves in order), CH tile pairs at a time
    double *pb = part + (int64_t)bid * pmax * pmax;
#pragma unroll
    for (int r0 = 0; r0 < NPAIR; r0 += CH) {
        if (r0) __syncthreads();
#pragma unroll
        for (int qc = 0; qc < CH; ++qc)
            if (r0 + qc < NPAIR)
#pragma unroll
                for (int v = 0; v < 4; ++v) red[((wv * CH + qc) * 4 + v) * 64 + lane] = (double)acc[r0 + qc][v];
        __syncthreads();
        for (int o = threadIdx.x; o < CH * 256; o += 256) {
            const int qc = o >> 8, v = (o >> 6) & 3, ln = o & 63;
            const int q = r0 + qc;
            if (q >= NPAIR) continue;
            // pair q -> (I, J), I <= J, in the order of the accumulation loop
            int I = 0, rem = q;
            while (rem >= BT - I) {
                rem -= BT - I;
                ++I;
            }
            const int J = I + rem;
            if (J >= NT16) continue;
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < 4; ++w) sum += red[((w * CH + qc) * 4 + v) * 64 + ln];
            const int i = 16 * I + acc_row<float>(ln, v), j = 16 * J + (ln & 15);
            if (I < J || i <= j) {
                pb[i + (int64_t)j * pmax] = sum;
                pb[j + (int64_t)i * pmax] = sum;
            }
        }
    }
}

template <int BT>
__global__ __launch_bounds__(256) void k_gram_bf16_direct(SrcT<float> s, int64_t m, const DevState *ds, int which_p,
                                                          int pmax, double *__restrict__ part, int nblk, int vec)
{
    gram_bf16_direct_body<BT>(s, m, ds, which_p, pmax, part, nblk, vec, blockIdx.x);
}

// The three terms of T (pin x pout, ld ldt; counts from the device state),
// transposed: Tb[term][j][k] (JP x KP per term, zero outside pin x pout), so
// that one 16-byte read gives a lane its eight k values of a B operand.
__global__ __launch_bounds__(256) void k_split_t(const float *__restrict__ T, int ldt, const DevState *ds, int sel_in,
                                                 int sel_out, int KP, int JP, __bf16 *__restrict__ Tb, int guard)
{
    if (guard && merge_halted(ds)) return;
    const int pin = sel_count(ds, sel_in), pout = sel_count(ds, sel_out);
    const int tot = JP * KP;
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < tot; idx += gridDim.x * 256) {
        const int j = idx / KP, k = idx % KP;
        const float x = (k < pin && j < pout) ? T[k + (int64_t)j * ldt] : 0.0f;
        __bf16 h, d, l;
        split3(x, h, d, l);
        Tb[idx] = h;
        Tb[idx + tot] = d;
        Tb[idx + 2 * tot] = l;
    }
}


// Packed LDS layout of the split factor: column tile jc keeps its 16 columns of
// kmax(jc) k values (tri: only k < 16 (jc + 1), rounded up to 32).
__host__ __device__ __forceinline__ int tall_kmax(int jc, int KP, int tri)
{
    const int k = 32 * ((jc + 2) / 2);
    return (tri && k < KP) ? k : KP;
}
__host__ __device__ __forceinline__ int tall_koff(int jc, int KP, int tri)
{
    int o = 0;
    for (int c = 0; c < jc; ++c) o += 16 * tall_kmax(c, KP, tri);
    return o;
}

// Tall transform Y = X T on the split operands straight from registers.  Each
// wave takes whole 32-row groups (grid-strided): lane (i, kq) = (l % 16, l / 16)
// loads X(row, k) for rows 16 rb + i and k = 32 ks + 8 kq + t (eight columns of
// a k step, through column pointers kept in LDS), one group ahead, splits them
// into three bf16 terms per k step and accumulates every output tile of its
// rows (2 row blocks x NJM column tiles) against the split factor, which the
// workgroup copies to LDS once (packed; B operands by 16-byte reads).  No
// barrier in the row loop; each lane stores four consecutive rows of one output
// column.
template <int KS, int NJM>
__global__ __launch_bounds__(256) void k_gemm_tall_bf16_direct(SrcT<float> s, int64_t m, const DevState *ds,
                                                               int sel_in, int sel_out, const __bf16 *__restrict__ Tb,
                                                               int KP, int JP, float *__restrict__ Yout,
                                                               float *__restrict__ Yout1, int vout, int tri)
{
    extern __shared__ unsigned char lds_raw[];
    const float **cptr = reinterpret_cast<const float **>(lds_raw);   // KS * 32 column pointers
    __bf16 *Ts = reinterpret_cast<__bf16 *>(lds_raw + KS * 32 * sizeof(const float *));
    if (s.guard && merge_halted(ds)) return;
    if (Yout1 && (ds->it & 1)) Yout = Yout1;
    const int pin = sel_count(ds, sel_in), pout = sel_count(ds, sel_out);
    s.rs = ds->rs;
    s.g = ds->g;
    if (s.U1 && (ds->it & 1)) s.U = s.U1;
    const int NKS = (pin + 31) >> 5;   // k steps used (<= KS)
    const int NJ = (pout + 15) >> 4;   // output column tiles used (<= NJM)
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ci = lane & 15, kq = lane >> 4;
    for (int k = threadIdx.x; k < KS * 32; k += 256)
        cptr[k] = reinterpret_cast<const float *>(col_ptr<float>(s, m, (k < pin) ? k : 0).p);
    const int tot = tall_koff(JP / 16, KP, tri);   // packed elements per term
    {
        const int64_t tsz = (int64_t)JP * KP;
        const int k8 = KP / 8;
        for (int idx = threadIdx.x; idx < 3 * JP * k8; idx += 256) {
            const int t = idx / (JP * k8), rem = idx % (JP * k8);
            const int j = rem / k8, k = 8 * (rem % k8);
            const int jc = j >> 4, km = tall_kmax(jc, KP, tri);
            if (k < km)
                *reinterpret_cast<bf16x8 *>(Ts + t * tot + tall_koff(jc, KP, tri) + (j & 15) * km + k) =
                    *reinterpret_cast<const bf16x8 *>(Tb + t * tsz + (int64_t)j * KP + k);
        }
    }
    __syncthreads();
    int toff[NJM], tkm[NJM];
#pragma unroll
    for (int jc = 0; jc < NJM; ++jc) {
        tkm[jc] = tall_kmax(jc, KP, tri);
        toff[jc] = tall_koff(jc, KP, tri);
    }
    const int64_t ngr = (m + 31) >> 5;
    const int64_t W = (int64_t)blockIdx.x * 4 + wv, NW = (int64_t)gridDim.x * 4;
    // every load issued with no branch around it (a load inside a branch is
    // waited for where the branch ends, and every load before it): rows past
    // m read row m - 1, columns past pin read column 0 (cptr), and both are
    // replaced by zero afterwards
    auto load = [&](int64_t gr, float (&x)[2][KS][8]) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int k = 32 * ks + 8 * kq + t;
                const float *cp = cptr[k];
                const bool kin = ks < NKS && k < pin;
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    const int64_t row = gr * 32 + 16 * rb + ci;
                    const bool rin = row < m;
                    const float v = cp[rin ? row : m - 1];
                    x[rb][ks][t] = (kin && rin) ? v : 0.0f;
                }
            }
        }
    };
    auto process = [&](int64_t gr, const float (&x)[2][KS][8]) {
        v4f acc[2][NJM];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int jc = 0; jc < NJM; ++jc) acc[rb][jc] = v4f{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            if (ks >= NKS) continue;   // uniform
            bf16x8 ah[2], ad[2], al[2];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    __bf16 a0, a1, a2;
                    split3(x[rb][ks][t], a0, a1, a2);
                    ah[rb][t] = a0;
                    ad[rb][t] = a1;
                    al[rb][t] = a2;
                }
#pragma unroll
            for (int jc = 0; jc < NJM; ++jc) {
                // with T upper triangular the k steps past column tile jc are zero
                if (jc < NJ && !(tri && 32 * ks >= 16 * (jc + 1))) {
                    const __bf16 *tb = Ts + toff[jc] + ci * tkm[jc] + 32 * ks + 8 * kq;
                    const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(tb);
                    const bf16x8 bd = *reinterpret_cast<const bf16x8 *>(tb + tot);
                    const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(tb + 2 * tot);
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb)
                        acc[rb][jc] = mfma_split(ah[rb], ad[rb], al[rb], bh, bd, bl, acc[rb][jc]);
                }
            }
        }
#pragma unroll
        for (int jc = 0; jc < NJM; ++jc) {
            const int col = 16 * jc + ci;
            if (jc >= NJ || col >= pout) continue;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const int64_t row0 = gr * 32 + 16 * rb + 4 * kq;
                float *y = Yout + (int64_t)col * m + row0;
                if (vout && row0 + 4 <= m) {
                    *reinterpret_cast<f32x4 *>(y) = acc[rb][jc];
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (row0 + v < m) y[v] = acc[rb][jc][v];
                }
            }
        }
    };
    if (W < ngr) {
        float xa[2][KS][8];
        load(W, xa);
        for (int64_t gr = W; gr < ngr; gr += NW) {
            float xc[2][KS][8];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                    for (int t = 0; t < 8; ++t) xc[rb][ks][t] = xa[rb][ks][t];
            // (the last group reloads itself: no branch around the prefetch)
            load((gr + NW < ngr) ? gr + NW : gr, xa);
            process(gr, xc);
        }
    }
}

template <int KS, int NJM>
static void tall_bf16_direct_launch(const SrcT<float> &s, int64_t m, const DevState *ds, int which_in,
                                    int which_out, const __bf16 *Tb, int KP, int JP, void *Yout, void *Yout1,
                                    int vout, int tri, hipStream_t st)
{
    const size_t lds = (size_t)KS * 32 * sizeof(const float *) + (size_t)3 * tall_koff(JP / 16, KP, tri) * 2;
    static bool attr = false;
    if (!attr) {
        if (hipFuncSetAttribute((const void *)k_gemm_tall_bf16_direct<KS, NJM>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, TALL_DYN_LDS) != hipSuccess)
            return;   // the launch below then fails and reports the error
        attr = true;
    }
    const int64_t ngr = (m + 31) >> 5;
    const int64_t want = (ngr + 3) / 4;
    const unsigned nb = (unsigned)((want < 256) ? ((want > 0) ? want : 1) : 256);
    hipLaunchKernelGGL((k_gemm_tall_bf16_direct<KS, NJM>), dim3(nb), dim3(256), lds, st, s, m, ds, which_in,
                       which_out, Tb, KP, JP, (float *)Yout, (float *)Yout1, vout, tri);
}

template <typename TC, int MAXPW, int ITEMS, int NWV>
static void gram_launch(const GemmDesc &d, const DevState *ds, int32_t which_p, int32_t pmax, double *part,
                        int32_t nblk, hipStream_t st)
{
    const SrcT<TC> s = make_src<TC>(d);
    // the stage holds every item's column (ITEMS * 64 NWV / GRP >= pmax)
    const size_t lds = (size_t)(ITEMS * 64 * NWV / GRP) * LDSR * sizeof(TC);
    if (lds > 64 * 1024) {
        // (should this fail, the launch below fails and reports the error)
        static bool attr = false;
        if (!attr)
            attr = hipFuncSetAttribute((const void *)k_gram_partial<TC, MAXPW, ITEMS, NWV>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess;
    }
    hipLaunchKernelGGL((k_gram_partial<TC, MAXPW, ITEMS, NWV>), dim3(nblk), dim3(64 * NWV), lds, st, s, d.m, ds,
                       which_p, pmax, part, nblk, (int)vec_ok(s, d.m));
}

hipError_t launch_gram_partial(const GemmDesc &d, const DevState *ds, int32_t which_p, int32_t pmax, double *part,
                               int32_t nblk, hipStream_t st)
{
    if (pmax > PMAX_ADJ) return hipErrorInvalidValue;
    ProfScope ps(POD_K_GRAM, st);
    const bool wide = pmax > 64;
    if (pmax > PMAX_WIDE) {
        if (d.prec == POD_F64) gram_launch<double, MAXPW208_8, ITEMS208_8, 8>(d, ds, which_p, pmax, part, nblk, st);
        else if (d.prec == POD_F32) gram_launch<float, MAXPW208_8, ITEMS208_8, 8>(d, ds, which_p, pmax, part, nblk, st);
        else return hipErrorInvalidValue;
    } else if (d.prec == POD_BF16_REFINE) {
        if (d.a_dtype != POD_F32) return hipErrorInvalidValue;
        const SrcT<float> s = make_src<float>(d);
        const int vec = (int)vec_ok(s, d.m);
        if (wide)
            hipLaunchKernelGGL((k_gram_bf16_direct<10>), dim3(nblk), dim3(256), gram_bf16_direct_lds(10), st, s, d.m,
                               ds, which_p, pmax, part, nblk, vec);
        else
            hipLaunchKernelGGL((k_gram_bf16_direct<4>), dim3(nblk), dim3(256), gram_bf16_direct_lds(4), st, s, d.m, ds,
                               which_p, pmax, part, nblk, vec);
    } else if (d.prec == POD_F64) {
        if (wide) {
            gram_launch<double, MAXPW160_8, ITEMS160_8, 8>(d, ds, which_p, pmax, part, nblk, st);
        } else {
            const SrcT<double> s = make_src<double>(d);
            hipLaunchKernelGGL(k_gram_direct<double>, dim3(nblk), dim3(512), GD_LDS, st, s, d.m, ds, which_p, pmax,
                               part, nblk, (int)vec_ok(s, d.m));
        }
    } else {
        if (wide) {
            gram_launch<float, MAXPW160_8, ITEMS160_8, 8>(d, ds, which_p, pmax, part, nblk, st);
        } else {
            const SrcT<float> s = make_src<float>(d);
            hipLaunchKernelGGL(k_gram_direct<float>, dim3(nblk), dim3(512), GD_LDS, st, s, d.m, ds, which_p, pmax,
                               part, nblk, (int)vec_ok(s, d.m));
        }
    }
    return hipGetLastError();
}

hipError_t launch_gram_reduce_sel(const double *part, int32_t nblk, int32_t pmax, const DevState *ds,
                                  int32_t which_p, double *G, hipStream_t st)
{
    ProfScope ps(POD_K_GRAM_REDUCE, st);
    hipLaunchKernelGGL(k_gram_reduce, dim3((pmax * pmax + 63) / 64), dim3(64 * GR_W), 0, st, part, nblk, pmax, ds,
                       which_p, G);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tall transform Y = X T (m x pout) with T pin x pout (ld ldt, compute type).
// Each workgroup stages T once and about TALL_ST stages of RB rows of X
// (grid-strided), producing
// the output as Y^T tiles = T^T X^T so that each lane's four results are
// consecutive rows of one output column.  T is staged in LDS in full, or,
// when it is upper triangular and square (T1 = R1^-1 of the first pass) and
// too large for that (FP64, 160 x 160), as its 16 x 16 tiles (kt, jt) with
// kt <= jt packed column by column (tile jt (jt + 1) / 2 + kt, rows of 16
// inside a tile); otherwise it is read from device memory (L2).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int tri_tiles(int nt) { return nt * (nt + 1) / 2; }

// Scatter output (SCAT): output columns below `split` go to Yout, column
// split + j is added to D(:, cmap[j]) (leading dimension ldd); the mapped
// columns are distinct, so each element has one writer.
struct TallScatter {
    int32_t split;
    const int32_t *cmap;
    void *D;
    int64_t ldd;
};

template <typename TC, int ITEMS, bool TG, bool SCAT = false, bool TP = false>
__device__ __forceinline__ void gemm_tall_body(SrcT<TC> s, int64_t m, const DevState *ds, int sel_in, int sel_out,
                                               int pmax_in, int pmax_out, const TC *__restrict__ T, int ldt,
                                               TC *__restrict__ Yout, TC *__restrict__ Yout1, int vec, int bid,
                                               int nbk, int tri, TallScatter sc = TallScatter{0, nullptr, nullptr, 0})
{
    typedef typename Acc<TC>::type AccT;
    extern __shared__ unsigned char lds_raw[];
    if (s.guard && merge_halted(ds)) return;
    if (Yout1 && (ds->it & 1)) Yout = Yout1;
    const int pin = sel_count(ds, sel_in), pout = sel_count(ds, sel_out);
    s.rs = ds->rs;
    s.g = ds->g;
    if (s.U1 && (ds->it & 1)) s.U = s.U1;
    const int PI = (pin + 15) & ~15, PO = (pout + 15) & ~15;
    TC *Xs = reinterpret_cast<TC *>(lds_raw);        // pmax_in x LDSR
    TC *Ts = Xs + pmax_in * LDSR;                    // PI x PO, row k at Ts + k * PO (when !TG)
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar tile loops
    // row stages bid, bid + nbk, bid + 2 nbk, ...: at each step the nbk
    // workgroups together read one contiguous span of every column
    const int64_t nst = (m + RB - 1) / RB;
    const int64_t ns = (bid < nst) ? (nst - 1 - bid) / nbk + 1 : 0;   // stages of this workgroup
    auto stage = [&](int64_t i) { return (int64_t)bid + i * nbk; };
    // T is read down its columns (16 consecutive k per 16 threads) and
    // written to LDS in the layout of the MFMA operand reads
    if (TP) {
        // packed upper-triangular tiles (PI == PO)
        const int nt = PO / 16;
        for (int idx = threadIdx.x; idx < tri_tiles(nt) * 256; idx += 256) {
            const int t = idx >> 8, e = idx & 255;
            int jt = 0;
            while (tri_tiles(jt + 1) <= t) ++jt;
            const int kt = t - tri_tiles(jt);
            const int kk = e & 15, jj = e >> 4;
            const int k = 16 * kt + kk, j = 16 * jt + jj;
            Ts[t * 256 + kk * 16 + jj] = (k < pin && j < pout && k <= j) ? T[k + (int64_t)j * ldt] : (TC)0;
        }
    } else if (!TG) {
        for (int idx = threadIdx.x; idx < PI * PO; idx += 256) {
            const int k = idx % PI, j = idx / PI;
            Ts[k * PO + j] = (k < pin && j < pout) ? T[k + (int64_t)j * ldt] : (TC)0;
        }
    }
    (void)pmax_out;
    const int ntile = (RB / 16) * (PO / 16);
    // one output tile (rows rbk of the stage, columns jc) to Y (or the scatter target)
    auto store_tile = [&](int64_t sg, int rbk, int jc, const AccT &acc) {
        const int64_t row = sg * RB + rbk * 16 + (lane & 15);
        if (row < m) {
            if (!SCAT) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int col = jc * 16 + acc_row<TC>(lane, v);
                    if (col < pout) Yout[(int64_t)col * m + row] = acc[v];
                }
            } else {
                // the scattered read-modify-writes: the column map and the old
                // values are read for all four first, with no branch (entries
                // that are not scattered read index 0 and D(row, column 0)),
                // so that the loads are in flight together
                int ci[4];
                TC *dst[4];
                TC old[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int col = jc * 16 + acc_row<TC>(lane, v);
                    const bool sct = col >= sc.split && col < pout;
                    ci[v] = sc.cmap[sct ? col - sc.split : 0];
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int col = jc * 16 + acc_row<TC>(lane, v);
                    const bool sct = col >= sc.split && col < pout;
                    dst[v] = reinterpret_cast<TC *>(sc.D) + (sct ? (int64_t)ci[v] * sc.ldd : 0) + row;
                    old[v] = *dst[v];
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int col = jc * 16 + acc_row<TC>(lane, v);
                    if (col >= pout) continue;
                    if (col < sc.split) Yout[(int64_t)col * m + row] = acc[v];
                    else *dst[v] = old[v] + acc[v];
                }
            }
        }
    };
    // T in LDS: wave wv owns the tiles of row block rbk = wv % 2 and column
    // tiles jc = wv / 2 + 2 i; each X operand read from LDS feeds the MFMAs of
    // all of them, which accumulate independently (no chained MFMAs)
    constexpr int MAXJ = (ITEMS * 256 / GRP) / 32;
    auto compute_lds = [&](int64_t sg) {
        const int rbk = wv & 1, j0 = wv >> 1;
        const int nj = (PO / 16 > j0) ? (PO / 16 - j0 + 1) / 2 : 0;
        // k extent: T upper triangular ends column tile jc at row 16 (jc + 1)
        const int jlast = j0 + 2 * (nj - 1);
        const int ke = (tri && nj > 0 && 16 * (jlast + 1) < PI) ? 16 * (jlast + 1) : PI;
        if (nj == 0) return;
        AccT acc[MAXJ];
#pragma unroll
        for (int i = 0; i < MAXJ; ++i) acc[i] = AccT{0, 0, 0, 0};
        const TC *xb = Xs + (lane >> 4) * LDSR + rbk * 16 + (lane & 15);
        for (int k4 = 0; k4 < ke; k4 += 16) {
            TC xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = xb[(k4 + 4 * u) * LDSR];
#pragma unroll
            for (int i = 0; i < MAXJ; ++i) {
                const int jc = j0 + 2 * i;
                if (i < nj && (!tri || k4 < 16 * (jc + 1))) {
                    TC av[4];
                    if (TP) {
                        const TC *tp = Ts + (tri_tiles(jc) + k4 / 16) * 256 + (lane >> 4) * 16 + (lane & 15);
#pragma unroll
                        for (int u = 0; u < 4; ++u) av[u] = tp[64 * u];
                    } else {
                        const TC *ta = Ts + (k4 + (lane >> 4)) * PO + jc * 16 + (lane & 15);
#pragma unroll
                        for (int u = 0; u < 4; ++u) av[u] = ta[4 * u * PO];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc[i] = mfma16x16x4(av[u], xv[u], acc[i]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < MAXJ; ++i)
            if (i < nj) store_tile(sg, rbk, j0 + 2 * i, acc[i]);
    };
    auto compute = [&](int64_t sg) {
        if (!TG) {
            compute_lds(sg);
            return;
        }
        // T read from device memory (L2 resident), zero outside pin x pout
        // (lanes past pin or pout load an element inside T and drop it: no
        // branch around the loads); the wave's tiles wv, wv + 4, ... in
        // groups of four with independent accumulators, each tile summing k in
        // order
        for (int t0 = wv; t0 < ntile; t0 += 16) {
            AccT acc[4];
            const TC *xb[4], *ta[4];
            bool ok[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int tile = t0 + 4 * u;
                const int rbk = tile % (RB / 16), jc = tile / (RB / 16);
                const int jj = jc * 16 + (lane & 15);
                ok[u] = tile < ntile && jj < pout;
                acc[u] = AccT{0, 0, 0, 0};
                xb[u] = Xs + (lane >> 4) * LDSR + rbk * 16 + (lane & 15);
                ta[u] = T + (lane >> 4) + (int64_t)(ok[u] ? jj : 0) * ldt;
            }
            for (int k4 = 0; k4 < PI; k4 += 4) {
                const bool kin = k4 + (lane >> 4) < pin;
                TC tv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) tv[u] = ta[u][kin ? k4 : 0];
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[u] = mfma16x16x4((ok[u] && kin) ? tv[u] : (TC)0, xb[u][k4 * LDSR], acc[u]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int tile = t0 + 4 * u;
                if (tile < ntile) store_tile(sg, tile % (RB / 16), tile / (RB / 16), acc[u]);
            }
        }
    };
    Stage<TC, ITEMS> sa, sb;
    sa.prepare(s, m, pin, vec);
    sb.fast = sa.fast;
    sb.f32col = sa.f32col;
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) sb.base[it] = sa.base[it];
    // stages entirely inside [0, m) on the fast path (the last stage may be partial)
    const int64_t full_end = m / RB;
    int64_t nf = (bid < full_end) ? (full_end - 1 - bid) / nbk + 1 : 0;
    if (!sa.fast) nf = 0;
    if (nf > ns) nf = ns;
    if (nf > 0) {
        const int64_t last = nf - 1;
        sa.load_full(stage(0) * RB);
        sb.load_full(stage((1 < last) ? 1 : last) * RB);
        int64_t i = 0;
        for (; i + 1 < nf; i += 2) {
            __syncthreads();
            sa.store_all(Xs, pin);
            __syncthreads();
            sa.load_full(stage((i + 2 < last) ? i + 2 : last) * RB);
            compute(stage(i));
            __syncthreads();
            sb.store_all(Xs, pin);
            __syncthreads();
            sb.load_full(stage((i + 3 < last) ? i + 3 : last) * RB);
            compute(stage(i + 1));
        }
        if (i < nf) {
            __syncthreads();
            sa.store_all(Xs, pin);
            __syncthreads();
            compute(stage(i));
        }
    }
    for (int64_t i = nf; i < ns; ++i) {
        sa.load(s, m, stage(i) * RB, pin, vec);
        __syncthreads();
        sa.store(Xs, PI, pin);
        __syncthreads();
        compute(stage(i));
    }
}

template <typename TC, int ITEMS, bool TG, bool TP>
__global__ __launch_bounds__(256) void k_gemm_tall(SrcT<TC> s, int64_t m, const DevState *ds, int sel_in,
                                                   int sel_out, int pmax_in, int pmax_out, const TC *__restrict__ T,
                                                   int ldt, TC *__restrict__ Yout, TC *__restrict__ Yout1, int vec,
                                                   int tri)
{
    gemm_tall_body<TC, ITEMS, TG, false, TP>(s, m, ds, sel_in, sel_out, pmax_in, pmax_out, T, ldt, Yout, Yout1, vec,
                                             blockIdx.x, gridDim.x, tri);
}

template <typename TC, int ITEMS>
__global__ __launch_bounds__(256) void k_gemm_tall_scatter(SrcT<TC> s, int64_t m, const DevState *ds, int sel_in,
                                                           int sel_out, int pmax_in, const TC *__restrict__ T,
                                                           int ldt, TC *__restrict__ Yout, TallScatter sc, int vec)
{
    gemm_tall_body<TC, ITEMS, false, true>(s, m, ds, sel_in, sel_out, pmax_in, 0, T, ldt, Yout, nullptr, vec,
                                           blockIdx.x, gridDim.x, 0, sc);
}

// Batched scatter (P <= 64): matrix blockIdx.y, its own block count.
template <typename TC>
__global__ __launch_bounds__(256) void k_gemm_tall_scatter_b(const ScatterArgs *__restrict__ arr)
{
    const ScatterArgs &a = arr[blockIdx.y];
    if ((int)blockIdx.x >= a.nb) return;
    const TallScatter sc{a.split, a.cmap, a.D, a.ldd};
    gemm_tall_body<TC, ITEMS64, false, true>(make_src<TC>(a.d), a.d.m, a.ds, a.which_in, a.which_out, 64, 0,
                                             reinterpret_cast<const TC *>(a.T), a.ldt, reinterpret_cast<TC *>(a.Yout),
                                             nullptr, a.vec, blockIdx.x, a.nb, 0, sc);
}

template <typename TC, int ITEMS>
__global__ __launch_bounds__(256) void k_gemm_tall_b(const TallArgs *__restrict__ arr)
{
    const TallArgs &a = arr[blockIdx.y];
    if ((int)blockIdx.x >= a.nb || a.ds->done) return;
    gemm_tall_body<TC, ITEMS, false>(make_src<TC>(a.d), a.d.m, a.ds, a.sel_in, a.sel_out, ITEMS * 256 / GRP, a.pout_max,
                                     reinterpret_cast<const TC *>(a.T), a.ldt, reinterpret_cast<TC *>(a.Yout),
                                     reinterpret_cast<TC *>(a.Yout1), a.vec, blockIdx.x, a.nb, a.tri);
}

// ---------------------------------------------------------------------------
// FP64 tall transform Y = X T (X: m x pin gathered source, T: pin x pout,
// pin <= 16 KT, pout <= 16 NJ) with the X operands loaded straight into the
// matrix-core registers: wave w of a workgroup takes the 16-row tiles
// 8 b + w, 8 (b + nb) + w, ... and for each computes all of the output's
// column tiles as Y^T = T^T X^T on v_mfma_f64_16x16x4.  The B operand (X^T,
// four k-chunks per 16 columns of X) is read from device memory, 16
// consecutive rows of one column per 16 lanes; the A operand (T^T) from T
// staged once per workgroup in LDS, tile (kt, jt) at jt (jt + 1) / 2 + kt (TP:
// upper triangular, kt <= jt) or jt KT + kt, 256 doubles in the operand
// layout.  The products of a row tile run k-chunk by k-chunk across the
// column tiles' accumulators (independent chains), each accumulator in k
// order: the arithmetic of the staged kernel, bit for bit.  Two waves per
// SIMD overlap one tile's loads with another's products; no barrier after
// the staging.  The lane's results are rows l % 16 of columns
// 16 jt + l / 16 + 4 v.  Column sources come from a table (LDS) of base
// addresses, bit 0 marking an FP32 column of A.
// ---------------------------------------------------------------------------
constexpr int T64_WAVES = 8;

typedef __attribute__((address_space(1))) const double gdouble;
typedef __attribute__((address_space(1))) const uint32_t gu32;

// SCAT: the reverse pass's transform of [U | A(:, I) | Ubar] (scatter output
// as TallScatter; D leading dimension m): workgroup row blockIdx.y takes the
// output columns [16 NJ y, 16 NJ (y + 1)) with that slice of T.
// TS: the storage type of the basis columns, T and the outputs (float on the
// FP32 path: every operand widened to FP64, the products in FP64).
template <int KT, int NJ, bool TP, bool MIX, bool SCAT = false, typename TS = double>
__global__ __launch_bounds__(64 * T64_WAVES) void k_tall64(SrcT<TS> s, int64_t m, const DevState *ds, int sel_in,
                                                           int sel_out, const TS *__restrict__ T, int ldt,
                                                           TS *Yout, TS *Yout1, int tri, TallScatter sc)
{
    extern __shared__ double tl[];
    __shared__ uint64_t cptr[16 * KT];
    if (s.guard && merge_halted(ds)) return;
    if (Yout1 && (ds->it & 1)) Yout = Yout1;
    const int pin = sel_count(ds, sel_in);
    int pout = sel_count(ds, sel_out);
    if (SCAT) {
        const int j0 = (int)blockIdx.y * 16 * NJ;
        T += (int64_t)j0 * ldt;
        Yout += (int64_t)j0 * m;
        sc.split -= j0;
        pout = (pout - j0 < 16 * NJ) ? pout - j0 : 16 * NJ;
    }
    s.rs = ds->rs;
    s.g = ds->g;
    if (s.U1 && (ds->it & 1)) s.U = s.U1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // entry 64 q + l of tile (kt, jt) is T(16 kt + 4 q + l / 16, 16 jt + l % 16)
    const int ntl = TP ? NJ * (NJ + 1) / 2 : KT * NJ;   // every tile, zero outside pin x pout
    for (int idx = threadIdx.x; idx < ntl * 256; idx += 64 * T64_WAVES) {
        const int t = idx >> 8, e = idx & 255;
        int kt, jt;
        if (TP) {
            jt = 0;
            while ((jt + 1) * (jt + 2) / 2 <= t) ++jt;
            kt = t - jt * (jt + 1) / 2;
        } else {
            jt = t / KT;
            kt = t % KT;
        }
        const int k = 16 * kt + 4 * (e >> 6) + ((e >> 4) & 3), j = 16 * jt + (e & 15);
        tl[idx] = (k < pin && j < pout && (!tri || k <= j)) ? (double)T[k + (int64_t)j * ldt] : 0.0;
    }
    for (int c = threadIdx.x; c < 16 * KT; c += 64 * T64_WAVES) {
        uint64_t v = 0;
        if (c < pin) {
            const ColPtr cp = col_ptr<TS>(s, m, c);
            v = (uint64_t)(uintptr_t)cp.p | (cp.f64 ? 0u : 1u);
        }
        cptr[c] = v;
    }
    __syncthreads();
    const int64_t ntile = (m + 15) >> 4;
    const int r16 = lane & 15, cg = lane >> 4;
    // SCAT: the target column of D of every output column of the lane (0 where
    // the column is not scattered)
    int ci[SCAT ? NJ : 1][4];
#pragma unroll
    for (int jt = 0; jt < (SCAT ? NJ : 1); ++jt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int col = 16 * jt + cg + 4 * v;
            const bool sct = SCAT && col >= sc.split && col < pout;
            ci[jt][v] = SCAT ? sc.cmap[sct ? col - sc.split : 0] : 0;
            if (!sct) ci[jt][v] = 0;
        }
    // one row tile: its X operands (raw bits, FP32 columns widened by widen),
    // then the products and the stores
    auto load_tile = [&](int64_t rt, double (&x)[KT][4], uint32_t (&xf)[KT][4], uint32_t (&sel)[KT]) {
        const int64_t row = 16 * rt + r16;
        const bool rin = row < m;
        // X^T chunks: X(row, 16 kt + 4 q + l / 16).  Every load is issued with
        // no branch around it (a load inside a branch, even a wave-uniform one,
        // is waited for where the branch ends): with FP32 columns in the
        // source (MIX) both the FP64 and the FP32 read of every element, the
        // one that does not apply from a fixed valid address, selected and
        // widened afterwards.  Columns at or beyond pin (a zero table entry)
        // read T(0, 0) and meet zero rows of the staged T; rows past m read
        // row m - 1 and feed only output rows that are not stored.
        const int64_t rowc = rin ? row : m - 1;
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            sel[kt] = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint64_t cpv = cptr[16 * kt + 4 * q + cg];
                const bool f32 = MIX && (cpv & 1u);
                const uint64_t a64 = (cpv && !f32) ? cpv + 8 * (uint64_t)rowc : (uint64_t)(uintptr_t)T;
                x[kt][q] = *reinterpret_cast<const gdouble *>(a64);
                if (MIX) {
                    const uint64_t a32 = f32 ? (cpv & ~(uint64_t)1) + 4 * (uint64_t)rowc : (uint64_t)(uintptr_t)T;
                    xf[kt][q] = *reinterpret_cast<const gu32 *>(a32);
                }
                sel[kt] |= f32 ? 1u << q : 0u;
            }
            // (keeps the address arithmetic of later chunks from being hoisted
            // here, which would hold every address in registers at once)
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    auto widen = [&](double (&x)[KT][4], const uint32_t (&xf)[KT][4], const uint32_t (&sel)[KT]) {
        if (MIX) {
#pragma unroll
            for (int kt = 0; kt < KT; ++kt)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    x[kt][q] = ((sel[kt] >> q) & 1u) ? (double)__uint_as_float(xf[kt][q]) : x[kt][q];
        }
    };
    auto mma_store = [&](int64_t rt, const double (&x)[KT][4]) {
        const int64_t row = 16 * rt + r16;
        const bool rin = row < m;
        // T's operands are read from LDS anew for every row tile (a base offset
        // the compiler cannot see through keeps them from being hoisted out of
        // the row loop into registers)
        int toff = 0;
        asm volatile("" : "+s"(toff));
        const double *tlr = tl + toff;
        v4d acc[NJ];
#pragma unroll
        for (int jt = 0; jt < NJ; ++jt) acc[jt] = v4d{0.0, 0.0, 0.0, 0.0};
        // (every tile of the template's shape, with no test of the live widths:
        // the staged T is zero outside them, so the extra products add zeros,
        // and a branch here would cost more, in register copies of the
        // accumulators, than the products it saves)
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int jt = 0; jt < NJ; ++jt) {
                    if (TP && kt > jt) continue;
                    const int t = TP ? jt * (jt + 1) / 2 + kt : jt * KT + kt;
                    acc[jt] = mfma16x16x4(tlr[256 * t + 64 * q + lane], x[kt][q], acc[jt]);
                }
        }
        if (SCAT) {
            // read-modify-write of the scattered columns, four at a time: the
            // old values are loaded with no branch (row m - 1 past the end,
            // column 0 of D where the column is not scattered)
            const int64_t rowc = rin ? row : m - 1;
            TS *D = reinterpret_cast<TS *>(sc.D);
#pragma unroll
            for (int jt = 0; jt < NJ; ++jt) {
                TS old[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) old[v] = D[(int64_t)ci[jt][v] * sc.ldd + rowc];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int col = 16 * jt + cg + 4 * v;
                    if (rin && col < pout) {
                        if (col < sc.split) Yout[(int64_t)col * m + row] = (TS)acc[jt][v];
                        else D[(int64_t)ci[jt][v] * sc.ldd + row] = (TS)((double)old[v] + acc[jt][v]);
                    }
                }
            }
        } else if (rin) {
            // (the column stride laundered per row tile: the forty column
            // addresses are not hoisted out of the row loop into registers)
            int64_t ms = m;
            asm volatile("" : "+s"(ms));
#pragma unroll
            for (int jt = 0; jt < NJ; ++jt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int col = 16 * jt + cg + 4 * v;
                    if (col < pout) Yout[(int64_t)col * ms + row] = (TS)acc[jt][v];
                }
        }
    };
    const int64_t stride = (int64_t)gridDim.x * T64_WAVES;
    int64_t rt = (int64_t)blockIdx.x * T64_WAVES + wv;
    for (; rt < ntile; rt += stride) {
        double x[KT][4];
        uint32_t xf[KT][4], sel[KT];
        load_tile(rt, x, xf, sel);
        widen(x, xf, sel);
        mma_store(rt, x);
    }
}

template <int KT, int NJ, bool TP, bool MIX>
static void tall64_launch_t(const GemmDesc &d, const DevState *ds, int32_t which_in, int32_t which_out, const void *T,
                          int32_t ldt, void *Yout, void *Yout1, int tri, hipStream_t st)
{
    const SrcT<double> s = make_src<double>(d);
    const size_t lds = (size_t)(TP ? NJ * (NJ + 1) / 2 : KT * NJ) * 256 * sizeof(double);
    static bool attr = false;
    if (lds > 64 * 1024 && !attr) {
        if (hipFuncSetAttribute((const void *)k_tall64<KT, NJ, TP, MIX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return;   // the launch below then fails and reports the error
        attr = true;
    }
    // one workgroup per CU where T fills most of the LDS, more where it is
    // small; at least four row tiles per wave, so that staging T pays off
    const int per_cu = (lds > 80 * 1024) ? 1 : (lds > 40 * 1024 ? 2 : 4);
    const int64_t ntile = (d.m + 15) / 16;
    const int64_t want = (ntile + 4 * T64_WAVES - 1) / (4 * T64_WAVES);
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 256 * per_cu));
    hipLaunchKernelGGL((k_tall64<KT, NJ, TP, MIX>), dim3(nb), dim3(64 * T64_WAVES), lds, st, s, d.m, ds, which_in,
                       which_out, (const double *)T, ldt, (double *)Yout, (double *)Yout1, tri, TallScatter{0, nullptr, nullptr, 0});
}

// The scatter transform of the reverse pass on FP64 (column groups of 16 NJ).
template <int KT, int NJ, bool MIX, typename TS = double>
static hipError_t tall64_scatter_launch(const GemmDesc &d, const DevState *ds, int32_t which_in, int32_t which_out,
                                        int32_t pout_max, const TS *T, int32_t ldt, TS *Yout,
                                        const TallScatter &sc, hipStream_t st)
{
    const SrcT<TS> s = make_src<TS>(d);
    const size_t lds = (size_t)KT * NJ * 256 * sizeof(double);
    static bool attr = false;
    if (lds > 64 * 1024 && !attr)
        attr = hipFuncSetAttribute((const void *)k_tall64<KT, NJ, false, MIX, true, TS>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess;
    const unsigned ng = (unsigned)((pout_max + 16 * NJ - 1) / (16 * NJ));
    const int64_t ntile = (d.m + 15) / 16;
    const int64_t want = (ntile + 4 * T64_WAVES - 1) / (4 * T64_WAVES);
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 256));
    hipLaunchKernelGGL((k_tall64<KT, NJ, false, MIX, true, TS>), dim3(nb, ng), dim3(64 * T64_WAVES), lds, st, s, d.m,
                       ds, which_in, which_out, T, ldt, Yout, (TS *)nullptr, 0, sc);
    return hipGetLastError();
}

// MIX: some columns of the source are FP32 (gathered columns of an FP32 A)
template <int KT, int NJ, bool TP>
static void tall64_launch(const GemmDesc &d, const DevState *ds, int32_t which_in, int32_t which_out, const void *T,
                          int32_t ldt, void *Yout, void *Yout1, int tri, hipStream_t st)
{
    if (d.gather && d.a_dtype != POD_F64)
        tall64_launch_t<KT, NJ, TP, true>(d, ds, which_in, which_out, T, ldt, Yout, Yout1, tri, st);
    else
        tall64_launch_t<KT, NJ, TP, false>(d, ds, which_in, which_out, T, ldt, Yout, Yout1, tri, st);
}

template <typename TC, int ITEMS, bool TG, bool TP = false>
static void tall_launch(const GemmDesc &d, const DevState *ds, int32_t which_in, int32_t which_out, int PI, int PO,
                        const void *T, int32_t ldt, void *Yout, void *Yout1, unsigned nb, int tri, hipStream_t st)
{
    const SrcT<TC> s = make_src<TC>(d);
    constexpr int CW = ITEMS * 256 / GRP;   // columns of the LDS stage (every item stored)
    const size_t tsz = TP ? (size_t)tri_tiles(PO / 16) * 256 : (TG ? 0 : (size_t)PI * PO);
    const size_t lds = (CW * LDSR + tsz) * sizeof(TC);
    static bool attr = false;
    if (lds > 64 * 1024 && !attr) {
        if (hipFuncSetAttribute((const void *)k_gemm_tall<TC, ITEMS, TG, TP>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, TALL_DYN_LDS) != hipSuccess)
            return;   // the launch below then fails and reports the error
        attr = true;
    }
    hipLaunchKernelGGL((k_gemm_tall<TC, ITEMS, TG, TP>), dim3(nb), dim3(256), lds, st, s, d.m, ds, which_in,
                       which_out, CW, PO, (const TC *)T, ldt, (TC *)Yout, (TC *)Yout1, (int)vec_ok(s, d.m), tri);
}

hipError_t launch_gemm_tall(const GemmDesc &d, const DevState *ds, int32_t which_in, int32_t which_out,
                            int32_t pin_max, int32_t pout_max, const void *T, int32_t ldt, void *Yout, void *Yout1,
                            hipStream_t st, int32_t tri)
{
    if (pin_max > PMAX_WIDE || pout_max > PMAX_WIDE) return hipErrorInvalidValue;
    ProfScope ps(POD_K_TALL, st);
    const int64_t nst = (d.m + RB - 1) / RB;
    const int PI = (pin_max + 15) & ~15, PO = (pout_max + 15) & ~15;
    const bool wide = PI > 64;
    if (!wide && PO > 64) return hipErrorInvalidValue;   // the narrow class holds 4 column tiles
    const int stw = wide ? TALL_ST_WIDE : TALL_ST;
    const unsigned nb = (unsigned)((nst + stw - 1) / stw);
    if (d.prec == POD_BF16_REFINE) {
        if (d.a_dtype != POD_F32 || !d.tsplit) return hipErrorInvalidValue;
        const int KP = (pin_max + 31) & ~31, JP = PO;
        __bf16 *Tb = reinterpret_cast<__bf16 *>(d.tsplit);
        hipLaunchKernelGGL(k_split_t, dim3((JP * KP + 255) / 256), dim3(256), 0, st, (const float *)T, ldt, ds,
                           which_in, which_out, KP, JP, Tb, d.guard);
        const SrcT<float> s = make_src<float>(d);
        const int vout = (d.m % 4 == 0) && ((uintptr_t)Yout % 16 == 0) && ((uintptr_t)Yout1 % 16 == 0);
        if (KP <= 64 && JP <= 64)
            tall_bf16_direct_launch<2, 4>(s, d.m, ds, which_in, which_out, Tb, KP, JP, Yout, Yout1, vout, tri, st);
        else
            tall_bf16_direct_launch<5, 10>(s, d.m, ds, which_in, which_out, Tb, KP, JP, Yout, Yout1, vout, tri, st);
    } else if (d.prec == POD_F64) {
        // (inputs up to 64 wide: the staged kernel below is faster there, with
        // little work per loaded element)
        if (wide && PO <= 64) {
            tall64_launch<10, 4, false>(d, ds, which_in, which_out, T, ldt, Yout, Yout1, tri, st);
            return hipGetLastError();
        }
        if (wide && tri && PI == PO) {
            tall64_launch<10, 10, true>(d, ds, which_in, which_out, T, ldt, Yout, Yout1, tri, st);
            return hipGetLastError();
        }
        const bool tg = (size_t)PI * PO * sizeof(double) > TALL_T_LDS;
        // an upper-triangular square T packs into LDS beside the stage
        const bool tp = tg && tri && PI == PO &&
                        (size_t)(ITEMS160 * 256 / GRP * LDSR + tri_tiles(PO / 16) * 256) * sizeof(double) <=
                            (size_t)TALL_DYN_LDS;
        if (!wide) tall_launch<double, ITEMS64, false>(d, ds, which_in, which_out, PI, PO, T, ldt, Yout, Yout1, nb, tri, st);
        else if (!tg) tall_launch<double, ITEMS160, false>(d, ds, which_in, which_out, PI, PO, T, ldt, Yout, Yout1, nb, tri, st);
        else if (tp) tall_launch<double, ITEMS160, false, true>(d, ds, which_in, which_out, PI, PO, T, ldt, Yout, Yout1, nb, tri, st);
        else tall_launch<double, ITEMS160, true>(d, ds, which_in, which_out, PI, PO, T, ldt, Yout, Yout1, nb, tri, st);
    } else {
        const bool tg = (size_t)PI * PO * sizeof(float) > TALL_T_LDS;
        if (!wide) tall_launch<float, ITEMS64, false>(d, ds, which_in, which_out, PI, PO, T, ldt, Yout, Yout1, nb, tri, st);
        else if (!tg) tall_launch<float, ITEMS160, false>(d, ds, which_in, which_out, PI, PO, T, ldt, Yout, Yout1, nb, tri, st);
        else tall_launch<float, ITEMS160, true>(d, ds, which_in, which_out, PI, PO, T, ldt, Yout, Yout1, nb, tri, st);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Projection B = U^T A (r x n), one pass over A.  Workgroup (split, column
// block of 64) covers row stages [ns s / nsplit, ns (s+1) / nsplit) of 64
// columns of A; wave w owns 16 of those columns and all ceil(r/16) mode
// tiles.  The linear block index is remapped so that all column blocks of
// one row split run on the same XCD (workgroups are dealt round-robin to the
// 8 XCDs), where they share that split's rows of U in L2.
// ---------------------------------------------------------------------------
constexpr int PCB = 64;  // columns of A per workgroup

template <typename TC, typename TA, int MT, int UITEMS>
__global__ __launch_bounds__(256) void k_project_partial(const TC *__restrict__ U, const TA *__restrict__ A,
                                                         int64_t m, int64_t n, int64_t lda, int r, int nsplit,
                                                         int ncb, double *__restrict__ Bpart, int vec,
                                                         const TC *__restrict__ U1, const DevState *ds)
{
    typedef typename Acc<TC>::type AccT;
    extern __shared__ unsigned char lds_raw[];
    const int RP = (r + 15) & ~15;
    // device-selected basis (ORT weights during the loop): the live rank, the
    // current buffer, nothing on the first iteration or after the stop
    int rl = r;
    if (ds) {
        if (ds->it == 0 || merge_halted(ds)) return;
        rl = (ds->rs < r) ? ds->rs : r;
        if (U1 && (ds->it & 1)) U = U1;
    }
    TC *As = reinterpret_cast<TC *>(lds_raw);   // PCB x LDSR
    TC *Us = As + PCB * LDSR;                   // RP x LDSR
    const int total = nsplit * ncb;
    const int id = blockIdx.x;
    int sidx, cb;
    if (total % 8 == 0 && nsplit % 8 == 0) {
        const int xcd = id % 8, local = id / 8;
        const int spx = nsplit / 8;
        sidx = xcd * spx + local / ncb;
        cb = local % ncb;
    } else {
        sidx = id / ncb;
        cb = id % ncb;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nst = (m + RB - 1) / RB;
    const int64_t s0 = (nst * sidx) / nsplit, s1 = (nst * (sidx + 1)) / nsplit;
    const int64_t c0 = (int64_t)cb * PCB;
    const int ncol = (n - c0 < PCB) ? (int)(n - c0) : PCB;
    SrcT<TC> su;
    su.U = nullptr;
    su.U1 = nullptr;
    su.Z = nullptr;
    su.g = 0;
    su.A = nullptr;
    su.lda = 0;
    su.cols = nullptr;
    su.Y = U;
    su.gather = 0;
    su.a_f64 = 0;
    su.rs = 0;
    su.guard = 0;
    AccT acc[MT];   // MT mode tiles: r <= 16 MT
#pragma unroll
    for (int q = 0; q < MT; ++q) acc[q] = AccT{0, 0, 0, 0};
    // A stage: 64 columns x 8 groups = 512 items; U stage: RP columns x 8 groups <= 256 UITEMS items;
    // two register stages in flight (stages sg + 1 and sg + 2 load while sg is on the matrix cores)
    // A's stage is held in its storage type and widened at the LDS store: a
    // value converted inside a branch would be waited for there, and with it
    // the other stage's loads.  Columns past n read column 0 and are stored as
    // zeros.
    TA ast[2][2][4];
    Stage<TC, UITEMS> stu[2];
    const TA *Ab = A + c0 * lda;
    // a full stage of A (r0 + RB <= m, aligned): vector loads with no branch
    auto loadA_full = [&](int64_t sg, TA (&st)[2][4]) {
        const int64_t r0 = sg * RB;
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int idx = threadIdx.x + 256 * it;
            const int c = idx / GRP, g = idx % GRP;
            const TA *p = Ab + (int64_t)((c < ncol) ? c : 0) * lda + r0 + 4 * g;
            if (sizeof(TA) == 4) {
                const f32x4 a = *reinterpret_cast<const f32x4 *>(p);
#pragma unroll
                for (int q = 0; q < 4; ++q) st[it][q] = (TA)a[q];
            } else {
                const f64x2 a = *reinterpret_cast<const f64x2 *>(p);
                const f64x2 b = *reinterpret_cast<const f64x2 *>(p + 2);
                st[it][0] = (TA)a[0];
                st[it][1] = (TA)a[1];
                st[it][2] = (TA)b[0];
                st[it][3] = (TA)b[1];
            }
        }
    };
    // any stage (the partial last one, or unaligned data): element loads
    auto loadA = [&](int64_t sg, TA (&st)[2][4]) {
        const int64_t r0 = sg * RB;
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int idx = threadIdx.x + 256 * it;
            const int c = idx / GRP, g = idx % GRP;
            const TA *p = Ab + (int64_t)((c < ncol) ? c : 0) * lda + r0 + 4 * g;
#pragma unroll
            for (int q = 0; q < 4; ++q) st[it][q] = (r0 + 4 * g + q < m) ? p[q] : (TA)0;
        }
    };
    auto storeA = [&](const TA (&st)[2][4]) {
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int idx = threadIdx.x + 256 * it;
            const int c = idx / GRP, g = idx % GRP;
#pragma unroll
            for (int q = 0; q < 4; ++q) As[c * LDSR + 4 * g + q] = (c < ncol) ? (TC)st[it][q] : (TC)0;
        }
    };
    stu[0].prepare(su, m, rl, vec);
    stu[1].fast = stu[0].fast;
    stu[1].f32col = stu[0].f32col;
#pragma unroll
    for (int it = 0; it < UITEMS; ++it) stu[1].base[it] = stu[0].base[it];
    // (k-chunk outer, mode tiles inner: independent chains alternate; each
    // tile still sums its k in order)
    auto compute = [&]() {
        const TC *xb = As + (wv * 16 + (lane & 15)) * LDSR + (lane >> 4);
#pragma unroll
        for (int k4 = 0; k4 < RB; k4 += 4)
#pragma unroll
            for (int q = 0; q < MT; ++q)
                if (q * 16 < RP) {
                    const TC *ua = Us + (q * 16 + (lane & 15)) * LDSR + (lane >> 4);
                    acc[q] = mfma16x16x4(ua[k4], xb[k4], acc[q]);
                }
    };
    // full stages [s0, e) on the fast path: two register stages in flight,
    // every load issued with no branch around it (the prefetch index clamped
    // to the last full stage, so every iteration issues the same loads; a
    // load inside a branch would be waited for where the branch ends)
    const int64_t full_end = m / RB;
    const bool fast = vec && stu[0].fast;
    const int64_t e = fast ? ((s1 < full_end) ? s1 : ((full_end > s0) ? full_end : s0)) : s0;
    if (e > s0) {
        const int64_t last = e - 1;
        loadA_full(s0, ast[0]);
        stu[0].load_full(s0 * RB);
        const int64_t s1n = (s0 + 1 < last) ? s0 + 1 : last;
        loadA_full(s1n, ast[1]);
        stu[1].load_full(s1n * RB);
        int64_t sg = s0;
        for (; sg + 1 < e; sg += 2) {
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                __syncthreads();
                storeA(ast[b]);
                stu[b].store(Us, RP, rl);
                __syncthreads();
                const int64_t nx = (sg + b + 2 < last) ? sg + b + 2 : last;
                loadA_full(nx, ast[b]);
                stu[b].load_full(nx * RB);
                compute();
            }
        }
        if (sg < e) {
            __syncthreads();
            storeA(ast[0]);
            stu[0].store(Us, RP, rl);
            __syncthreads();
            compute();
        }
    }
    // the remaining stages one at a time (a partial last stage, or every
    // stage off the fast path)
    for (int64_t sg = e; sg < s1; ++sg) {
        loadA(sg, ast[0]);
        stu[0].load(su, m, sg * RB, rl, vec);
        __syncthreads();
        storeA(ast[0]);
        stu[0].store(Us, RP, rl);
        __syncthreads();
        compute();
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

template <typename TC, typename TA, int MT, int UITEMS>
static void project_launch(const ProjArgs &a, unsigned total, int ncb, int vec, hipStream_t st)
{
    const int RP = (a.r + 15) & ~15;
    const size_t lds = (size_t)(PCB + RP) * LDSR * sizeof(TC);
    hipLaunchKernelGGL((k_project_partial<TC, TA, MT, UITEMS>), dim3(total), dim3(256), lds, st, (const TC *)a.U,
                       (const TA *)a.A, a.m, a.n, a.lda, a.r, a.nsplit, ncb, a.Bpart, vec, (const TC *)a.U1, a.ds);
}

hipError_t launch_project_partial(const ProjArgs &a, hipStream_t st)
{
    if (a.r > PMAX_WIDE) return hipErrorInvalidValue;
    if (a.prec != POD_F64 && a.a_dtype == POD_F64) return hipErrorInvalidValue;
    const int ncb = (int)((a.n + PCB - 1) / PCB);
    const unsigned total = (unsigned)(a.nsplit * ncb);
    ProfScope ps(POD_K_PROJECT, st);
    const size_t ae = (a.a_dtype == POD_F64) ? 8 : 4;
    const size_t ce = (a.prec == POD_F64) ? 8 : 4;
    const int vec = ((uintptr_t)a.A % 16 == 0) && ((a.lda * ae) % 16 == 0) && ((uintptr_t)a.U % 16 == 0) &&
                    ((uintptr_t)a.U1 % 16 == 0) && ((a.m * ce) % 16 == 0);
    const bool wide = a.r > 64;
    if (a.prec == POD_F64) {
        if (a.a_dtype == POD_F64) {
            if (wide) project_launch<double, double, 10, ITEMS160>(a, total, ncb, vec, st);
            else project_launch<double, double, 4, ITEMS64>(a, total, ncb, vec, st);
        } else {
            if (wide) project_launch<double, float, 10, ITEMS160>(a, total, ncb, vec, st);
            else project_launch<double, float, 4, ITEMS64>(a, total, ncb, vec, st);
        }
    } else {
        if (wide) project_launch<float, float, 10, ITEMS160>(a, total, ncb, vec, st);
        else project_launch<float, float, 4, ITEMS64>(a, total, ncb, vec, st);
    }
    return hipGetLastError();
}

hipError_t launch_project_reduce(const ProjArgs &a, hipStream_t st)
{
    const int64_t rn = (int64_t)a.r * a.n;
    ProfScope ps(POD_K_PROJECT, st);
    hipLaunchKernelGGL(k_project_reduce, dim3((unsigned)((rn + 255) / 256)), dim3(256), 0, st, a.Bpart, rn,
                       a.nsplit, a.B);
    return hipGetLastError();
}

// ---------------------------------------------------------------- batched launches

int32_t gemm_vec_ok(const GemmDesc &d)
{
    if (d.prec == POD_F64) return (int32_t)vec_ok(make_src<double>(d), d.m);
    return (int32_t)vec_ok(make_src<float>(d), d.m);
}

int32_t tall_blocks(int64_t m)
{
    const int64_t nst = (m + RB - 1) / RB;
    return (int32_t)((nst + TALL_ST - 1) / TALL_ST);
}

hipError_t launch_gram_partial_b(const GramArgs *arr, int32_t count, int32_t max_nblk, int32_t pmax_max, int32_t prec,
                                 hipStream_t st)
{
    if (pmax_max > 64 || count < 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)max_nblk, (unsigned)count);
    if (prec == POD_F64)
        hipLaunchKernelGGL(k_gram_direct_b<double>, grid, dim3(512), GD_LDS, st, arr);
    else
        hipLaunchKernelGGL(k_gram_direct_b<float>, grid, dim3(512), GD_LDS, st, arr);
    return hipGetLastError();
}

hipError_t launch_gram_reduce_b(const GramArgs *arr, int32_t count, int32_t pmax_max, hipStream_t st)
{
    if (count < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gram_reduce_b, dim3((unsigned)((pmax_max * pmax_max + 63) / 64), (unsigned)count),
                       dim3(64 * GR_W), 0, st, arr);
    return hipGetLastError();
}

hipError_t launch_gemm_tall_b(const TallArgs *arr, int32_t count, int32_t max_nb, int32_t pi_max, int32_t po_max,
                              int32_t prec, hipStream_t st)
{
    if (pi_max > 64 || po_max > 64 || count < 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)max_nb, (unsigned)count);
    if (prec == POD_F64)
        hipLaunchKernelGGL((k_gemm_tall_b<double, ITEMS64>), grid, dim3(256),
                           (size_t)(64 * LDSR + pi_max * po_max) * sizeof(double), st, arr);
    else
        hipLaunchKernelGGL((k_gemm_tall_b<float, ITEMS64>), grid, dim3(256),
                           (size_t)(64 * LDSR + pi_max * po_max) * sizeof(float), st, arr);
    return hipGetLastError();
}

hipError_t launch_gemm_tall_scatter_b(const ScatterArgs *arr, int32_t count, int32_t max_nb, int32_t pi_max,
                                      int32_t po_max, int32_t prec, hipStream_t st)
{
    const int PI = (pi_max + 15) & ~15, PO = (po_max + 15) & ~15;
    if (PI > 64 || PO > 64 || count < 1) return hipErrorInvalidValue;
    const size_t esz = (prec == POD_F64) ? 8 : 4;
    const size_t lds = (size_t)(64 * LDSR + PI * PO) * esz;
    const dim3 grid((unsigned)max_nb, (unsigned)count);
    if (prec == POD_F64)
        hipLaunchKernelGGL(k_gemm_tall_scatter_b<double>, grid, dim3(256), lds, st, arr);
    else
        hipLaunchKernelGGL(k_gemm_tall_scatter_b<float>, grid, dim3(256), lds, st, arr);
    return hipGetLastError();
}

hipError_t launch_gemm_tall_scatter(const GemmDesc &d, const DevState *ds, int32_t which_in, int32_t which_out,
                                    int32_t pin_max, int32_t pout_max, const void *T, int32_t ldt, void *Yout,
                                    int32_t split, const int32_t *cmap, void *D, int64_t ldd, hipStream_t st)
{
    const int PI = (pin_max + 15) & ~15, PO = (pout_max + 15) & ~15;
    const size_t esz = (d.prec == POD_F64) ? 8 : 4;
    if (PI > PMAX_ADJ || PO > PMAX_WIDE) return hipErrorInvalidValue;
    if (d.prec == POD_F32 && PI > PMAX_WIDE) {
        // the FP32 path on the same kernel: every column read as FP32 (or
        // FP64 for an FP64 A) and widened, T widened into LDS, FP64 products
        if (which_in < 0 || which_out < 0 || which_out > pout_max || which_in > pin_max) return hipErrorInvalidValue;
        const TallScatter sc{split, cmap, D, ldd};
        return tall64_scatter_launch<13, 5, true, float>(d, ds, which_in, which_out, pout_max, (const float *)T, ldt,
                                                         (float *)Yout, sc, st);
    }
    if (d.prec == POD_F64 && PI > 64 && (PI > PMAX_WIDE || (size_t)PI * PO * esz > TALL_T_LDS)) {
        // X straight into the matrix-core registers, column groups of 80
        // with their slice of T in LDS; the output count is literal
        if (which_in < 0 || which_out < 0 || which_out > pout_max || which_in > pin_max) return hipErrorInvalidValue;
        const TallScatter sc{split, cmap, D, ldd};
        const bool mix = d.gather && d.a_dtype != POD_F64;
        if (PI > PMAX_WIDE)
            return mix ? tall64_scatter_launch<13, 5, true>(d, ds, which_in, which_out, pout_max, (const double *)T,
                                                             ldt, (double *)Yout, sc, st)
                       : tall64_scatter_launch<13, 5, false>(d, ds, which_in, which_out, pout_max, (const double *)T,
                                                              ldt, (double *)Yout, sc, st);
        return mix ? tall64_scatter_launch<10, 4, true>(d, ds, which_in, which_out, pout_max, (const double *)T, ldt,
                                                         (double *)Yout, sc, st)
                   : tall64_scatter_launch<10, 4, false>(d, ds, which_in, which_out, pout_max, (const double *)T, ldt,
                                                          (double *)Yout, sc, st);
    }
    // (the register-operand kernel above takes every T too large for LDS)
    if (PI > PMAX_WIDE || (size_t)PI * PO * esz > TALL_T_LDS) return hipErrorInvalidValue;
    if (PI <= 64 && PO > 64) return hipErrorInvalidValue;   // the narrow class holds 4 column tiles
    const unsigned nb = (unsigned)tall_blocks(d.m);
    const TallScatter sc{split, cmap, D, ldd};
    const int CW = (PI > 64) ? 160 : 64;   // columns of the LDS stage of the tile class
    const size_t lds = (size_t)(CW * LDSR + PI * PO) * esz;
    if (d.prec == POD_F64) {
        const SrcT<double> s = make_src<double>(d);
        if (PI > 64) {
            static bool attr = false;
            if (!attr) {
                if (hipFuncSetAttribute((const void *)k_gemm_tall_scatter<double, ITEMS160>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, TALL_DYN_LDS) != hipSuccess)
                    return hipErrorInvalidValue;
                attr = true;
            }
            hipLaunchKernelGGL((k_gemm_tall_scatter<double, ITEMS160>), dim3(nb), dim3(256), lds, st, s, d.m, ds,
                               which_in, which_out, CW, (const double *)T, ldt, (double *)Yout, sc,
                               (int)vec_ok(s, d.m));
        } else {
            hipLaunchKernelGGL((k_gemm_tall_scatter<double, ITEMS64>), dim3(nb), dim3(256), lds, st, s, d.m, ds,
                               which_in, which_out, CW, (const double *)T, ldt, (double *)Yout, sc,
                               (int)vec_ok(s, d.m));
        }
    } else {
        const SrcT<float> s = make_src<float>(d);
        if (PI > 64) {
            static bool attr = false;
            if (!attr) {
                if (hipFuncSetAttribute((const void *)k_gemm_tall_scatter<float, ITEMS160>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, TALL_DYN_LDS) != hipSuccess)
                    return hipErrorInvalidValue;
                attr = true;
            }
            hipLaunchKernelGGL((k_gemm_tall_scatter<float, ITEMS160>), dim3(nb), dim3(256), lds, st, s, d.m, ds,
                               which_in, which_out, CW, (const float *)T, ldt, (float *)Yout, sc,
                               (int)vec_ok(s, d.m));
        } else {
            hipLaunchKernelGGL((k_gemm_tall_scatter<float, ITEMS64>), dim3(nb), dim3(256), lds, st, s, d.m, ds,
                               which_in, which_out, CW, (const float *)T, ldt, (float *)Yout, sc,
                               (int)vec_ok(s, d.m));
        }
    }
    return hipGetLastError();
}

}  // namespace pod

"""Pins of the oracle's sampling strategies, row centring, the mode criterion,
the sample-size formulas and the one-shot sampled SVDs of Appendix A.

CPU only.  Each expected value comes from a closed form, from Python integers
driven by numpy's Philox (an implementation independent of the oracle's), from
a construction whose answer is known exactly, or from LAPACK through numpy.
"""
import math

import numpy as np
import pytest

import oracle
import snapgen
from oracle import oneshot
from oracle.isma import (IsmaParams, center_rows, isma, ls_row_weights, mode_sines, ort_col_weights,
                         sample_size_ctsvd, sample_size_ltsvd)

U64 = 2.0 ** -53


def _philox_words(counter, key):
    """Philox-4x64-10 block from numpy (it pre-increments its counter)."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(counter))
    c = (c - 1) % (1 << 256)
    start = np.array([(c >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=start)
    return [int(x) for x in bg.random_raw(4)]


def _u(seed, stream, it, d, block=0):
    """Word d mod 4 of the block of draw d at iteration it."""
    return _philox_words((it, d // 4, block, 0), (seed, stream))[d % 4]


def _inverse_cdf(weights, u):
    """Python integers: first j with F_j > floor(u W / 2^64)."""
    W = sum(int(x) for x in weights)
    t = (u * W) >> 64
    run = 0
    for j, x in enumerate(weights):
        run += int(x)
        if run > t:
            return j
    raise AssertionError("target beyond the total weight")


def _distinct(draws):
    vals = sorted(set(draws))
    return np.array(vals), np.array([draws.count(v) for v in vals])


# ------------------------------------------------------------------ row centring (Sec. 1)

def test_center_rows_exact_on_integers():
    rng = np.random.default_rng(3)
    n = 8
    A = rng.integers(-50, 50, size=(301, n)).astype(np.float64)
    # rows whose sum is a multiple of 1/8: every mean is a dyadic rational,
    # every difference exact
    Ac, mean = center_rows(A)
    want_mean = np.array([sum(int(x) for x in row) / n for row in A])
    assert np.array_equal(mean, want_mean)
    assert np.array_equal(Ac, A - want_mean[:, None])
    assert np.all(Ac.sum(axis=1) == 0.0)


def test_center_rows_fp32_rounds_once():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((500, 37)).astype(np.float32)
    Ac, mean = center_rows(A)
    assert Ac.dtype == np.float32
    exact_mean = np.array([math.fsum(float(x) for x in row) / 37 for row in A])
    assert np.max(np.abs(mean - exact_mean)) <= 64 * U64 * np.max(np.abs(A))
    # one rounding of the FP64 difference to FP32
    assert np.array_equal(Ac, (A.astype(np.float64) - mean[:, None]).astype(np.float32))


def test_center_rows_keeps_spectrum_of_mean_free_part():
    s = np.array([3.0, 1.0, 0.5])
    sm = snapgen.spectrum_matrix(200, 40, s, 0.0, 8, centre=False)
    shifted = sm.A + np.linspace(-2.0, 2.0, 200)[:, None]   # add a row offset
    Ac, mean = center_rows(shifted)
    assert np.allclose(mean, np.linspace(-2.0, 2.0, 200), atol=1e-14)
    sv = np.linalg.svd(Ac, compute_uv=False)
    assert np.max(np.abs(sv[:3] - s) / s) < 1e-13 and sv[3] < 1e-13


# ------------------------------------------------------------------ mode criterion (Alg. 1)

def test_mode_sines_closed_form_rotations_and_sign():
    m, k = 40, 4
    thetas = [1e-12, 1e-7, 0.3, 1.2]
    Uold = np.eye(m)[:, :k]
    Unew = np.zeros((m, k))
    for i, th in enumerate(thetas):
        Unew[i, i] = math.cos(th)
        Unew[k + i, i] = math.sin(th)
    Unew[:, 2] *= -1.0                       # a sign flip changes nothing
    got = mode_sines(Uold, Unew)
    assert np.allclose(got, np.sin(thetas), rtol=1e-12, atol=1e-17)


def test_mode_and_subspace_criteria_differ_on_a_swap():
    m, k = 30, 3
    Uold = np.eye(m)[:, :k]
    Unew = Uold[:, [1, 0, 2]]
    assert np.allclose(mode_sines(Uold, Unew), [1.0, 1.0, 0.0], atol=1e-15)
    assert oracle.subspace_sines(Uold, Unew).max() < 1e-15


# ------------------------------------------------------------------ UNF columns

def test_unf_draws_are_uniform_over_S():
    """From the second iteration UNF ignores the norms: each draw is
    S_sorted[floor(u |S| / 2^64)]."""
    rng = np.random.default_rng(9)
    A = rng.standard_normal((60, 50))
    A[:, 7] *= 1e6          # L2N would draw column 7 every time
    prm = IsmaParams(k=3, c=6, seed=77, col_strategy="unf", theta_tol=0.0)
    res = isma(A, prm, n_iter=5, final_step=False)
    S = set(range(50))
    for t, lg in enumerate(res.log):
        if t > 0:
            Ss = sorted(S)
            draws = [Ss[(_u(77, 0, t, d) * len(Ss)) >> 64] for d in range(prm.c)]
            cols, cnt = _distinct(draws)
            assert np.array_equal(lg.cols, cols) and np.array_equal(lg.col_counts, cnt)
        S -= set(int(j) for j in lg.cols)


# ------------------------------------------------------------------ LS rows

def test_ls_weights_use_the_first_k_columns_only():
    m, r, k = 50, 5, 3
    rows = [4, 17, 33, 40, 45]
    U = np.zeros((m, r))
    for l, i in enumerate(rows):
        U[i, l] = 1.0
    q = ls_row_weights(U, k)
    want = np.zeros(m)
    want[rows[:k]] = 1.0
    assert np.array_equal(q, want)
    wr = oracle.quantize(q)
    assert set(np.flatnonzero(wr)) == set(rows[:k]) and len(set(wr[rows[:k]])) == 1


def test_ls_rows_follow_the_current_state():
    """Rows drawn at iteration t >= 1 follow |u^i|^2 of the first k columns of
    the state after t merges (Python-integer inverse CDF on its weights)."""
    sm = snapgen.spectrum_matrix(300, 80, np.exp(-np.arange(20) / 4.0), 1e-6, 5, centre=True)
    prm = IsmaParams(k=3, c=8, w=40, r=6, seed=21, row_strategy="ls", theta_tol=0.0)
    full = isma(sm.A, prm, n_iter=4, final_step=False)
    for t in range(1, 4):
        state = isma(sm.A, prm, n_iter=t, final_step=False).U_merge
        rho = np.array([sum(float(state[i, l]) ** 2 for l in range(3)) for i in range(300)])
        wr = oracle.quantize(rho)
        draws = [_inverse_cdf(wr, _u(21, 1, t, d)) for d in range(prm.w)]
        rows, cnt = _distinct(draws)
        assert np.array_equal(full.log[t].rows, rows) and np.array_equal(full.log[t].row_counts, cnt)
        # the stale state or all r columns would draw other rows
        rho_r = np.sum(state ** 2, axis=1)
        draws_r = [_inverse_cdf(oracle.quantize(rho_r), _u(21, 1, t, d)) for d in range(prm.w)]
        assert draws_r != draws


# ------------------------------------------------------------------ ORT columns

def test_ort_weights_closed_form():
    """Integer A and a state of unit vectors: the residual of column i is A
    with the state's rows zeroed, so |a_i - U U^T a_i|^2 is an integer sum.
    Every column of the state counts, columns outside S get 0."""
    rng = np.random.default_rng(12)
    m, n = 40, 9
    A = rng.integers(-9, 10, size=(m, n)).astype(np.float64)
    rows = [2, 11, 30]
    U = np.zeros((m, 3))
    for l, i in enumerate(rows):
        U[i, l] = 1.0
    inS = np.ones(n, dtype=bool)
    inS[[1, 5]] = False
    rho = ort_col_weights(A, U, inS)
    keep = [i for i in range(m) if i not in rows]
    want = np.array([sum(int(A[i, j]) ** 2 for i in keep) if inS[j] else 0 for j in range(n)], dtype=np.float64)
    assert np.array_equal(rho, want)


def test_ort_draws_follow_the_current_residuals():
    rng = np.random.default_rng(13)
    sm = snapgen.spectrum_matrix(200, 90, np.exp(-np.arange(30) / 5.0), 1e-5, 6, centre=True)
    A = sm.A
    prm = IsmaParams(k=4, c=10, r=6, seed=31, col_strategy="ort", theta_tol=0.0)
    full = isma(A, prm, n_iter=4, final_step=False)
    inS = np.ones(90, dtype=bool)
    inS[full.log[0].cols] = False
    for t in range(1, 4):
        state = isma(A, prm, n_iter=t, final_step=False).U_merge
        rho = np.zeros(90)
        for i in np.flatnonzero(inS):
            # the residual's squared norm through an orthonormal complement (LAPACK)
            Qc = np.linalg.svd(np.eye(200) - state @ state.T)[0][:, :200 - state.shape[1]]
            rho[i] = float(np.sum((Qc.T @ A[:, i]) ** 2))
        assert np.allclose(ort_col_weights(A, state, inS), rho, rtol=1e-10, atol=1e-14)
        wq = oracle.quantize(ort_col_weights(A, state, inS))
        draws = [_inverse_cdf(wq, _u(31, 0, t, d)) for d in range(prm.c)]
        cols, cnt = _distinct(draws)
        assert np.array_equal(full.log[t].cols, cols)
        assert all(inS[j] for j in cols)
        inS[cols] = False


def test_ort_exhausts_when_the_state_explains_every_column():
    s = np.array([2.0, 1.0])
    sm = snapgen.spectrum_matrix(100, 30, s, 0.0, 2, centre=True)
    res = isma(sm.A, IsmaParams(k=2, c=40, r=2, seed=1, col_strategy="ort", theta_tol=0.0))
    # the first draw (norm weights) already spans the rank-2 column space
    assert res.exhausted and len(res.log) == 1
    assert np.max(np.abs(res.sigma - s) / s) < 1e-12


# ------------------------------------------------------------------ sample sizes, Eqs. (c_LTSVD), (c_w_CTSVD)

# hand-derived: c = 4k (1 + sqrt(8 ln(1/delta)))^2 / eps^2 and
# c = w = k^2 (1 + sqrt(ln(2/delta)))^2 / eps^4, rounded up (parameters of the
# paper's tables of LTSVD / CTSVD and iterative-run settings)
LTSVD_TABLE = [((10, 0.7, 0.6), 746), ((2, 0.7, 0.6), 150), ((20, 0.6, 0.6), 2029), ((5, 0.6, 0.6), 508),
               ((10, 1.0, 0.75), 254), ((10, 0.7, 0.45), 1016), ((20, 0.35, 0.35), 9924), ((2, 1.0, 0.8), 44)]
CTSVD_TABLE = [((10, 0.7, 0.6), 1832), ((2, 0.7, 0.6), 74), ((20, 0.6, 0.6), 13576), ((5, 0.6, 0.6), 849),
               ((10, 1.0, 0.75), 397), ((10, 1.04, 0.94), 299), ((5, 1.0, 0.1), 187), ((2, 1.0, 0.8), 16)]


@pytest.mark.parametrize("args,want", LTSVD_TABLE)
def test_sample_size_ltsvd_hand_derived(args, want):
    assert sample_size_ltsvd(*args) == want


@pytest.mark.parametrize("args,want", CTSVD_TABLE)
def test_sample_size_ctsvd_hand_derived(args, want):
    assert sample_size_ctsvd(*args) == want


# ------------------------------------------------------------------ Alg. 4 / Alg. 5

def test_ltsvd_preserves_frobenius_norm_for_every_draw():
    """sum over the draws of |a_s|^2 / (c p_s) = |A|_F^2 exactly when p_s is
    proportional to |a_s|^2: the scaled sample keeps the Frobenius norm (up to
    the quantisation of the weights)."""
    rng = np.random.default_rng(20)
    A = rng.standard_normal((150, 60)) * rng.uniform(0.1, 3.0, size=60)[None, :]
    for seed in (1, 2, 3):
        res = oneshot.ltsvd(A, k=5, c=25, seed=seed)
        C = A[:, res.cols] * res.col_scale[None, :]
        assert abs(np.sum(C * C) / np.sum(A * A) - 1.0) < 1e-12
        assert int(res.col_counts.sum()) == 25


def test_ltsvd_equals_svd_of_the_duplicated_sample():
    rng = np.random.default_rng(21)
    A = rng.standard_normal((120, 30)) * np.exp(-np.arange(30) / 6.0)[None, :]
    c = 40
    res = oneshot.ltsvd(A, k=6, c=c, seed=5)
    # Alg. 4 literally: c columns a_s / sqrt(c p_s), duplicates kept
    nu = oracle.col_sqnorms(A, 8)
    wq = oracle.quantize(nu)
    W = sum(int(x) for x in wq)
    draws = [_inverse_cdf(wq, _u(5, 0, 0, d)) for d in range(c)]
    Cdup = np.stack([A[:, s] / math.sqrt(c * int(wq[s]) / W) for s in draws], axis=1)
    Ul, sl, _ = np.linalg.svd(Cdup, full_matrices=False)
    assert np.max(np.abs(res.sigma - sl[:6]) / sl[:6]) < 1e-12
    assert oracle.subspace_sines(Ul[:, :6], res.U).max() < 1e-10
    assert np.allclose(np.abs(np.sum(Ul[:, :6] * res.U, axis=0)), 1.0, atol=1e-10)


def test_ltsvd_exact_on_low_rank():
    s = np.array([4.0, 2.0, 1.0])
    sm = snapgen.spectrum_matrix(100, 50, s, 0.0, 31, centre=False)
    res = oneshot.ltsvd(sm.A, k=5, c=12, seed=2)
    assert res.l == 3                        # l = min(k, rank C)
    assert oracle.subspace_sines(sm.U, res.U).max() < 1e-11


def test_ctsvd_row_sample_preserves_frobenius_norm_and_equals_duplicated_form():
    rng = np.random.default_rng(22)
    A = rng.standard_normal((200, 40)) * np.exp(-np.arange(40) / 5.0)[None, :]
    c, w, k = 30, 60, 4
    res = oneshot.ctsvd(A, k=k, c=c, w=w, eps=0.5, seed=9)
    C = A[:, res.cols] * res.col_scale[None, :]
    W = C[res.rows, :] * res.row_scale[:, None]
    assert abs(np.sum(W * W) / np.sum(C * C) - 1.0) < 1e-12
    # Alg. 5 literally: w rows c^s / sqrt(w q_s) with duplicates, right vectors
    # of W^T W (LAPACK), u~ = C v~ / sigma~
    wr = oracle.quantize(oracle.row_sqnorms(C))
    Om = sum(int(x) for x in wr)
    rdraws = [_inverse_cdf(wr, _u(9, 1, 0, d)) for d in range(w)]
    Wdup = np.stack([C[i, :] / math.sqrt(w * int(wr[i]) / Om) for i in rdraws], axis=0)
    ev, V = np.linalg.eigh(Wdup.T @ Wdup)
    order = np.argsort(ev)[::-1][:res.l]
    sig = np.sqrt(ev[order])
    U = C @ V[:, order] / sig[None, :]
    assert np.max(np.abs(res.sigma - sig) / sig) < 1e-11
    assert np.allclose(np.abs(np.sum(U * res.U, axis=0) / np.sum(U * U, axis=0)), 1.0, atol=1e-9)


def test_ctsvd_filter_drops_weak_directions():
    """gamma = eps / (100 k): directions with sigma~^2 < gamma |W|_F^2 are cut."""
    s = np.array([1.0, 0.5, 1e-3, 1e-4])
    sm = snapgen.spectrum_matrix(300, 60, s, 0.0, 4, centre=False)
    res = oneshot.ctsvd(sm.A, k=4, c=40, w=200, eps=0.5, seed=3)
    # gamma |W|^2 ~ 0.5/400 * 1.25 ~ 1.6e-3: 1e-6 and 1e-8 fall below, 0.25 does not
    assert res.l == 2


def test_svd_ata_truth_matches_lapack_svd():
    rng = np.random.default_rng(23)
    A = rng.standard_normal((300, 25)) * np.exp(-np.arange(25) / 4.0)[None, :]
    U, s = oneshot.svd_ata(A, 5)
    Ul, sl, _ = np.linalg.svd(A, full_matrices=False)
    assert np.max(np.abs(s - sl[:5]) / sl[:5]) < 1e-12
    assert oracle.subspace_sines(Ul[:, :5], U).max() < 1e-10

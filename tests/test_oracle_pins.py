"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Every test here is CPU-only.  None compares the oracle with itself: each one
checks a closed form, an invariant, an independent implementation (numpy's
Philox, Python integers, LAPACK through numpy/scipy as an outside opinion) or
a bound stated in the paper.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import snapgen
from oracle.isma import (IsmaParams, block_bounds, incremental, isma, sample_and_scale_unique_rows)

U64 = 2.0 ** -53


# ----------------------------------------------------------------- Philox

def _numpy_philox_block(counter, key):
    """Philox-4x64-10 block for `counter` from numpy's implementation.
    numpy increments its 256-bit counter before producing a block, so it is
    started at counter - 1."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(counter))
    c = (c - 1) % (1 << 256)
    start = np.array([(c >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=start)
    return bg.random_raw(4)


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (2001, 0)),
    ((7, 3, 0, 0), (2001, 1)),
    ((2**64 - 1, 5, 9, 2**63), (2**64 - 1, 12345)),
    ((123456789, 987654321, 31, 0), (0xDEADBEEF, 1)),
])
def test_philox_matches_numpy(counter, key):
    got = oracle.philox4x64_10(counter, key)
    want = _numpy_philox_block(counter, key)
    assert np.array_equal(got, want)


# ----------------------------------------------------------------- norms

def test_col_norms_exact_on_integers():
    rng = np.random.default_rng(0)
    A = rng.integers(-1000, 1000, size=(3001, 7)).astype(np.float64)
    nu = oracle.col_sqnorms(A, 8)
    want = np.array([sum(int(x) ** 2 for x in A[:, j]) for j in range(A.shape[1])], dtype=np.float64)
    assert np.array_equal(nu, want)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_col_norms_close_to_exact_sum(dtype):
    rng = np.random.default_rng(1)
    A = rng.standard_normal((5000, 5)).astype(dtype)
    nu = oracle.col_sqnorms(A)
    for j in range(A.shape[1]):
        x = A[:, j].astype(np.float64)
        exact = math.fsum(float(v) * float(v) for v in x) if dtype == np.float32 else \
            math.fsum(math.fsum([float(v) * float(v), 0.0]) for v in x)
        assert abs(nu[j] - exact) <= 8 * U64 * exact


def test_col_norms_documented_pairing_order():
    """Accumulator t holds rows t*V.. first; accumulators pair by XOR of
    their lane index (32 first).  Four small squares that each fall below
    half an ulp of the big square survive only if they are added to one
    another before the big one: placed in lanes 1, 33, 17, 49 (which the
    butterfly combines first) they add one ulp; placed sequentially after
    the big value inside one accumulator they vanish."""
    e = 30
    big, small = 2.0 ** e, 2.0 ** (e - 27)       # big^2 = 2^60, small^2 = 2^6 = ulp(2^60)/4
    V = 4                                        # FP32 storage -> 4 values per vector
    m = 4096
    x = np.zeros(m, dtype=np.float32)
    x[0] = big
    for lane in (1, 33, 17, 49):
        x[lane * V] = small
    nu = oracle.col_sqnorms(x[:, None], 4)[0]
    assert nu == 2.0 ** 60 + 2.0 ** 8
    y = np.zeros(m, dtype=np.float32)
    y[0] = big
    y[1:4] = small                               # rows 1..3: same accumulator, same step
    y[256 * V] = small                           # accumulator 0, next step
    nu2 = oracle.col_sqnorms(y[:, None], 4)[0]
    assert nu2 == 2.0 ** 60


def test_row_norms_sequential_exact_small_ints():
    D = np.array([[1.0, 2.0, 3.0], [0.0, 0.0, 0.0], [-4.0, 0.5, 2.0]])
    assert np.array_equal(oracle.row_sqnorms(D), np.array([14.0, 0.0, 20.25]))


# ----------------------------------------------------------------- weights / draws

def test_quantize_closed_form():
    w = oracle.quantize(np.array([1.0, 0.5, 0.25, 0.0]))
    # n = 4 -> B = 61; max = 1 = 0.5 * 2^1 -> e = 1 -> w = nu * 2^59
    assert list(map(int, w)) == [2**59, 2**58, 2**57, 0]


def test_quantize_sum_bound_and_errors():
    rng = np.random.default_rng(3)
    for n in (1, 2, 3, 1000, 16000, 2_000_000):
        v = rng.random(n) * 10.0 ** rng.integers(-30, 30)
        w = oracle.quantize(v)
        assert int(w.astype(object).sum()) < 2**62
        assert int(w.max()) >= 2 ** (63 - math.ceil(math.log2(n)) - 2) if n > 1 else True
    with pytest.raises(ValueError):
        oracle.quantize(np.array([1.0, np.nan]))
    with pytest.raises(ValueError):
        oracle.quantize(np.array([1.0, -1.0]))
    assert int(oracle.quantize(np.zeros(5)).sum()) == 0


@pytest.mark.parametrize("weights", [[3, 0, 5, 2], [1], [0, 0, 7], [2**61, 1, 0, 2**60 + 3]])
def test_draw_matches_python_integer_inverse_cdf(weights):
    """Independent re-derivation: numpy Philox words, Python big integers,
    and a linear scan for the first F_j > t."""
    w = np.array(weights, dtype=np.uint64)
    seed, stream, it, block = 99, 0, 5, 2
    got, W = oracle.draw(w, 37, seed, stream, it, block)
    F = np.cumsum([int(x) for x in weights], dtype=object)
    assert W == int(F[-1])
    for d in range(37):
        u = int(_numpy_philox_block((it, d // 4, block, 0), (seed, stream))[d % 4])
        t = (u * W) >> 64
        j = next(i for i, f in enumerate(F) if f > t)
        assert got[d] == j
        assert weights[j] > 0


def test_draw_frequencies_follow_weights():
    w = np.array([1, 0, 2, 4, 1], dtype=np.uint64)
    counts = np.zeros(5)
    N = 0
    for it in range(400):
        d, _ = oracle.draw(w, 64, 7, 0, it)
        counts += np.bincount(d, minlength=5)
        N += 64
    p = w / w.sum()
    assert counts[1] == 0
    chi2 = sum((counts[i] - N * p[i]) ** 2 / (N * p[i]) for i in range(5) if p[i] > 0)
    assert chi2 < 20.0        # 3 d.o.f.: P(chi2 > 20) < 2e-4


def test_unique_counts():
    d = np.array([5, 1, 5, 9, 1, 5])
    u, c = oracle.unique(d)
    uu, cc = np.unique(d, return_counts=True)
    assert np.array_equal(u, uu) and np.array_equal(c, cc)


def test_row_scaling_equals_duplicate_rows():
    """SAMPLE AND SCALE UNIQUE ROWS: scaling the distinct rows by
    sqrt(t_hat / (w q)) gives the same W^T W as keeping every drawn row
    scaled by 1 / sqrt(w q)."""
    rng = np.random.default_rng(11)
    D = rng.standard_normal((30, 6))
    wr = oracle.quantize(oracle.row_sqnorms(D))
    w = 200
    rows, tcnt, W = sample_and_scale_unique_rows(D, wr, w, 5, 0)
    assert tcnt.sum() == w and tcnt.max() > 1
    draws, _ = oracle.draw(wr, w, 5, 1, 0)
    q = wr.astype(np.float64) / float(int(wr.astype(object).sum()))
    Wdup = D[draws, :] / np.sqrt(w * q[draws])[:, None]
    G1, G2 = W.T @ W, Wdup.T @ Wdup
    assert np.max(np.abs(G1 - G2)) <= 1e-13 * np.max(np.abs(G2))


# ----------------------------------------------------------------- dense kernels

@pytest.mark.parametrize("m,p", [(7, 7), (50, 9), (300, 40)])
def test_householder_qr(m, p):
    rng = np.random.default_rng(m * p)
    X = rng.standard_normal((m, p))
    Q, R = oracle.householder_qr(X)
    assert np.allclose(np.tril(R, -1), 0.0)
    assert np.linalg.norm(Q.T @ Q - np.eye(p)) <= 50 * p * U64
    assert np.linalg.norm(Q @ R - X) <= 50 * p * U64 * np.linalg.norm(X)
    _, Rl = np.linalg.qr(X)                         # outside opinion (LAPACK)
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rl)), rtol=1e-12)


def test_householder_rank_deficient():
    X = np.zeros((10, 3))
    X[:, 0] = 1.0
    X[:, 2] = 2.0
    Q, R = oracle.householder_qr(X)
    assert np.linalg.norm(Q @ R - X) < 1e-14


def test_jacobi_svd_closed_forms():
    U, s, V = oracle.jacobi_svd(np.diag([3.0, -5.0, 1.0]))
    assert np.allclose(s, [5, 3, 1], rtol=0, atol=1e-15)
    # [[a, b], [0, d]] with a = d: singular values |a| +- |b|/2 ... use the general formula
    a, b, d = 2.0, 1.0, 3.0
    M = np.array([[a, b], [0.0, d]])
    S2 = a * a + b * b + d * d
    disc = math.sqrt(S2 * S2 - 4 * (a * d) ** 2)
    want = [math.sqrt((S2 + disc) / 2), math.sqrt((S2 - disc) / 2)]
    _, s2, _ = oracle.jacobi_svd(M)
    assert np.allclose(s2, want, rtol=1e-15)


@pytest.mark.parametrize("rows,cols", [(30, 30), (150, 150), (400, 25), (60, 60)])
def test_jacobi_svd_vs_lapack(rows, cols):
    rng = np.random.default_rng(rows + cols)
    X = rng.standard_normal((rows, cols)) @ np.diag(np.logspace(0, -6, cols))
    U, s, V = oracle.jacobi_svd(X)
    sl = scipy.linalg.svd(X, compute_uv=False)
    assert np.max(np.abs(s - sl) / sl) < 1e-12
    assert np.linalg.norm(U.T @ U - np.eye(cols)) < 1e-12 * cols
    assert np.linalg.norm(X @ V - U * s[None, :]) <= 1e-13 * np.linalg.norm(X)
    assert np.all(np.diff(s) <= 0)


def test_jacobi_eig_vs_closed_form_and_lapack():
    ev, V = oracle.jacobi_eig(np.array([[2.0, 1.0], [1.0, 2.0]]))
    assert np.allclose(ev, [3.0, 1.0], rtol=1e-15)
    rng = np.random.default_rng(8)
    B = rng.standard_normal((40, 40))
    G = B.T @ B
    ev, V = oracle.jacobi_eig(G)
    el = scipy.linalg.eigh(G, eigvals_only=True)[::-1]
    assert np.max(np.abs(ev - el)) <= 1e-12 * el[0]
    assert np.linalg.norm(G @ V - V * ev[None, :]) <= 1e-12 * el[0]


# ----------------------------------------------------------------- principal angles

@pytest.mark.parametrize("theta", [1e-12, 1e-10, 1e-8, 1e-5, 1e-2, 1.0])
def test_subspace_sines_closed_form(theta):
    m, k = 40, 4
    Ua = np.zeros((m, k))
    Ub = np.zeros((m, k))
    th = theta * np.array([1.0, 0.5, 0.25, 0.0])
    for i in range(k):
        Ua[i, i] = 1.0
        Ub[i, i] = math.cos(th[i])
        Ub[k + i, i] = math.sin(th[i])
    # random rotation of the ambient space and of the bases: angles are invariant
    rng = np.random.default_rng(5)
    Qm, _ = np.linalg.qr(rng.standard_normal((m, m)))
    Qa, _ = np.linalg.qr(rng.standard_normal((k, k)))
    s = oracle.subspace_sines(Qm @ Ua @ Qa, Qm @ Ub)
    want = np.sort(np.sin(th))[::-1]
    assert np.all(np.abs(s - want) <= 1e-6 * want + 2e-15)     # arccos would lose everything below ~1e-8


# ----------------------------------------------------------------- BLOCK MERGE (Alg. 2)

def test_merge_all_columns_is_thin_svd():
    rng = np.random.default_rng(21)
    X = rng.standard_normal((300, 12)) @ np.diag(np.logspace(0, -3, 12))
    U, s = oracle.merge(None, None, X, 12)
    Ul, sl, _ = np.linalg.svd(X, full_matrices=False)
    assert np.max(np.abs(s - sl) / sl) < 1e-13
    assert oracle.subspace_sines(Ul[:, :6], U[:, :6]).max() < 1e-12


def test_merge_of_exact_svds_is_exact_when_rank_fits():
    """[X Y] ~ [U1 U_o] E blkdiag(V1^T, V2^T) is exact when rank <= r."""
    sm = snapgen.spectrum_matrix(200, 40, np.array([5.0, 3.0, 2.0, 1.0, 0.5]), 0.0, 4, centre=False)
    X, Y = sm.A[:, :25], sm.A[:, 25:]
    Ux, sx, _ = np.linalg.svd(X, full_matrices=False)
    Uy, sy, _ = np.linalg.svd(Y, full_matrices=False)
    r = 6
    U, s = oracle.merge(Ux[:, :r], sx[:r], Uy[:, :r] * sy[None, :r], r)
    assert U.shape[1] == 5                        # rank guard drops the exactly-zero direction
    assert np.max(np.abs(s - sm.s) / sm.s) < 1e-13
    assert oracle.subspace_sines(sm.U, U).max() < 1e-12


def test_merge_weighting_by_sigma_matters():
    """Merging U1 without its singular values would not give the SVD of
    [X Y]: this pins the U1 S1 block of E."""
    rng = np.random.default_rng(2)
    X = rng.standard_normal((100, 8)) @ np.diag([10, 9, 1, 0.5, 0.1, 0.1, 0.1, 0.1])
    Y = rng.standard_normal((100, 5))
    Ux, sx, _ = np.linalg.svd(X, full_matrices=False)
    U, s = oracle.merge(Ux, sx, Y, 13)
    sl = np.linalg.svd(np.hstack([X, Y]), compute_uv=False)
    assert np.max(np.abs(s - sl) / sl) < 1e-12


@pytest.mark.parametrize("r,r_update", [(4, 0), (4, 4), (8, 8)])
def test_series_of_merges_error_bound(r, r_update):
    """|X - P_U X|_2 <= |X - Z_r|_2 <= (2^(P+1) - 3) sigma_{r+1}(X) for the
    sampled columns X in draw order after P merges (error analysis of a
    series of MAT operations)."""
    sm = snapgen.spectrum_matrix(400, 120, np.exp(-np.arange(60) / 4.0), 1e-6, 31, centre=True)
    prm = IsmaParams(k=min(4, r), c=30, r=r, seed=77, r_update=r_update, theta_tol=0.0, max_iter=4)
    res = isma(sm.A, prm, final_step=False)
    P = len(res.log)
    cols = np.concatenate([lg.cols for lg in res.log])
    X = sm.A[:, cols]
    U = res.U_merge
    err = np.linalg.norm(X - U @ (U.T @ X), 2)
    sig = np.linalg.svd(X, compute_uv=False)
    assert err <= (2 ** (P + 1) - 3) * sig[r] * (1 + 1e-10)
    assert err >= sig[r] * (1 - 1e-10)            # Eckart-Young: no rank-r basis does better


# ----------------------------------------------------------------- final step (RR)

def test_project_recovers_exact_spectrum_and_right_vectors():
    sm = snapgen.spectrum_matrix(300, 80, np.array([4.0, 2.0, 1.0, 0.3]), 0.0, 9, centre=False)
    Q, _ = np.linalg.qr(sm.U @ np.random.default_rng(1).standard_normal((4, 4)))  # rotated exact basis
    U, s, V = oracle.project(sm.A, Q)
    assert np.max(np.abs(s - sm.s) / sm.s) < 1e-13
    S = sm.A.T @ U - V * s[None, :]                  # the Wedin S residual vanishes after RR
    assert np.linalg.norm(S) < 1e-12 * s[0]
    assert oracle.subspace_sines(sm.V, V).max() < 1e-12


# ----------------------------------------------------------------- ISMA (Alg. 1)

@pytest.mark.parametrize("w,col_strategy", [(0, "l2n"), (0, "unf"), (30, "l2n")])
def test_isma_exact_on_low_rank(w, col_strategy):
    s = np.array([3.0, 2.0, 1.5, 1.0, 0.7, 0.4])
    sm = snapgen.spectrum_matrix(500, 90, s, 0.0, 13, centre=True)
    prm = IsmaParams(k=6, c=12, w=w, r=6, seed=5, col_strategy=col_strategy, theta_tol=1e-13)
    res = isma(sm.A, prm)
    assert np.max(np.abs(res.sigma - s) / s) < 1e-12
    assert oracle.subspace_sines(sm.U, res.U).max() < 1e-11


def test_isma_stops_when_S_is_empty_and_samples_each_column_once():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((80, 37))
    res = isma(A, IsmaParams(k=3, c=8, seed=1, theta_tol=0.0))
    cols = np.concatenate([lg.cols for lg in res.log])
    assert res.exhausted and not res.converged
    assert np.array_equal(np.sort(cols), np.arange(37))
    for lg in res.log:
        assert np.all(np.diff(lg.cols) > 0)


def test_isma_first_merge_is_svd_of_sampled_columns():
    rng = np.random.default_rng(6)
    A = rng.standard_normal((120, 40))
    res = isma(A, IsmaParams(k=5, c=10, seed=3), n_iter=1, final_step=False)
    D = A[:, res.log[0].cols]
    sl = np.linalg.svd(D, compute_uv=False)
    assert np.max(np.abs(res.s_merge - sl[:5]) / sl[:5]) < 1e-13


def test_isma_all_columns_in_one_draw_gives_truncated_svd():
    """c large enough to draw every column at once: the first merge is the
    truncated SVD of A itself (the SVD-A^T A truth of the evaluation)."""
    sm = snapgen.spectrum_matrix(200, 12, np.logspace(0, -2, 11), 1e-6, 2, centre=True)
    res = isma(sm.A, IsmaParams(k=4, c=2000, seed=8), final_step=True)
    assert len(res.log[0].cols) == 12
    Ul, sl, _ = np.linalg.svd(sm.A, full_matrices=False)
    assert np.max(np.abs(res.sigma - sl[:4]) / sl[:4]) < 1e-12
    assert oracle.subspace_sines(Ul[:, :4], res.U).max() < 1e-11


def test_isma_converges_on_tolerance():
    sm = snapgen.spectrum_matrix(300, 400, np.array([5.0, 4.0, 3.0]), 0.0, 17, centre=True)
    res = isma(sm.A, IsmaParams(k=3, c=10, seed=2, theta_tol=1e-8))
    assert res.converged and len(res.log) == 2      # second merge already reproduces the subspace
    assert res.log[-1].sin_theta < math.sin(1e-8)


def test_incremental_exact_on_low_rank():
    s = np.array([2.0, 1.0, 0.5, 0.25])
    sm = snapgen.spectrum_matrix(300, 200, s, 0.0, 23, centre=True)
    blocks = block_bounds(200, t=4)
    assert blocks == [(0, 50), (50, 100), (100, 150), (150, 200)]
    Uk, sk, _, _ = incremental(sm.A, IsmaParams(k=4, c=10, r=4, seed=3, theta_tol=1e-12), blocks)
    assert np.max(np.abs(sk - s) / s) < 1e-12
    assert oracle.subspace_sines(sm.U, Uk).max() < 1e-11
    assert block_bounds(1100, width=512) == [(0, 512), (512, 1024), (1024, 1100)]


# ---------------------------------------------------------------- quality measure (Eq. ang_meas)
def _orth(X):
    Q, _ = np.linalg.qr(X)
    return Q


def test_wedin_zero_for_exact_triplets():
    """The exact top-k singular triplets leave R = S = 0 (rounding only)."""
    from oracle.wedin import wedin_measure
    rng = np.random.default_rng(11)
    A = rng.standard_normal((300, 80)) @ np.diag(0.9 ** np.arange(80)) @ _orth(rng.standard_normal((80, 80)))
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    k = 6
    rn, sn, om, b = wedin_measure(A, U[:, :k], s[:k], Vt[:k].T, s[k])
    assert rn < 1e-12 * s[0] and sn < 1e-12 * s[0]
    assert om == pytest.approx(min(s[k - 1] - s[k], s[k - 1]), rel=1e-15)
    assert b < 1e-10


def test_wedin_closed_form_rotation():
    """A = diag(d); the k-th left vector turned by theta towards e_{k+1}, the
    rest exact: ||R|| = d_k 2 sin(theta/2), ||S||^2 = d_k^2 (1 - cos theta)^2
    + d_{k+1}^2 sin^2 theta."""
    from oracle.wedin import wedin_measure
    m, n, k, th = 40, 30, 4, 0.03
    d = np.array([10.0, 7.0, 5.0, 3.0, 2.0] + [1.0 / (i + 2) for i in range(n - 5)])
    A = np.zeros((m, n))
    A[np.arange(n), np.arange(n)] = d
    U = np.eye(m)[:, :k].copy()
    U[:, k - 1] = math.cos(th) * np.eye(m)[:, k - 1] + math.sin(th) * np.eye(m)[:, k]
    V = np.eye(n)[:, :k]
    rn, sn, om, b = wedin_measure(A, U, d[:k], V, d[k])
    assert rn == pytest.approx(d[k - 1] * 2 * math.sin(th / 2), rel=1e-13)
    assert sn == pytest.approx(math.sqrt(d[k - 1] ** 2 * (1 - math.cos(th)) ** 2 + d[k] ** 2 * math.sin(th) ** 2),
                               rel=1e-13)
    assert om == pytest.approx(min(d[k - 1] - d[k], d[k - 1]))
    assert b == pytest.approx(math.sqrt(rn * rn + sn * sn) / om, rel=1e-15)


@pytest.mark.parametrize("eps", [1e-6, 1e-4, 1e-2])
def test_wedin_theorem_holds(eps):
    """Wedin's theorem: with omega from the exact singular values, the
    measure bounds the Frobenius norm of the sines of the principal angles
    between exact and perturbed subspaces (left and right)."""
    from oracle.wedin import wedin_measure
    rng = np.random.default_rng(int(-math.log10(eps)))
    m, n, k = 200, 60, 5
    s_true = np.concatenate([[20.0, 15.0, 11.0, 8.0, 6.0], 3.0 * 0.8 ** np.arange(n - 5)])
    Ux = _orth(rng.standard_normal((m, n)))
    Vx = _orth(rng.standard_normal((n, n)))
    A = (Ux * s_true) @ Vx.T
    Ut = _orth(Ux[:, :k] + eps * rng.standard_normal((m, k)))
    Vt = _orth(Vx[:, :k] + eps * rng.standard_normal((n, k)))
    st = s_true[:k] * (1 + eps * rng.standard_normal(k))
    rn, sn, _, _ = wedin_measure(A, Ut, st, Vt, s_true[k])
    omega = min(np.min(np.abs(st[-1] - s_true[k:])), st[-1])
    sin_t = scipy.linalg.subspace_angles(Ux[:, :k], Ut)
    sin_p = scipy.linalg.subspace_angles(Vx[:, :k], Vt)
    lhs = math.sqrt(np.sum(np.sin(sin_t) ** 2) + np.sum(np.sin(sin_p) ** 2))
    assert lhs <= math.sqrt(rn * rn + sn * sn) / omega * (1 + 1e-9)
    assert lhs > 0.0


def test_oracle_bits_do_not_depend_on_threads():
    """The C oracle splits only loops over independent columns between
    threads: merges, projections and norms are bitwise the same at 1 and 4
    threads."""
    rng = np.random.default_rng(17)
    A = rng.standard_normal((3000, 90))
    U0, _ = np.linalg.qr(rng.standard_normal((3000, 12)))
    outs = []
    for th in (1, 4):
        oracle.set_threads(th)
        Um, sm = oracle.merge(U0, np.linspace(3, 1, 12), A[:, :40], 12)
        Up, sp, Vp = oracle.project(A, Um)
        outs.append((Um, sm, Up, sp, Vp, oracle.col_sqnorms(A)))
    oracle.set_threads(os.cpu_count() or 1)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)

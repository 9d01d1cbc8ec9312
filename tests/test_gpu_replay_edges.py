"""GPU checks through the C ABI: replayed draws (pod_set_indices), the stop
reason, row centring, failure statuses, steep spectra and the rank guard.

Replay reading: the leverage-score (LS) row weights depend on the computed
modes, so the FP32 path cannot draw the oracle's rows bit for bit; parity for
LS is checked by replaying one side's draws on the other.  The same replay
freezes the indices for finite differences of the GPU path itself.
"""
import numpy as np
import pytest

import oracle
import snapgen
from oracle.isma import IsmaParams, IterLog, center_rows, isma as oracle_isma

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1905_05107_amd as pod  # noqa: E402

U64 = 2.0 ** -53


def _dev(A_np):
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(A_np).T)).cuda()
    return t.T


def _angles(Ua, Ub):
    return float(np.max(oracle.subspace_sines(np.asarray(Ua, np.float64), np.asarray(Ub, np.float64))))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pod.lib()


@pytest.fixture(scope="module")
def c1():
    return snapgen.config_small_fp64()


def _c1(**kw):
    d = dict(k=10, c=20, seed=2001, theta_tol=1e-10)
    d.update(kw)
    return d


# ------------------------------------------------------------------ replay

@pytest.mark.parametrize("w", [0, 20])
def test_replay_of_own_draws_is_bit_identical(c1, w):
    """A second context with another seed, fed the first run's draws through
    pod_set_indices, merges bit for bit the same states."""
    print(f"replay own draws w={w}", flush=True)
    with pod.PodContext(_dev(c1.A), **_c1(w=w)) as ctx:
        sines = ctx.run(stepwise=True)
        T = ctx.info().iter
        draws = [ctx.indices(t, rows=True) if w else ctx.indices(t) for t in range(T)]
        U0, s0 = ctx.basis()
    with pod.PodContext(_dev(c1.A), **_c1(w=w, seed=99)) as ctx:
        sines2 = ctx.replay(draws)
        assert ctx.info().iter == T
        for t in range(T):
            got = ctx.indices(t, rows=True) if w else ctx.indices(t)
            for a, b in zip(got, draws[t]):
                assert np.array_equal(a, b), t
        U1, s1 = ctx.basis()
    assert np.array_equal(np.array(sines), np.array(sines2), equal_nan=True)
    assert torch.equal(U0, U1) and torch.equal(s0, s1)


def test_set_indices_rejects_bad_input(c1):
    A = _dev(c1.A)
    n, m = c1.A.shape[1], c1.A.shape[0]
    print("set_indices errors", flush=True)
    with pod.PodContext(A, k=3, c=5, seed=1) as ctx:
        for cols, cnt in [([5, 3], None), ([3, 3], None), ([n], None), ([-1], None), (list(range(6)), None),
                          ([2, 4], [1, 0])]:
            with pytest.raises(pod.PodError) as e:
                ctx.set_indices(0, cols, cnt)
            assert e.value.status == pod.POD_EINVAL, cols
        with pytest.raises(pod.PodError) as e:
            ctx.set_indices(1, [0])                  # not the next merge
        assert e.value.status == pod.POD_ESTATE
        ctx.set_indices(0, [3, 7], [2, 1])
        assert ctx.sample() is True
        with pytest.raises(pod.PodError) as e:       # a draw is pending
            ctx.set_indices(1, [4])
        assert e.value.status == pod.POD_ESTATE
        ctx.merge()
        assert np.array_equal(ctx.indices(0)[0], [3, 7]) and np.array_equal(ctx.indices(0)[1], [2, 1])
        with pytest.raises(pod.PodError) as e:       # column 7 left S
            ctx.set_indices(1, [7])
        assert e.value.status == pod.POD_EINVAL
        ctx.set_indices(1, [0, n - 1])
        ctx.sample()
        ctx.merge()
        assert ctx.info().rank == 3
    with pod.PodContext(A, k=3, c=5, w=6, seed=1) as ctx:
        for rows, rcnt in [(None, None), ([4, 2], [3, 3]), ([2, 2], [3, 3]), ([1, 2], [3, 2]), ([m], [6]),
                           (list(range(7)), [1] * 7)]:
            with pytest.raises((pod.PodError, ValueError)):
                ctx.set_indices(0, [1, 2], None, rows, rcnt)
        ctx.set_indices(0, [1, 2], None, [10, 20], [4, 2])
        ctx.sample()
        ctx.merge()
        got = ctx.indices(0, rows=True)
        assert np.array_equal(got[2], [10, 20]) and np.array_equal(got[3], [4, 2])


def _oracle_logs(draws):
    return [IterLog(cols=np.asarray(d[0], np.int64), col_counts=np.asarray(d[1], np.int32),
                    rows=np.asarray(d[2], np.int64), row_counts=np.asarray(d[3], np.int32)) for d in draws]


def test_ls_rows_fp32_parity_by_replay(c1):
    """Leverage-score rows on the FP32 path: the oracle replays the GPU's draws,
    and the GPU replays the oracle's; both against the FP32 bars (sigma 1e-5
    relative, largest principal angle 1e-5)."""
    A = c1.A.astype(np.float32)
    kw = _c1(w=20, theta_tol=1e-6)
    print("ls rows fp32 replay", flush=True)
    # oracle <- GPU
    with pod.PodContext(_dev(A), precision=pod.POD_F32, row_strategy=pod.POD_ROW_LS, **kw) as ctx:
        ctx.run()
        T = ctx.info().iter
        draws = [ctx.indices(t, rows=True) for t in range(T)]
        U, s, _ = ctx.project(want_v=False)
    ref = oracle_isma(A, IsmaParams(row_strategy="ls", **kw), n_iter=T, replay=_oracle_logs(draws), elem_bytes=4)
    rel = np.max(np.abs(s.cpu().numpy() - ref.sigma) / ref.sigma)
    ang = _angles(ref.U, U.cpu().numpy())
    print(f"  oracle replays GPU: iters={T} sigma_rel={rel:.2e} angle={ang:.2e}", flush=True)
    assert rel <= 1e-5 and ang <= 1e-5
    # GPU <- oracle
    ref2 = oracle_isma(A, IsmaParams(row_strategy="ls", **kw), elem_bytes=4)
    odraws = [(lg.cols, lg.col_counts, lg.rows, lg.row_counts) for lg in ref2.log]
    with pod.PodContext(_dev(A), precision=pod.POD_F32, row_strategy=pod.POD_ROW_LS, **kw) as ctx:
        ctx.replay(odraws)
        assert ctx.info().iter == len(odraws)
        U2, s2, _ = ctx.project(want_v=False)
    rel2 = np.max(np.abs(s2.cpu().numpy() - ref2.sigma) / ref2.sigma)
    ang2 = _angles(ref2.U, U2.cpu().numpy())
    print(f"  GPU replays oracle: iters={len(odraws)} sigma_rel={rel2:.2e} angle={ang2:.2e}", flush=True)
    assert rel2 <= 1e-5 and ang2 <= 1e-5


def test_loss_gradient_fd_of_the_gpu_path_with_frozen_indices():
    """Central differences (h = 1e-6) of the GPU path's own loss
    |A - U_k U_k^T A|_F^2, with the draws of the base run replayed at A +- hE,
    against the GPU gradient along 8 random unit directions (FP64, 500 x 100,
    s_i = e^(-i/6), k = 4, c = 8): relative error <= 1e-6."""
    sm = snapgen.spectrum_matrix(500, 100, np.exp(-np.arange(100) / 6.0), 1e-8, seed=1005, centre=False,
                                 v_orthogonal_to_ones=False)
    A = sm.A
    kw = dict(k=4, c=8, seed=2005, theta_tol=1e-8, precision=pod.POD_F64)
    print("fd of the gpu path", flush=True)
    with pod.PodContext(_dev(A), **kw) as ctx:
        ctx.enable_adjoint()
        ctx.run()
        T = ctx.info().iter
        draws = [ctx.indices(t) for t in range(T)]
        L0, G = ctx.loss_grad()
        G = G.cpu().numpy()

    def loss(X):
        with pod.PodContext(_dev(X), **dict(kw, seed=77)) as c2:
            c2.enable_adjoint()
            c2.replay(draws)
            assert c2.info().iter == T
            return c2.loss_grad()[0]

    rng = np.random.default_rng(6)
    h = 1e-6
    worst = 0.0
    for _ in range(8):
        E = rng.standard_normal(A.shape)
        E /= np.linalg.norm(E)
        fd = (loss(A + h * E) - loss(A - h * E)) / (2 * h)
        an = float(np.sum(G * E))
        err = abs(fd - an) / max(abs(an), 1e-2 * np.linalg.norm(G))
        worst = max(worst, err)
    print(f"  merges={T} L={L0:.6e} worst rel={worst:.2e}", flush=True)
    assert worst <= 1e-6


# ------------------------------------------------------------------ stop reason and failures

def test_stop_reason_exhausted_converged_max_iter(c1):
    """Exactly rank-6 data with r = k = 6 converges at the second merge (sine
    ~1e-15); the small FP64 workload runs until S is exhausted (28 merges);
    max_iter cuts a run short; a fixed number of merges leaves no rule met."""
    print("stop reasons", flush=True)
    sm = snapgen.spectrum_matrix(500, 90, np.array([3.0, 2.0, 1.5, 1.0, 0.7, 0.4]), 0.0, 13, centre=True)
    res = pod.isma(_dev(sm.A), k=6, r=6, c=12, seed=5, theta_tol=1e-10)
    assert res.stopped_by == "converged" and res.converged and res.iters == 2
    res = pod.isma(_dev(c1.A), **_c1())
    assert res.stopped_by == "exhausted" and not res.converged and res.iters == 28
    res = pod.isma(_dev(c1.A), max_iter=3, **_c1())
    assert res.stopped_by == "max_iter" and res.iters == 3
    with pod.PodContext(_dev(c1.A), **_c1()) as ctx:
        ctx.run(n_iter=2)
        assert ctx.info().stop_reason == pod.POD_STOP_NONE


@pytest.mark.parametrize("dtype,bad", [(np.float64, np.nan), (np.float32, np.inf)])
def test_nonfinite_column_reports_enonfinite(c1, dtype, bad):
    """A NaN or Inf in A: the norm pass flags it, the run stops with
    POD_ENONFINITE, and the stop reason says so."""
    A = c1.A.astype(dtype).copy(order="F")
    A[17, 123] = bad
    prec = pod.POD_F64 if dtype == np.float64 else pod.POD_F32
    print(f"nonfinite {dtype.__name__}", flush=True)
    with pytest.raises(pod.PodError) as e:
        pod.isma(_dev(A), precision=prec, **_c1())
    assert e.value.status == pod.POD_ENONFINITE
    with pod.PodContext(_dev(A), precision=prec, **_c1()) as ctx:
        with pytest.raises(pod.PodError) as e:
            ctx.run()
        assert e.value.status == pod.POD_ENONFINITE
        assert ctx.info().stop_reason == pod.POD_STOP_NONFINITE


def test_zero_block_reports_enotpd():
    """A merge block whose Gram is zero (a replayed zero column on an empty
    state): the Cholesky fails, and so does the shifted retry (the shift
    scales with the trace); POD_ENOTPD, stop reason "breakdown"."""
    rng = np.random.default_rng(2)
    A = rng.standard_normal((300, 12))
    A[:, 0] = 0.0
    print("zero block", flush=True)
    with pod.PodContext(_dev(A), k=2, c=4, seed=3) as ctx:
        ctx.set_indices(0, [0])
        ctx.sample()
        ctx.merge()
        with pytest.raises(pod.PodError) as e:
            ctx.converged()
        assert e.value.status == pod.POD_ENOTPD
        inf = ctx.info()
        assert inf.stop_reason == pod.POD_STOP_BREAKDOWN and (inf.flags & 16)


# ------------------------------------------------------------------ row centring (A0)

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_center_rows_parity(dtype):
    """center_rows = 1 subtracts the FP64 row means from A in place: against
    the oracle's centring within the rounding of the two summation orders,
    then the run on the centred matrix against the oracle (indices bit-exact
    on the same bytes; the FP64 / FP32 bars against the oracle's own centred
    matrix)."""
    sm = snapgen.spectrum_matrix(1500, 300, np.exp(-np.arange(60) / 6.0), 1e-8, seed=31, centre=False,
                                 v_orthogonal_to_ones=False)
    rng = np.random.default_rng(32)
    raw = np.asfortranarray((sm.A + 3.0 * rng.standard_normal((1500, 1))).astype(dtype))
    prec = pod.POD_F64 if dtype == np.float64 else pod.POD_F32
    kw = dict(k=8, c=16, seed=33, theta_tol=1e-9 if dtype == np.float64 else 1e-5)
    print(f"center rows {dtype.__name__}", flush=True)
    want, mean = center_rows(raw)
    Ad = _dev(raw)
    Bd = pod.center_rows(_dev(raw))                  # the stand-alone entry point, same kernels
    with pod.PodContext(Ad, precision=prec, center_rows=True, **kw) as ctx:
        got = Ad.cpu().numpy()
        assert torch.equal(Ad, Bd)
        ctx.run()
        T = ctx.info().iter
        cols = [ctx.indices(t)[0] for t in range(T)]
        U, s, _ = ctx.project(want_v=False)
    if dtype == np.float64:
        assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(raw))
    else:
        ulp = np.spacing(np.abs(want).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(got.astype(np.float64) - want.astype(np.float64)) <= ulp + 1e-7 * np.abs(mean)[:, None])
    assert np.max(np.abs(got.astype(np.float64).mean(axis=1))) <= 1e-6 * np.max(np.abs(raw))
    ref_same = oracle_isma(got, IsmaParams(**kw), n_iter=T, final_step=False)
    for t in range(T):
        assert np.array_equal(cols[t], ref_same.log[t].cols), t
    ref = oracle_isma(want, IsmaParams(**kw), n_iter=T)
    tol_s, tol_a = (1e-10, 1e-8) if dtype == np.float64 else (1e-5, 1e-5)
    rel = np.max(np.abs(s.cpu().numpy() - ref.sigma) / ref.sigma)
    ang = _angles(ref.U, U.cpu().numpy())
    print(f"  iters={T} sigma_rel={rel:.2e} angle={ang:.2e}", flush=True)
    assert rel <= tol_s and ang <= tol_a


# ------------------------------------------------------------------ steep spectra and the rank guard

def test_steep_spectrum_fp64():
    """s_i = 10^(-6 i / 9) for i < 10 (sigma_10 / sigma_1 = 1e-6) over a noise
    floor of standard deviation 1e-9, k = 10: singular values within 1e-10
    relative of the oracle and largest principal angle <= 1e-8.  The merge and
    Rayleigh-Ritz singular values are row norms of U_R^T R and B^T U_B, whose
    error is about p u sigma_1 absolute (the backward-error floor of any FP64
    method: 3e-7 of sigma_10 here, the bound checked first); the square roots
    of the eigenvalues of R R^T would lose p u sigma_1^2 / sigma_i, 3e-3 of
    sigma_10."""
    s = 10.0 ** (-6.0 * np.arange(10) / 9.0)
    sm = snapgen.spectrum_matrix(3000, 400, s, 1e-18, seed=41, centre=False, v_orthogonal_to_ones=False)
    kw = dict(k=10, c=20, seed=42, theta_tol=1e-12)
    print("steep spectrum", flush=True)
    res = pod.isma(_dev(sm.A), want_v=False, **kw)
    ref = oracle_isma(sm.A, IsmaParams(**kw), n_iter=res.iters, want_v=False)
    g = res.sigma.cpu().numpy()
    p = 10 + 20
    err = np.abs(g - ref.sigma)
    bound = 1e-10 * ref.sigma + 100 * p * U64 * ref.sigma[0]
    ang = _angles(ref.U, res.U.cpu().numpy())
    print(f"  iters={res.iters} flags={res.flags} max err/bound={np.max(err / bound):.2e} "
          f"rel(sigma_10)={err[-1] / ref.sigma[-1]:.2e} angle={ang:.2e}", flush=True)
    assert res.iters == len(ref.log) or res.stopped_by == "exhausted"
    assert np.all(err <= bound)
    assert np.max(err / ref.sigma) <= 1e-10
    assert ang <= 1e-8


def test_rank_guard_below_the_fp64_eigenvalue_resolution():
    """An exactly rank-6 matrix whose sixth singular value is 1e-9 sigma_1,
    r = k = 6.  The oracle (Householder QR, one-sided Jacobi on R) keeps all
    six directions (sigma_6 > p u sigma_1).  The GPU merge reads the
    eigenvalues of R R^T, which resolve a direction only down to about
    sqrt(p u_64) sigma_1 (~1e-7): its rank guard drops sigma_6 (the reading of
    the guard for the eigenvalue route).  The five leading modes and values
    agree with the oracle's to the FP64 bars."""
    s = np.array([1.0, 0.5, 0.2, 0.1, 0.05, 1e-9])
    sm = snapgen.spectrum_matrix(2000, 200, s, 0.0, seed=43, centre=False, v_orthogonal_to_ones=False)
    kw = dict(k=6, c=12, seed=44, theta_tol=1e-12)
    print("rank guard", flush=True)
    with pod.PodContext(_dev(sm.A), **kw) as ctx:
        ctx.run()
        inf = ctx.info()
        U, sg, _ = ctx.project(want_v=False)
    ref = oracle_isma(sm.A, IsmaParams(**kw), n_iter=inf.iter, want_v=False)
    g = sg.cpu().numpy()
    print(f"  iters={inf.iter} gpu rank={inf.rank} oracle rank={ref.U_merge.shape[1]} gpu sigma={g} "
          f"oracle sigma={ref.sigma}", flush=True)
    assert ref.U_merge.shape[1] == 6
    assert inf.rank == 5 and g.shape[0] == 5
    assert np.max(np.abs(g - ref.sigma[:5]) / ref.sigma[:5]) <= 1e-10
    assert _angles(ref.U[:, :5], U.cpu().numpy()) <= 1e-8

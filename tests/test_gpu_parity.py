"""Parity of the HIP library (called through its C ABI) with the FP64 oracle.

Bars: sampled indices and column norms bit-exact; FP64 path singular values
within 1e-10 relative and largest principal angle <= 1e-8; FP32 path within
1e-5 / 1e-5 rad (angles measured between the GPU's and the oracle's first k
modes after the final Rayleigh-Ritz step, sign-free).
"""
import math

import numpy as np
import pytest

import oracle
import snapgen
from oracle.isma import IsmaParams, isma as oracle_isma

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1905_05107_amd as pod  # noqa: E402


def _dev(A_np):
    """Column-major device copy of an m x n numpy array."""
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(A_np).T)).cuda()
    return t.T


def _angles(Ua, Ub):
    return float(np.max(oracle.subspace_sines(np.asarray(Ua, np.float64), np.asarray(Ub, np.float64))))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pod.lib()


# ------------------------------------------------------------------ column norms

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("m,n", [(1, 3), (5, 2), (1023, 4), (1024, 3), (1025, 5), (4097, 7), (20011, 9),
                                 (262147, 3)])
def test_col_sqnorms_bit_exact(dtype, m, n):
    rng = np.random.default_rng(m + n)
    A = (rng.standard_normal((m, n)) * np.exp(rng.uniform(-3, 3, size=(1, n)))).astype(dtype)
    print(f"col_sqnorms dtype={np.dtype(dtype).name} m={m} n={n}", flush=True)
    nu = pod.col_sqnorms(_dev(A)).cpu().numpy()
    want = oracle.col_sqnorms(A)
    assert np.array_equal(nu, want)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_col_sqnorms_unaligned_leading_dimension(dtype):
    rng = np.random.default_rng(7)
    m, n, lda = 3001, 6, 3003       # lda not a multiple of the vector width
    store = rng.standard_normal((n, lda)).astype(dtype)
    t = torch.from_numpy(store).cuda()
    A_dev = t[:, :m].T
    nu = pod.col_sqnorms(A_dev).cpu().numpy()
    want = oracle.col_sqnorms(store[:, :m].T.copy())
    assert np.array_equal(nu, want)


# ------------------------------------------------------------------ small FP64 workload

def _c1_params(**kw):
    d = dict(k=10, c=20, seed=2001, theta_tol=1e-10)
    d.update(kw)
    return d


@pytest.fixture(scope="module")
def c1():
    return snapgen.config_small_fp64()


def test_c1_indices_and_norms_bit_exact(c1):
    A = c1.A
    print("c1 indices", flush=True)
    ref = oracle_isma(A, IsmaParams(**_c1_params()), final_step=False)
    with pod.PodContext(_dev(A), **_c1_params()) as ctx:
        nu = ctx.col_sqnorms()
        assert np.array_equal(nu, oracle.col_sqnorms(A))
        sines = ctx.run()
        assert len(sines) == len(ref.log)
        for it, lg in enumerate(ref.log):
            cols, cnt = ctx.indices(it)
            assert np.array_equal(cols, lg.cols), it
            assert np.array_equal(cnt, lg.col_counts), it


@pytest.mark.parametrize("criterion", [pod.POD_CRIT_SUBSPACE, pod.POD_CRIT_MODE])
def test_c1_fp64_parity(c1, criterion):
    A = c1.A
    crit = "subspace" if criterion == pod.POD_CRIT_SUBSPACE else "mode"
    print(f"c1 fp64 parity {crit}", flush=True)
    ref = oracle_isma(A, IsmaParams(**_c1_params(criterion=crit)))
    res = pod.isma(_dev(A), criterion=criterion, **_c1_params())
    assert res.iters == len(ref.log)
    U = res.U.cpu().numpy()
    s = res.sigma.cpu().numpy()
    assert np.max(np.abs(s - ref.sigma) / ref.sigma) <= 1e-10
    assert _angles(ref.U, U) <= 1e-8
    # per-iteration convergence sines agree (explicit residual vs. small-SVD shortcut)
    for g_s, lg in zip(res.sin_theta[1:], ref.log[1:]):
        assert abs(g_s - lg.sin_theta) <= 1e-9 * max(1.0, lg.sin_theta) + 1e-12
    # sign convention: largest-magnitude entry positive
    for i in range(U.shape[1]):
        j = int(np.argmax(np.abs(U[:, i])))
        assert U[j, i] > 0
    V = res.V.cpu().numpy()
    assert _angles(ref.V, V) <= 1e-8


def test_c1_merge_state_each_iteration(c1):
    A = c1.A
    print("c1 merge state", flush=True)
    for t in (1, 2, 5):
        ref = oracle_isma(A, IsmaParams(**_c1_params()), n_iter=t, final_step=False)
        with pod.PodContext(_dev(A), **_c1_params()) as ctx:
            ctx.run(n_iter=t)
            U, s = ctx.basis()
            U, s = U.cpu().numpy(), s.cpu().numpy()
        assert U.shape[1] == ref.U_merge.shape[1]
        assert np.max(np.abs(s - ref.s_merge) / ref.s_merge) <= 1e-10, t
        assert _angles(ref.U_merge[:, :10], U[:, :10]) <= 1e-8, t
        assert np.linalg.norm(U.T @ U - np.eye(U.shape[1])) <= 1e-12


@pytest.mark.parametrize("kw", [dict(), dict(precision=pod.POD_F32), dict(precision=pod.POD_BF16_REFINE), dict(w=60),
                                dict(r_update=8), dict(n_iter=5)])
def test_device_loop_equals_stepwise_loop(c1, kw):
    """pod_run (the loop of Alg. 1 with a device-side stop test and chunked
    launches) gives the host loop's merges bit for bit: same sines, same basis."""
    kw = dict(kw)
    n_iter = kw.pop("n_iter", None)
    print(f"device loop vs stepwise {kw} n_iter={n_iter}", flush=True)
    A = c1.A.astype(np.float32) if kw.get("precision") in (pod.POD_F32, pod.POD_BF16_REFINE) else c1.A
    outs = []
    for stepwise, chunk in [(True, 8), (False, 3), (False, 64)]:
        with pod.PodContext(_dev(A), **_c1_params(**kw)) as ctx:
            sines = ctx.run(n_iter=n_iter, chunk=chunk, stepwise=stepwise)
            inf = ctx.info()
            U, sig, _ = ctx.project(want_v=False)
            outs.append((sines, inf.iter, U.cpu().numpy(), sig.cpu().numpy()))
    ref = outs[0]
    assert len(ref[0]) >= 2
    for o in outs[1:]:
        assert o[1] == ref[1] and len(o[0]) == len(ref[0])
        assert np.array_equal(np.array(o[0]), np.array(ref[0]), equal_nan=True)
        assert np.array_equal(o[2], ref[2]) and np.array_equal(o[3], ref[3])


def test_unf_strategy_and_r_larger_than_k(c1):
    A = c1.A
    kw = _c1_params(col_strategy="unf", r=30)
    ref = oracle_isma(A, IsmaParams(**kw))
    kw_gpu = dict(kw)
    kw_gpu["col_strategy"] = pod.POD_COL_UNF
    print("c1 unf r=30", flush=True)
    res = pod.isma(_dev(A), **kw_gpu)
    assert res.iters == len(ref.log)
    s = res.sigma.cpu().numpy()
    assert np.max(np.abs(s - ref.sigma) / ref.sigma) <= 1e-10
    assert _angles(ref.U, res.U.cpu().numpy()) <= 1e-8


# ------------------------------------------------------------------ edge cases

def test_exact_low_rank_recovers_spectrum():
    s = np.array([3.0, 2.0, 1.5, 1.0, 0.7, 0.4])
    sm = snapgen.spectrum_matrix(500, 90, s, 0.0, 13, centre=True)
    print("low rank", flush=True)
    res = pod.isma(_dev(sm.A), k=6, r=6, c=12, seed=5, theta_tol=1e-13)
    assert np.max(np.abs(res.sigma.cpu().numpy() - s) / s) < 1e-11
    assert _angles(sm.U, res.U.cpu().numpy()) < 1e-10


def test_exhaustion_samples_each_column_once():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((80, 37))
    ref = oracle_isma(A, IsmaParams(k=3, c=8, seed=1, theta_tol=0.0))
    print("exhaustion", flush=True)
    with pod.PodContext(_dev(A), k=3, c=8, seed=1, theta_tol=0.0) as ctx:
        ctx.run()
        inf = ctx.info()
        assert inf.exhausted and inf.iter == len(ref.log)
        cols = np.concatenate([ctx.indices(i)[0] for i in range(inf.iter)])
        assert np.array_equal(np.sort(cols), np.arange(37))
        assert ctx.sample() is False
        U, s, V = ctx.project()
    assert np.max(np.abs(s.cpu().numpy() - ref.sigma) / ref.sigma) <= 1e-10


def test_single_column_and_c_above_n():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((300, 12))
    print("c above n", flush=True)
    res = pod.isma(_dev(A), k=4, c=200, seed=8)
    Ul, sl, _ = np.linalg.svd(A, full_matrices=False)
    assert res.iters == 1
    assert np.max(np.abs(res.sigma.cpu().numpy() - sl[:4]) / sl[:4]) < 1e-12
    assert _angles(Ul[:, :4], res.U.cpu().numpy()) < 1e-11
    B = rng.standard_normal((50, 1))
    res1 = pod.isma(_dev(B), k=1, c=3, seed=1)
    assert abs(res1.sigma.cpu().numpy()[0] - np.linalg.norm(B)) <= 1e-13 * np.linalg.norm(B)


def test_invalid_arguments_rejected():
    A = _dev(np.zeros((10, 4)))
    with pytest.raises(pod.PodError) as e:
        pod.PodContext(A, k=5, c=2, r=3)          # r < k
    assert e.value.status == pod.POD_EINVAL
    with pytest.raises(pod.PodError):
        pod.PodContext(A, k=1, c=0)


def test_zero_matrix_is_exhausted_at_once():
    A = _dev(np.zeros((64, 5)))
    with pod.PodContext(A, k=1, c=2) as ctx:
        assert ctx.sample() is True       # no sync: exhaustion is found on the device
        ctx.merge()
        done, _ = ctx.converged()
        assert done and ctx.info().exhausted and ctx.info().iter == 0


# ------------------------------------------------------------------ FP32 path (travelling waves)

@pytest.fixture(scope="module")
def waves_small():
    return snapgen.waves_np(20000, 400, 60, 1.5, 1e-3, seed=1002)


def test_waves_indices_bit_exact_fp32(waves_small):
    A = waves_small
    kw = dict(k=20, c=40, seed=2002, theta_tol=1e-5, max_iter=6)
    ref = oracle_isma(A, IsmaParams(**kw), n_iter=4, final_step=False, elem_bytes=4)
    print("waves fp32 indices", flush=True)
    with pod.PodContext(_dev(A), precision=pod.POD_F32, **kw) as ctx:
        assert np.array_equal(ctx.col_sqnorms(), oracle.col_sqnorms(A))
        ctx.run(n_iter=4)
        for it in range(4):
            assert np.array_equal(ctx.indices(it)[0], ref.log[it].cols)


@pytest.mark.parametrize("precision", [pod.POD_F64, pod.POD_F32, pod.POD_BF16_REFINE])
def test_waves_parity(waves_small, precision):
    A = waves_small
    kw = dict(k=20, c=40, seed=2002, theta_tol=1e-5)
    print(f"waves parity precision={precision}", flush=True)
    res = pod.isma(_dev(A), precision=precision, **kw)
    ref = oracle_isma(A, IsmaParams(**kw), n_iter=res.iters, elem_bytes=4)
    s = res.sigma.cpu().numpy()
    U = res.U.cpu().numpy()
    tol_s, tol_a = (1e-10, 1e-8) if precision == pod.POD_F64 else (1e-5, 1e-5)
    rel = np.max(np.abs(s - ref.sigma) / ref.sigma)
    ang = _angles(ref.U, U)
    print(f"  iters={res.iters} sigma_rel={rel:.3e} angle={ang:.3e} flags={res.flags}", flush=True)
    assert rel <= tol_s
    assert ang <= tol_a


# ------------------------------------------------------------------ rows (ICRS) and truncated blocks

def _check_run_parity(A, kw, gpu_kw, tol_s=1e-10, tol_a=1e-8, rows=True, elem_bytes=None, tol_sin=1e-9):
    ref = oracle_isma(A, IsmaParams(**kw), elem_bytes=elem_bytes)
    res = None
    with pod.PodContext(_dev(A), **gpu_kw) as ctx:
        sines = ctx.run()
        assert len(sines) == len(ref.log)
        for it, lg in enumerate(ref.log):
            got = ctx.indices(it, rows=True)
            assert np.array_equal(got[0], lg.cols), it
            assert np.array_equal(got[1], lg.col_counts), it
            if rows:
                assert np.array_equal(got[2], lg.rows), it
                assert np.array_equal(got[3], lg.row_counts), it
        for g_s, lg in zip(sines[1:], ref.log[1:]):
            assert abs(g_s - lg.sin_theta) <= tol_sin * max(1.0, lg.sin_theta) + 1e-12
        U, s, _ = ctx.project(want_v=False)
        res = (U.cpu().numpy(), s.cpu().numpy())
    U, s = res
    rel = np.max(np.abs(s - ref.sigma) / ref.sigma)
    ang = _angles(ref.U, U)
    print(f"  iters={len(ref.log)} sigma_rel={rel:.3e} angle={ang:.3e}", flush=True)
    assert rel <= tol_s
    assert ang <= tol_a


@pytest.mark.parametrize("strategy", ["l2", "ls"])
def test_c1_rows_parity(c1, strategy):
    """C1 with w = 20 rows per iteration (SAMPLE AND SCALE UNIQUE ROWS):
    columns, rows and multiplicities bit-exact, FP64 bars on the result."""
    kw = _c1_params(w=20, row_strategy=strategy)
    print(f"c1 rows {strategy}", flush=True)
    rs = pod.POD_ROW_L2 if strategy == "l2" else pod.POD_ROW_LS
    _check_run_parity(c1.A, kw, dict(_c1_params(w=20), row_strategy=rs))


def test_rows_fewer_than_rank(c1):
    """h < r: the block keeps at most h directions."""
    kw = _c1_params(w=3, r=12, max_iter=8)
    print("c1 rows w=3", flush=True)
    _check_run_parity(c1.A, kw, dict(kw))


def test_c1_truncated_block_parity(c1):
    """GET UPDATE without rows, each block cut to its top r_update right
    singular directions before the merge."""
    kw = _c1_params(r_update=6)
    print("c1 r_update=6", flush=True)
    _check_run_parity(c1.A, kw, dict(kw), rows=False)


def test_waves_rows_fp32(waves_small):
    """FP32 path with rows: indices bit-exact (row norms of FP32 data are
    exact), result within the FP32 bars."""
    A = waves_small
    kw = dict(k=20, c=40, w=200, seed=2002, theta_tol=1e-5, max_iter=12)
    print("waves rows fp32", flush=True)
    _check_run_parity(A, kw, dict(kw, precision=pod.POD_F32), tol_s=1e-5, tol_a=1e-5, elem_bytes=4, tol_sin=1e-5)


# ------------------------------------------------------------------ wide merges (p > 64: matrices outside LDS)

@pytest.fixture(scope="module")
def wide_fp64():
    s = np.exp(-np.arange(150) / 25.0)
    return snapgen.spectrum_matrix(3000, 700, s, 1e-8, seed=1007).A


@pytest.mark.parametrize("precision", [pod.POD_F64, pod.POD_F32, pod.POD_BF16_REFINE])
def test_wide_merge_parity(wide_fp64, precision):
    """k = 40, c = 100: merge width p = 140 (C3-like), FP64, FP32 and split-BF16 paths."""
    A = wide_fp64 if precision == pod.POD_F64 else wide_fp64.astype(np.float32)
    kw = dict(k=40, c=100, seed=2007, theta_tol=1e-9, max_iter=5)
    print(f"wide merge precision={precision}", flush=True)
    tol = (1e-10, 1e-8, 1e-9) if precision == pod.POD_F64 else (1e-5, 1e-5, 1e-5)
    _check_run_parity(A, kw, dict(kw, precision=precision), tol_s=tol[0], tol_a=tol[1], rows=False,
                      tol_sin=tol[2])


def test_wide_rows_and_rank(wide_fp64):
    """Rows with a wide block (g up to 100 > 64) and r = 2k."""
    kw = dict(k=30, r=60, c=90, w=300, seed=2008, theta_tol=1e-9, max_iter=4)
    print("wide rows", flush=True)
    _check_run_parity(wide_fp64, kw, dict(kw))


# ------------------------------------------------------------------ Alg. 3 (incremental over column blocks)

def _inc_check(A, kw, blocks, gpu_kw, host: bool, tol_s, tol_a):
    from oracle.isma import incremental
    Uk, sk, _, _ = incremental(A, IsmaParams(**kw), blocks, elem_bytes=A.dtype.itemsize)
    width = max(j1 - j0 for j0, j1 in blocks)
    m = A.shape[0]
    with pod.Incremental(m, width, dtype=str(A.dtype), **gpu_kw) as inc:
        if host:
            hb = [torch.from_numpy(np.ascontiguousarray(A[:, j0:j1].T)).pin_memory() for j0, j1 in blocks]
            inc.add_host_blocks(hb)
            info = inc.info()
            assert info.blocks == len(blocks) and info.columns == A.shape[1]
            assert info.host_bytes == A.size * A.dtype.itemsize
        else:
            for j0, j1 in blocks:
                inc.add_block(_dev(A[:, j0:j1]))
        U, s = inc.result()
    U, s = U.cpu().numpy(), s.cpu().numpy()
    rel = np.max(np.abs(s - sk) / sk)
    ang = _angles(Uk, U)
    print(f"  blocks={len(blocks)} sigma_rel={rel:.3e} angle={ang:.3e}", flush=True)
    assert U.shape == Uk.shape
    assert rel <= tol_s
    assert ang <= tol_a
    for i in range(U.shape[1]):       # sign convention
        j = int(np.argmax(np.abs(U[:, i])))
        assert U[j, i] > 0


def test_incremental_device_blocks_fp64(c1):
    from oracle.isma import block_bounds
    kw = _c1_params(theta_tol=1e-9)
    print("incremental fp64 device blocks", flush=True)
    _inc_check(c1.A, kw, block_bounds(c1.A.shape[1], 4), dict(kw, precision=pod.POD_F64), False, 1e-10, 1e-8)


def test_incremental_host_blocks_bf16_split(waves_small):
    """Alg. 3 over pinned host blocks with the merges on split-BF16 matrix cores."""
    from oracle.isma import block_bounds
    A = waves_small
    kw = dict(k=20, c=40, seed=2004, theta_tol=1e-5, max_iter=30)
    print("incremental bf16 host blocks", flush=True)
    _inc_check(A, kw, block_bounds(A.shape[1], width=128), dict(kw, precision=pod.POD_BF16_REFINE), True, 1e-5,
               1e-5)


def test_incremental_host_blocks_ragged_fp32(waves_small):
    """Pinned host blocks of 128 columns and a 16-column tail, FP32 path."""
    from oracle.isma import block_bounds
    A = waves_small
    kw = dict(k=20, c=40, seed=2004, theta_tol=1e-5, max_iter=30)
    print("incremental fp32 host blocks", flush=True)
    _inc_check(A, kw, block_bounds(A.shape[1], width=128), dict(kw, precision=pod.POD_F32), True, 1e-5, 1e-5)


def test_incremental_rows_r_above_k(c1):
    """Blocks sampled with rows, r = 2k."""
    from oracle.isma import block_bounds
    kw = _c1_params(w=20, r=20, theta_tol=1e-9)
    print("incremental rows", flush=True)
    _inc_check(c1.A, kw, block_bounds(c1.A.shape[1], 3), dict(kw, precision=pod.POD_F64), False, 1e-10, 1e-8)


# ------------------------------------------------------------------ batched runs (one launch per kernel for all matrices)

def _batch_mats(count, seed, dtype=np.float32):
    rng = np.random.default_rng(seed)
    mats, kws = [], []
    for i in range(count):
        m = int(rng.integers(3000, 12000))
        n = int(rng.integers(120, 400))
        k = int(rng.integers(4, 17))
        tau = float(rng.uniform(3, 12))
        s = np.exp(-np.arange(min(n, 200)) / tau)
        A = snapgen.spectrum_matrix(m, n, s, 1e-8, seed=seed * 100 + i, centre=False,
                                    v_orthogonal_to_ones=False).A.astype(dtype)
        mats.append(A)
        kws.append(dict(k=k, c=2 * k, seed=5000 + i, theta_tol=1e-6))
    return mats, kws


@pytest.mark.parametrize("precision,use_graph", [(pod.POD_F32, True), (pod.POD_F32, False), (pod.POD_F64, True)])
def test_batch_equals_single_runs(precision, use_graph):
    """Each matrix of a batch gives bit-for-bit the result of its own run."""
    mats, kws = _batch_mats(6, 11, np.float32 if precision == pod.POD_F32 else np.float64)
    print(f"batch precision={precision} graph={use_graph}", flush=True)
    dev = [_dev(A) for A in mats]
    with pod.Batch(dev, [dict(kw, precision=precision) for kw in kws]) as b:
        rounds = b.run(use_graph=use_graph)
        got = [b.project(i) for i in range(len(mats))]
        iters = [b.info(i)[0].iter for i in range(len(mats))]
    assert rounds >= max(iters)
    for i, (A, kw) in enumerate(zip(dev, kws)):
        res = pod.isma(A, precision=precision, want_v=False, **kw)
        assert res.iters == iters[i]
        assert torch.equal(res.U, got[i][0]), i
        assert torch.equal(res.sigma, got[i][1]), i


def test_batch_autotuned_matches_oracle():
    """FP64 batch after the tile autotuner, each matrix against the oracle."""
    mats, kws = _batch_mats(5, 12, np.float64)
    print("batch autotune", flush=True)
    with pod.Batch([_dev(A) for A in mats], [dict(kw, precision=pod.POD_F64) for kw in kws]) as b:
        assert b.autotune() >= 1
        b.run()
        for i, (A, kw) in enumerate(zip(mats, kws)):
            inf, nblk = b.info(i)
            assert nblk >= 1
            U, s, _ = b.project(i)
            ref = oracle_isma(A, IsmaParams(**kw), n_iter=inf.iter, want_v=False)
            rel = np.max(np.abs(s.cpu().numpy() - ref.sigma) / ref.sigma)
            ang = _angles(ref.U, U.cpu().numpy())
            print(f"  matrix {i}: iters={inf.iter} nblk={nblk} sigma_rel={rel:.2e} angle={ang:.2e}", flush=True)
            assert rel <= 1e-10 and ang <= 1e-8


# ------------------------------------------------------------------ reverse mode

@pytest.fixture(scope="module")
def adj_case():
    from oracle import adjoint as adj
    sm = snapgen.spectrum_matrix(500, 100, np.exp(-np.arange(100) / 6.0), 1e-8, seed=1005, centre=False,
                                 v_orthogonal_to_ones=False)
    kw = dict(k=4, c=8, seed=2005, theta_tol=1e-8)
    ref = oracle_isma(sm.A, IsmaParams(**kw), final_step=False)
    return sm.A, kw, adj.col_sets_of(ref.log)


def test_loss_gradient_fp64_matches_oracle_and_fd(adj_case):
    """FP64 gradient of |A - U_k U_k^T A|^2 against the oracle's reverse pass
    and against central differences of the oracle's loss (h = 1e-6)."""
    from oracle import adjoint as adj
    A, kw, cs = adj_case
    print("adjoint fp64", flush=True)
    with pod.PodContext(_dev(A), precision=pod.POD_F64, **kw) as ctx:
        ctx.enable_adjoint()
        ctx.run()
        for it, c in enumerate(cs):
            assert np.array_equal(ctx.indices(it)[0], c)
        L, dA = ctx.loss_grad()
        dA = dA.cpu().numpy()
    Lr, Gr = adj.loss_and_grad(A, cs, 4, 4)
    rel = np.linalg.norm(dA - Gr) / np.linalg.norm(Gr)
    print(f"  loss rel={abs(L - Lr) / Lr:.2e} grad rel={rel:.2e}", flush=True)
    assert abs(L - Lr) <= 1e-10 * Lr
    assert rel <= 1e-8
    rng = np.random.default_rng(3)
    for _ in range(8):
        E = rng.standard_normal(A.shape)
        E /= np.linalg.norm(E)
        fd = adj.fd_directional(A, cs, 4, 4, E)
        an = float(np.sum(dA * E))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-2 * np.linalg.norm(dA))


def test_backward_vjp_fp64_and_autograd(adj_case):
    """pod_backward for given (dU, dsigma) against the oracle (columns of the
    two bases may differ in sign: dU is mapped accordingly), and the same
    through torch.autograd."""
    from oracle import adjoint as adj
    A, kw, cs = adj_case
    rng = np.random.default_rng(4)
    Ad = _dev(A).requires_grad_(True)
    U, s = pod.pod_function(Ad, kw["k"], kw["c"], precision=pod.POD_F64, seed=kw["seed"],
                            theta_tol=kw["theta_tol"])
    dU = rng.standard_normal(U.shape)
    ds = rng.standard_normal(s.shape)
    (U * torch.from_numpy(dU).cuda()).sum().add((s * torch.from_numpy(ds).cuda()).sum()).backward()
    got = Ad.grad.cpu().numpy()
    _, Uo, so = adj.vjp(A, cs, 4, 4)
    sg = np.sign(np.sum(Uo * U.detach().cpu().numpy(), axis=0))
    want, _, _ = adj.vjp(A, cs, 4, 4, dU=dU * sg[None, :], dsigma=ds)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"  vjp rel={rel:.2e}", flush=True)
    assert np.max(np.abs(s.detach().cpu().numpy() - so) / so) <= 1e-10
    assert rel <= 1e-8


def test_loss_gradient_fp32_path(adj_case):
    """FP32 merges, the same reverse pass, against the oracle's FP64 reverse
    pass on the FP32 data and the GPU's draws.  Bound: the forward merges move
    U_k by about u_32 (relative), and the thin-SVD adjoint's coupling
    1 / (s_i^2 - s_j^2) across the truncation amplifies that by at most
    s_1^2 / (s_k^2 - s_{k+1}^2); with the spectrum s_i = e^(-i/6), k = 4 that
    is 9.6, and the tolerance is 100 u_32 times it (5.7e-5; the products'
    length factors stay well inside the 100)."""
    from oracle import adjoint as adj
    A, kw, cs = adj_case
    A32 = A.astype(np.float32)
    with pod.PodContext(_dev(A32), precision=pod.POD_F32, **kw) as ctx:
        ctx.enable_adjoint()
        ctx.run()
        got_cs = [ctx.indices(i)[0] for i in range(ctx.info().iter)]
        L, dA = ctx.loss_grad()
    Lr, Gr = adj.loss_and_grad(A32.astype(np.float64), got_cs, 4, 4)
    rel = np.linalg.norm(dA.cpu().numpy() - Gr) / np.linalg.norm(Gr)
    print(f"  fp32 loss rel={abs(L - Lr) / Lr:.2e} grad rel={rel:.2e}", flush=True)
    u32 = 2.0 ** -24
    s = np.exp(-np.arange(6) / 6.0)
    bound = 100 * u32 * s[0] ** 2 / (s[3] ** 2 - s[4] ** 2)
    assert abs(L - Lr) <= bound * Lr
    assert rel <= bound


@pytest.mark.parametrize("precision", [pod.POD_F64, pod.POD_F32])
def test_batch_loss_gradients(precision):
    """Batched forward with checkpoints, per-matrix reverse pass: equal to the
    single-matrix gradients bit for bit, and (FP64) to the oracle's."""
    from oracle import adjoint as adj
    dtype = np.float64 if precision == pod.POD_F64 else np.float32
    mats, kws = _batch_mats(4, 21, dtype)
    print(f"batch gradients precision={precision}", flush=True)
    dev = [_dev(A) for A in mats]
    with pod.Batch(dev, [dict(kw, precision=precision) for kw in kws]) as b:
        b.enable_adjoint()
        b.run()
        out = [b.loss_grad(i) for i in range(len(mats))]
        cols = [[None]] * len(mats)
    total = 0.0
    for i, (A, kw) in enumerate(zip(mats, kws)):
        with pod.PodContext(dev[i], precision=precision, **kw) as ctx:
            ctx.enable_adjoint()
            ctx.run()
            L, dA = ctx.loss_grad()
            cs = [ctx.indices(t)[0] for t in range(ctx.info().iter)]
        assert L == out[i][0]
        assert torch.equal(dA, out[i][1])
        total += L
        if precision == pod.POD_F64:
            Lr, Gr = adj.loss_and_grad(A, cs, kw["k"], kw["k"])
            rel = np.linalg.norm(dA.cpu().numpy() - Gr) / np.linalg.norm(Gr)
            print(f"  matrix {i}: L={L:.4e} grad rel={rel:.2e}", flush=True)
            assert abs(L - Lr) <= 1e-9 * Lr and rel <= 1e-8
    assert total > 0


@pytest.mark.parametrize("precision", [pod.POD_F64, pod.POD_F32])
def test_batch_loss_gradients_together(precision):
    """The reverse steps of all matrices launched together (loss_grad_all):
    losses and gradients equal to the matrix-by-matrix reverse passes bit for
    bit, for matrices with different merge counts."""
    dtype = np.float64 if precision == pod.POD_F64 else np.float32
    mats, kws = _batch_mats(5, 23, dtype)
    print(f"batch gradients together precision={precision}", flush=True)
    dev = [_dev(A) for A in mats]
    with pod.Batch(dev, [dict(kw, precision=precision) for kw in kws]) as b:
        b.enable_adjoint()
        b.run()
        iters = [b.info(i)[0].iter for i in range(len(mats))]
        each = [b.loss_grad(i) for i in range(len(mats))]
        together = b.loss_grad_all()
    print(f"  merges per matrix {iters}", flush=True)
    assert len(set(iters)) > 1
    for (L1, G1), (L2, G2) in zip(each, together):
        assert L1 == L2
        assert torch.equal(G1, G2)


# ------------------------------------------------------------------ split-BF16 merge path (POD_BF16_REFINE)

@pytest.mark.parametrize("shape", [(20000, 400, 20, 40), (6003, 300, 50, 100)])
def test_bf16_split_before_and_after_refinement(shape):
    """Merge products on BF16 matrix cores with a three-term split: indices
    bit-exact, every convergence sine within 1e-5, the merge-chain state
    (before the final FP32 Rayleigh-Ritz step) within 1e-4 and the final
    modes within 1e-5 of the oracle (sigma relative, largest principal
    angle).  The second shape has p = 150 and a ragged m (not a multiple of 4
    or of the 32-row stage)."""
    m, n, k, c = shape
    A = snapgen.waves_np(m, n, 60, 1.5, 1e-3, seed=1012)
    kw = dict(k=k, c=c, seed=2012, theta_tol=1e-5, max_iter=12)
    print(f"bf16 split m={m} n={n} k={k} c={c}", flush=True)
    with pod.PodContext(_dev(A), precision=pod.POD_BF16_REFINE, **kw) as ctx:
        sines = ctx.run()
        iters = ctx.info().iter
        idx = [ctx.indices(it)[0] for it in range(iters)]
        Ub, sb = ctx.basis()
        Ub, sb = Ub.cpu().numpy(), sb.cpu().numpy()
        U, s, _ = ctx.project(want_v=False)
        U, s = U.cpu().numpy(), s.cpu().numpy()
    ref = oracle_isma(A, IsmaParams(**kw), n_iter=iters, elem_bytes=4)
    assert len(ref.log) == iters
    for it in range(iters):
        assert np.array_equal(idx[it], ref.log[it].cols), it
    for g_s, lg in zip(sines[1:], ref.log[1:]):
        assert abs(g_s - lg.sin_theta) <= 1e-5 * max(1.0, lg.sin_theta) + 1e-12
    rb = np.max(np.abs(sb[:k] - ref.s_merge[:k]) / ref.s_merge[:k])
    ab = _angles(ref.U_merge[:, :k], Ub[:, :k])
    rel = np.max(np.abs(s - ref.sigma) / ref.sigma)
    ang = _angles(ref.U, U)
    print(f"  iters={iters} before: sigma_rel={rb:.3e} angle={ab:.3e}; after: sigma_rel={rel:.3e} angle={ang:.3e}",
          flush=True)
    assert rb <= 1e-4 and ab <= 1e-4
    assert rel <= 1e-5 and ang <= 1e-5


def test_bf16_split_rejected_where_unsupported(c1):
    """A stored in FP64 and the batched driver reject POD_BF16_REFINE."""
    with pytest.raises(pod.PodError):
        pod.PodContext(_dev(c1.A), k=10, c=20, precision=pod.POD_BF16_REFINE)
    A32 = _dev(c1.A.astype(np.float32))
    with pytest.raises(pod.PodError):
        pod.Batch([A32], [dict(k=10, c=20, precision=pod.POD_BF16_REFINE)])


# ------------------------------------------------------------------ quality measure (Eq. ang_meas)

def _wedin_case(A, kw, precision, tol_rs, tol_om):
    from oracle.wedin import wedin_measure
    ref = oracle_isma(A, IsmaParams(**kw), elem_bytes=np.asarray(A).dtype.itemsize)
    _, s_or, _ = oracle.project(np.asarray(A, np.float64), ref.U_merge, want_v=False)
    k = kw["k"]
    with pod.PodContext(_dev(A), precision=precision, **kw) as ctx:
        ctx.run()
        U, sig, V = ctx.project(want_v=True)
        out = ctx.wedin_bound(U, V)
        rn, sn, _, _ = wedin_measure(A, U.cpu().numpy(), sig.cpu().numpy(), V.cpu().numpy(), s_or[k])
    s = sig.cpu().numpy()
    om = min(abs(s[k - 1] - s_or[k]), s[k - 1])
    # R and S from the same modes: only the summation order differs (FP64 on both sides)
    assert out[0] == pytest.approx(rn, rel=tol_rs)
    assert out[1] == pytest.approx(sn, rel=tol_rs, abs=1e-12 * s[0])
    assert out[2] == pytest.approx(om, rel=tol_om)
    assert out[3] == pytest.approx(math.sqrt(out[0] ** 2 + out[1] ** 2) / out[2], rel=1e-12)
    return out


def test_wedin_bound_fp64(c1):
    """C1 (2000 x 500, FP64; ragged against the 256-row stripes and the
    64-column chunks), r = 2k."""
    print("wedin fp64 c1", flush=True)
    out = _wedin_case(c1.A, _c1_params(r=20), pod.POD_F64, 1e-9, 1e-9)
    assert 0.0 < out[3] < math.sqrt(2 * 10)


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_wedin_bound_fp32_paths(waves_small, precision):
    """20000 x 400 FP32 travelling waves, k = 20, r = 30: the modes in FP32,
    the residuals in FP64; omega^ agrees with the oracle's Rayleigh-Ritz
    values to the FP32 path's accuracy."""
    prec = pod.POD_F32 if precision == "f32" else pod.POD_BF16_REFINE
    kw = dict(k=20, c=40, r=30, seed=2002, theta_tol=1e-5)
    print("wedin", precision, flush=True)
    _wedin_case(waves_small, kw, prec, 1e-7, 1e-4)


def test_wedin_bound_state_errors(c1):
    """Before pod_project: POD_ESTATE; with r = k there is no sigma_{k+1}:
    POD_EINVAL."""
    A = _dev(c1.A)
    print("wedin errors", flush=True)
    import ctypes
    with pod.PodContext(A, precision=pod.POD_F64, **_c1_params(r=20)) as ctx:
        ctx.run(n_iter=3)
        U0 = torch.zeros((10, c1.A.shape[0]), dtype=torch.float64, device="cuda")
        V0 = torch.zeros((10, c1.A.shape[1]), dtype=torch.float64, device="cuda")
        with pytest.raises(ValueError):          # the binding refuses pairs no project() returned
            ctx.wedin_bound(U0.T, V0.T)
        out = (ctypes.c_double * 4)()
        st = pod.lib().pod_wedin_bound(ctx.h, ctypes.c_void_p(U0.data_ptr()), ctypes.c_void_p(V0.data_ptr()), out)
        assert st == pod.POD_ESTATE
    with pod.PodContext(A, precision=pod.POD_F64, **_c1_params()) as ctx:
        ctx.run(n_iter=3)
        U, _, V = ctx.project(want_v=True)
        with pytest.raises(pod.PodError) as e:
            ctx.wedin_bound(U, V)
        assert e.value.status == pod.POD_EINVAL


def test_wedin_bound_full_size():
    """The measured workload's size (200,000 x 2,000 FP32 travelling waves,
    k = 20, c = 40, r = 40): ||R|| and ||S|| against FP64 numpy on the same
    modes, omega^ and the bound consistent with the returned values."""
    from oracle.wedin import wedin_measure
    At = snapgen.travelling_waves(200_000, 2_000, 60, 1.5, 1e-3, seed=1002, device="cuda")
    A = At.T
    print("wedin full size", flush=True)
    with pod.PodContext(A, precision=pod.POD_F32, k=20, c=40, r=40, seed=2002, theta_tol=1e-5) as ctx:
        ctx.run()
        U, sig, V = ctx.project(want_v=True)
        out = ctx.wedin_bound(U, V)
    s = sig.cpu().numpy()
    rn, sn, _, _ = wedin_measure(A.cpu().numpy(), U.cpu().numpy(), s, V.cpu().numpy(), 0.0)
    assert out[0] == pytest.approx(rn, rel=1e-8)
    assert out[1] == pytest.approx(sn, rel=1e-6, abs=1e-10 * s[0])
    assert 0.0 < out[2] <= s[-1]
    assert out[3] == pytest.approx(math.sqrt(out[0] ** 2 + out[1] ** 2) / out[2], rel=1e-12)
    assert out[3] < math.sqrt(2 * 20)

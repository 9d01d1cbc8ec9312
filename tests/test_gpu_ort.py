"""ORT column sampling on the GPU (Sec. "Column sampling" (c): probabilities
proportional to the squared residuals of the unsampled columns against the
current modes), through the C ABI, against the oracle.

The GPU forms each residual as nu_j - |U^T a_j|^2 from one projection pass;
the oracle forms a_j - U U^T a_j explicitly.  On FP64 bases the two weights
agree to rounding, and a draw changes only if a target falls inside that
rounding of a cumulative sum (probability ~2^-40 per draw), so indices are
compared bit for bit.  On FP32 bases the weights agree only to FP32, so the
oracle replays the GPU's draws (FP32 bars)."""
import numpy as np
import pytest

import oracle
import snapgen
from oracle.isma import IsmaParams, IterLog, isma as oracle_isma

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1905_05107_amd as pod  # noqa: E402


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


@pytest.mark.parametrize("r", [10, 20])
def test_ort_fp64_indices_and_modes(r):
    """2000 x 500 FP64 (s_i = e^(-i/8), noise variance 1e-8, rows centred),
    k = 10, c = 20, ORT from the second iteration: indices bit-exact per
    iteration, the stop at the same merge, FP64 bars on the result."""
    c1 = snapgen.config_small_fp64()
    kw = dict(k=10, c=20, r=r, seed=2001, theta_tol=1e-10)
    print(f"ort fp64 r={r}", flush=True)
    ref = oracle_isma(c1.A, IsmaParams(col_strategy="ort", **kw))
    with pod.PodContext(_dev(c1.A), col_strategy=pod.POD_COL_ORT, **kw) as ctx:
        ctx.run()
        inf = ctx.info()
        assert inf.iter == len(ref.log)
        for t, lg in enumerate(ref.log):
            cols, cnt = ctx.indices(t)
            assert np.array_equal(cols, lg.cols), t
            assert np.array_equal(cnt, lg.col_counts), t
        U, s, _ = ctx.project(want_v=False)
    rel = np.max(np.abs(s.cpu().numpy() - ref.sigma) / ref.sigma)
    ang = _angles(ref.U, U.cpu().numpy())
    print(f"  iters={inf.iter} stop={pod.STOP_NAMES[inf.stop_reason]} sigma_rel={rel:.2e} angle={ang:.2e}",
          flush=True)
    assert rel <= 1e-10 and ang <= 1e-8
    # ORT draws differ from L2N draws after the first iteration
    l2n = oracle_isma(c1.A, IsmaParams(**kw), n_iter=3, final_step=False)
    assert np.array_equal(l2n.log[0].cols, ref.log[0].cols)
    assert any(not np.array_equal(l2n.log[t].cols, ref.log[t].cols) for t in (1, 2))


def test_ort_fp32_parity_by_replay():
    """20000 x 400 FP32 travelling waves, k = 20, c = 40, r = 30: the oracle
    replays the GPU's ORT draws; FP32 bars (sigma 1e-5, angle 1e-5)."""
    A = snapgen.waves_np(20000, 400, 60, 1.5, 1e-3, seed=1002)
    kw = dict(k=20, c=40, r=30, seed=2002, theta_tol=1e-5)
    print("ort fp32 replay", flush=True)
    with pod.PodContext(_dev(A), precision=pod.POD_F32, col_strategy=pod.POD_COL_ORT, **kw) as ctx:
        ctx.run()
        T = ctx.info().iter
        draws = [ctx.indices(t) for t in range(T)]
        U, s, _ = ctx.project(want_v=False)
    logs = [IterLog(cols=np.asarray(c, np.int64), col_counts=np.asarray(n, np.int32)) for c, n in draws]
    ref = oracle_isma(A, IsmaParams(col_strategy="ort", **kw), n_iter=T, replay=logs, elem_bytes=4)
    own = oracle_isma(A, IsmaParams(col_strategy="ort", **kw), n_iter=min(T, 4), final_step=False, elem_bytes=4)
    same = sum(np.array_equal(own.log[t].cols, draws[t][0]) for t in range(len(own.log)))
    rel = np.max(np.abs(s.cpu().numpy() - ref.sigma) / ref.sigma)
    ang = _angles(ref.U, U.cpu().numpy())
    print(f"  iters={T} oracle's own draws equal in {same}/{len(own.log)} iterations; sigma_rel={rel:.2e} "
          f"angle={ang:.2e}", flush=True)
    assert np.array_equal(own.log[0].cols, draws[0][0])
    assert rel <= 1e-5 and ang <= 1e-5


def test_ort_exhausts_when_the_state_explains_every_column():
    """Exactly rank 2, r = k = 2, c = 40 > n: the first (norm-weighted) draw
    spans the column space, every residual is then zero and the run stops
    exhausted after one merge with the exact singular values."""
    s = np.array([2.0, 1.0])
    sm = snapgen.spectrum_matrix(100, 30, s, 0.0, 2, centre=True)
    print("ort exhaustion", flush=True)
    res = pod.isma(_dev(sm.A), k=2, c=40, r=2, seed=1, theta_tol=0.0, col_strategy=pod.POD_COL_ORT)
    assert res.stopped_by == "exhausted" and res.iters == 1
    assert np.max(np.abs(res.sigma.cpu().numpy() - s) / s) < 1e-12


def test_ort_rejected_by_the_batch():
    A = _dev(np.random.default_rng(0).standard_normal((300, 40)))
    with pytest.raises(pod.PodError):
        pod.Batch([A], [dict(k=2, c=4, col_strategy=pod.POD_COL_ORT)])

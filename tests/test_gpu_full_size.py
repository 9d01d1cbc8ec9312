"""Parity at the measured sizes: the 200,000 x 2,000 travelling-wave workload
(k = 20, c = 40, merge width 60) and a 200,003-row case at merge width 150
(k = 50, c = 100: the wide kernels with a ragged m), each path of the GPU
(FP64, FP32, split-BF16 after its FP32 Rayleigh-Ritz step) against one FP64
oracle run with the same draws (the column weights come from A's bytes, so the
indices are bit-exact on every path)."""
import numpy as np
import pytest

import oracle
import snapgen
from oracle.isma import IsmaParams, isma as oracle_isma

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

import paper_1905_05107_amd as pod  # noqa: E402

BARS = {pod.POD_F64: (1e-10, 1e-8), pod.POD_F32: (1e-5, 1e-5), pod.POD_BF16_REFINE: (1e-5, 1e-5)}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pod.lib()


def _runs(At, kw):
    A = At.T
    out = {}
    for prec in BARS:
        with pod.PodContext(A, precision=prec, **kw) as ctx:
            ctx.run()
            inf = ctx.info()
            cols = [ctx.indices(t)[0] for t in range(inf.iter)]
            U, s, _ = ctx.project(want_v=False)
            out[prec] = (inf.iter, cols, U.cpu().numpy(), s.cpu().numpy(), pod.STOP_NAMES[inf.stop_reason])
    return out


def _check(A_np, kw, out):
    T = out[pod.POD_F64][0]
    ref = oracle_isma(A_np, IsmaParams(**kw), n_iter=T, want_v=False, elem_bytes=4)
    for prec, (iters, cols, U, s, stop) in out.items():
        assert iters == T, prec
        for t in range(T):
            assert np.array_equal(cols[t], ref.log[t].cols), (prec, t)
        rel = np.max(np.abs(s - ref.sigma) / ref.sigma)
        ang = float(np.max(oracle.subspace_sines(ref.U, U.astype(np.float64))))
        print(f"  precision={prec} merges={iters} stop={stop} sigma_rel={rel:.2e} angle={ang:.2e}", flush=True)
        tol_s, tol_a = BARS[prec]
        assert rel <= tol_s and ang <= tol_a, prec


def test_waves_200k_x_2k_every_path_against_one_oracle_run():
    kw = dict(k=20, c=40, seed=2002, theta_tol=1e-5)
    print("full size 200000 x 2000", flush=True)
    At = snapgen.travelling_waves(200_000, 2_000, 60, 1.5, 1e-3, seed=1002, device="cuda")
    out = _runs(At, kw)
    A_np = np.asfortranarray(At.cpu().numpy().T)
    del At
    _check(A_np, kw, out)


def test_merge_width_150_at_200k_rows():
    kw = dict(k=50, c=100, seed=2013, theta_tol=1e-5)
    print("merge width 150, 200003 x 600", flush=True)
    At = snapgen.travelling_waves(200_003, 600, 200, 1.2, 1e-3, seed=1013, device="cuda")
    out = _runs(At, kw)
    A_np = np.asfortranarray(At.cpu().numpy().T)
    del At
    _check(A_np, kw, out)

"""One-shot sampled SVDs of Appendix A on the GPU (pod_oneshot): Alg. 4
(LTSVD) and Alg. 5 (CTSVD) against the oracle's (oracle/oneshot.py) on the
same seeded draws.  The draws are those of the first iteration of Alg. 1
(integer weights from A's bytes), so both sides fold the same columns and
rows; the singular values and the u_i are compared to the FP64 / FP32 bars
(u_i up to sign: the oracle leaves the sign of its Jacobi eigenvectors, the
GPU signs each u_i by its largest entry)."""
import numpy as np
import pytest

import snapgen
from oracle import oneshot as os_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1905_05107_amd as pod  # noqa: E402


def _dev(A_np):
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(A_np).T)).cuda()
    return t.T


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pod.lib()


def _cmp_columns(U, ref, l, tol):
    """max over i < l of |u_i -/+ u_i^ref| / |u_i^ref| (sign of the best match)."""
    worst = 0.0
    for i in range(l):
        a, b = U[:, i].astype(np.float64), ref[:, i]
        d = min(np.linalg.norm(a - b), np.linalg.norm(a + b)) / np.linalg.norm(b)
        worst = max(worst, d)
    assert worst <= tol, worst
    return worst


@pytest.mark.parametrize("kind", ["ltsvd", "ctsvd"])
def test_oneshot_fp64(kind):
    c1 = snapgen.config_small_fp64()
    A = c1.A
    k, c, w, eps, seed = 10, 60, 300, 0.6, 71
    print(f"oneshot {kind} fp64", flush=True)
    if kind == "ltsvd":
        ref = os_oracle.ltsvd(A, k, c, seed)
        U, s, l = pod.oneshot(_dev(A), k, c, seed=seed)
    else:
        ref = os_oracle.ctsvd(A, k, c, w, eps, seed)
        U, s, l = pod.oneshot(_dev(A), k, c, w=w, eps=eps, seed=seed)
    s = s.cpu().numpy()
    U = U.cpu().numpy()
    assert l == ref.l and l >= 1
    rel = np.max(np.abs(s[:l] - ref.sigma) / ref.sigma)
    dU = _cmp_columns(U, ref.U, l, 1e-8)
    print(f"  l={l} sigma_rel={rel:.2e} u_rel={dU:.2e}", flush=True)
    assert rel <= 1e-10
    assert np.all(s[l:] == 0.0) and np.all(U[:, l:] == 0.0)


@pytest.mark.parametrize("kind", ["ltsvd", "ctsvd"])
def test_oneshot_fp32(kind):
    A = snapgen.waves_np(20000, 400, 60, 1.5, 1e-3, seed=1002)
    k, c, w, eps, seed = 20, 100, 800, 0.6, 72
    print(f"oneshot {kind} fp32", flush=True)
    if kind == "ltsvd":
        ref = os_oracle.ltsvd(A, k, c, seed, elem_bytes=4)
        U, s, l = pod.oneshot(_dev(A), k, c, seed=seed, precision=pod.POD_F32)
    else:
        ref = os_oracle.ctsvd(A, k, c, w, eps, seed, elem_bytes=4)
        U, s, l = pod.oneshot(_dev(A), k, c, w=w, eps=eps, seed=seed, precision=pod.POD_F32)
    s = s.cpu().numpy()
    U = U.cpu().numpy()
    assert l == ref.l and l >= 1
    rel = np.max(np.abs(s[:l] - ref.sigma) / ref.sigma)
    dU = _cmp_columns(U, ref.U, l, 1e-4)
    print(f"  l={l} sigma_rel={rel:.2e} u_rel={dU:.2e}", flush=True)
    assert rel <= 1e-5


def test_oneshot_ltsvd_exact_on_low_rank_and_errors():
    """Rank 5 and c well above it: the sample spans the column space, so LTSVD
    returns the exact singular values of A; bad arguments are refused."""
    s0 = np.array([4.0, 2.0, 1.0, 0.5, 0.25])
    sm = snapgen.spectrum_matrix(1200, 150, s0, 0.0, seed=73, centre=False, v_orthogonal_to_ones=False)
    U, s, l = pod.oneshot(_dev(sm.A), 5, 60, seed=74)
    ref = os_oracle.ltsvd(sm.A, 5, 60, 74)
    assert l == 5
    # the scaled sample is not A: its singular values estimate A's (Eq. LTSVD error bound), but the span is exact
    Ug = U.cpu().numpy()
    P = sm.U.T @ Ug
    assert np.linalg.norm(Ug - sm.U @ P) <= 1e-10
    assert np.max(np.abs(s.cpu().numpy() - ref.sigma) / ref.sigma) <= 1e-10
    with pytest.raises(pod.PodError):
        pod.oneshot(_dev(sm.A), 5, 60, w=10, eps=0.0)
    with pytest.raises(pod.PodError):
        pod.oneshot(_dev(sm.A), 100, 100)          # merge width above 160

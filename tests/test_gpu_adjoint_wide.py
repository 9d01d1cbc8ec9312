"""Reverse pass of merges wider than 64 columns on the GPU (through the C ABI)
against the oracle's reverse pass with the same column draws.

A merge of p = r + c columns takes the full eigen-decomposition of R R^T
(recomputed), the adjoint products of the truncated thin SVD (Townsend 2016),
and two passes over [U_{t-1} | A(:, I_t) | Ubar_t] of p + r columns: up to 160
in the staged kernels, up to 208 in the Gram class and the transform with its
right factor read from device memory.  Bars as for the narrow merges: FP64
loss within 1e-10 and gradient within 1e-8 (relative Frobenius) of the oracle,
and the gradient against central differences of the oracle's loss; the FP32
path against the oracle on the FP32 data with the GPU's draws, 100 u_32 times
the truncation gap factor s_1^2 / (s_k^2 - s_{k+1}^2)."""
import numpy as np
import pytest

import snapgen
from oracle import adjoint as adj
from oracle.isma import IsmaParams, isma as oracle_isma

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


TAU = 12.0


def _case(m, n, seed):
    sm = snapgen.spectrum_matrix(m, n, np.exp(-np.arange(min(m, n)) / TAU), 1e-8, seed=seed, centre=False,
                                 v_orthogonal_to_ones=False)
    return sm.A


# (m, n, k, c): p + r = 100 (staged transform), then p + r = 200 (the 208 class)
CASES = [(1500, 360, 20, 60, 3101), (2500, 600, 50, 100, 3102)]


@pytest.mark.parametrize("m,n,k,c,seed", CASES)
def test_wide_merge_gradient_fp64(m, n, k, c, seed):
    A = _case(m, n, seed)
    kw = dict(k=k, c=c, seed=seed + 7, theta_tol=1e-12)
    print(f"adjoint wide fp64 m={m} n={n} k={k} c={c}", flush=True)
    with pod.PodContext(_dev(A), precision=pod.POD_F64, **kw) as ctx:
        ctx.enable_adjoint()
        ctx.run()
        T = ctx.info().iter
        cs = [ctx.indices(t)[0] for t in range(T)]
        L, dA = ctx.loss_grad()
        dA = dA.cpu().numpy()
    ref = oracle_isma(A, IsmaParams(**kw), n_iter=T, final_step=False)
    for t in range(T):
        assert np.array_equal(cs[t], ref.log[t].cols), t
    assert max(len(x) for x in cs) + k > 64, "want merges wider than 64"
    Lr, Gr = adj.loss_and_grad(A, cs, k, k)
    rel = np.linalg.norm(dA - Gr) / np.linalg.norm(Gr)
    print(f"  merges={T} loss rel={abs(L - Lr) / Lr:.2e} grad rel={rel:.2e}", flush=True)
    assert abs(L - Lr) <= 1e-10 * Lr
    assert rel <= 1e-8
    rng = np.random.default_rng(seed)
    for _ in range(2):
        E = rng.standard_normal(A.shape)
        E /= np.linalg.norm(E)
        fd = adj.fd_directional(A, cs, k, k, E)
        an = float(np.sum(dA * E))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-2 * np.linalg.norm(dA))


@pytest.mark.parametrize("m,n,k,c,seed", CASES)
def test_wide_merge_gradient_fp32(m, n, k, c, seed):
    A32 = _case(m, n, seed).astype(np.float32)
    kw = dict(k=k, c=c, seed=seed + 7, theta_tol=1e-12)
    print(f"adjoint wide fp32 m={m} n={n} k={k} c={c}", flush=True)
    with pod.PodContext(_dev(A32), precision=pod.POD_F32, **kw) as ctx:
        ctx.enable_adjoint()
        ctx.run()
        T = ctx.info().iter
        cs = [ctx.indices(t)[0] for t in range(T)]
        L, dA = ctx.loss_grad()
    Lr, Gr = adj.loss_and_grad(A32.astype(np.float64), cs, k, k)
    rel = np.linalg.norm(dA.cpu().numpy() - Gr) / np.linalg.norm(Gr)
    print(f"  merges={T} fp32 loss rel={abs(L - Lr) / Lr:.2e} grad rel={rel:.2e}", flush=True)
    s = np.exp(-np.arange(k + 2) / TAU)
    bound = 100 * 2.0 ** -24 * s[0] ** 2 / (s[k - 1] ** 2 - s[k] ** 2)
    assert abs(L - Lr) <= bound * Lr
    assert rel <= bound


def test_wide_rows_rejected():
    """Row draws keep the narrow limit: a wide row-sampled merge is refused."""
    A = _case(600, 200, 3103)
    with pod.PodContext(_dev(A), precision=pod.POD_F64, k=20, c=60, w=80, seed=3, theta_tol=1e-12) as ctx:
        with pytest.raises(pod.PodError):
            ctx.enable_adjoint()


@pytest.mark.parametrize("m,n,k,c,seed", CASES[1:])
def test_wide_backward_vjp_fp64(m, n, k, c, seed):
    """pod_backward through torch.autograd for given (dU, dsigma) at merge
    width 150 against the oracle's vector-Jacobian product (columns of the two
    bases may differ in sign: dU is mapped accordingly); dsigma exercises the
    singular-value adjoint carried from merge to merge."""
    A = _case(m, n, seed)
    kw = dict(k=k, c=c, seed=seed + 7, theta_tol=1e-12)
    ref = oracle_isma(A, IsmaParams(**kw), final_step=False)
    cs = adj.col_sets_of(ref.log)
    rng = np.random.default_rng(seed + 1)
    Ad = _dev(A).requires_grad_(True)
    print(f"vjp wide fp64 m={m} n={n} k={k} c={c}", flush=True)
    U, s = pod.pod_function(Ad, k, c, precision=pod.POD_F64, seed=kw["seed"], theta_tol=kw["theta_tol"])
    dU = rng.standard_normal(U.shape)
    ds = rng.standard_normal(s.shape)
    (U * torch.from_numpy(dU).cuda()).sum().add((s * torch.from_numpy(ds).cuda()).sum()).backward()
    got = Ad.grad.cpu().numpy()
    _, Uo, so = adj.vjp(A, cs, k, k)
    sg = np.sign(np.sum(Uo * U.detach().cpu().numpy(), axis=0))
    want, _, _ = adj.vjp(A, cs, k, k, dU=dU * sg[None, :], dsigma=ds)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"  merges={len(cs)} vjp rel={rel:.2e}", flush=True)
    assert np.max(np.abs(s.detach().cpu().numpy() - so) / so) <= 1e-10
    assert rel <= 1e-8


@pytest.mark.parametrize("m,n,k,c,seed", CASES)
def test_wide_merge_gradient_fp64_on_fp32_storage(m, n, k, c, seed):
    """The FP64 path on an FP32-stored A (the measured workload's storage):
    FP32 columns widened inside the reverse pass's transform and loss kernels;
    against the oracle on the same values in FP64, FP64 bars."""
    A32 = _case(m, n, seed).astype(np.float32)
    A = A32.astype(np.float64)
    kw = dict(k=k, c=c, seed=seed + 7, theta_tol=1e-12)
    print(f"adjoint wide fp64/fp32-storage m={m} n={n} k={k} c={c}", flush=True)
    with pod.PodContext(_dev(A32), precision=pod.POD_F64, **kw) as ctx:
        ctx.enable_adjoint()
        ctx.run()
        T = ctx.info().iter
        cs = [ctx.indices(t)[0] for t in range(T)]
        L, dA = ctx.loss_grad()
        dA = dA.cpu().numpy()
    assert dA.dtype == np.float64
    Lr, Gr = adj.loss_and_grad(A, cs, k, k)
    rel = np.linalg.norm(dA - Gr) / np.linalg.norm(Gr)
    print(f"  merges={T} loss rel={abs(L - Lr) / Lr:.2e} grad rel={rel:.2e}", flush=True)
    assert abs(L - Lr) <= 1e-10 * Lr
    assert rel <= 1e-8

"""Reverse pass of row-sampled merges on the GPU (through the C ABI) against
the oracle's adjoint with the same frozen draws and row scales.

Each such merge runs on [U S | D V_u], V_u the leading eigenvectors of
W^T W with W the scaled sampled rows of D (Alg. 1, GET UPDATE with rows;
Alg. 2 on the merged block).  Its adjoint has the direct term through V_u
and the eigenvector term through W^T W onto the sampled rows.  Bars: FP64
loss within 1e-10 and gradient within 1e-8 (relative Frobenius) of the
oracle, and the GPU gradient against central differences of the oracle's
loss; FP32 merges against the oracle on the same data, the bound of the
column-only FP32 test (100 u_32 times the truncation gap factor)."""
import numpy as np
import pytest

import snapgen
from oracle import adjoint as adj
from oracle.isma import IsmaParams, IterLog, isma as oracle_isma

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


def _case(seed=2101, m=400, n=90):
    sm = snapgen.spectrum_matrix(m, n, np.exp(-np.arange(min(m, n)) / 7.0), 1e-6, seed=seed, centre=False,
                                 v_orthogonal_to_ones=False)
    return sm.A


KW = dict(k=4, c=10, w=60, seed=2108, theta_tol=1e-8)


@pytest.mark.parametrize("strategy", ["l2", "ls"])
def test_row_merge_gradient_fp64(strategy):
    A = _case()
    rs = pod.POD_ROW_L2 if strategy == "l2" else pod.POD_ROW_LS
    print(f"adjoint rows fp64 {strategy}", flush=True)
    with pod.PodContext(_dev(A), precision=pod.POD_F64, row_strategy=rs, max_iter=5, **KW) as ctx:
        ctx.enable_adjoint()
        ctx.run()
        T = ctx.info().iter
        draws = [ctx.indices(t, rows=True) for t in range(T)]
        L, dA = ctx.loss_grad()
        dA = dA.cpu().numpy()
    prm = IsmaParams(row_strategy=strategy, **KW)
    ref = oracle_isma(A, prm, n_iter=T, final_step=False)
    for t, (c, cc, r, rc) in enumerate(draws):
        assert np.array_equal(c, ref.log[t].cols) and np.array_equal(r, ref.log[t].rows), t
    cs, rows = adj.col_sets_of(ref.log), adj.row_sets_of(ref.log)
    assert any(ru < len(c) for (_, _, ru), c in zip(rows, cs)), "want truncated row blocks"
    Lr, Gr = adj.loss_and_grad(A, cs, prm.k, prm.rank, row_sets=rows)
    rel = np.linalg.norm(dA - Gr) / np.linalg.norm(Gr)
    print(f"  merges={T} loss rel={abs(L - Lr) / Lr:.2e} grad rel={rel:.2e}", flush=True)
    assert abs(L - Lr) <= 1e-10 * Lr
    assert rel <= 1e-8
    rng = np.random.default_rng(5)
    for _ in range(3):
        E = rng.standard_normal(A.shape)
        E /= np.linalg.norm(E)
        fd = adj.fd_directional(A, cs, prm.k, prm.rank, E, row_sets=rows)
        an = float(np.sum(dA * E))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-2 * np.linalg.norm(dA))


def test_row_merge_gradient_differs_from_column_chain():
    """The same draws through column-only merges give a different gradient:
    the rows path is really taken."""
    A = _case()
    with pod.PodContext(_dev(A), precision=pod.POD_F64, max_iter=5, **KW) as ctx:
        ctx.enable_adjoint()
        ctx.run()
        T = ctx.info().iter
        _, dA = ctx.loss_grad()
        dA = dA.cpu().numpy()
    ref = oracle_isma(A, IsmaParams(**KW), n_iter=T, final_step=False)
    _, G0 = adj.loss_and_grad(A, adj.col_sets_of(ref.log), KW["k"], KW["k"])
    assert np.linalg.norm(dA - G0) > 1e-3 * np.linalg.norm(G0)


def test_row_merge_gradient_fp32():
    A32 = _case().astype(np.float32)
    print("adjoint rows fp32", flush=True)
    with pod.PodContext(_dev(A32), precision=pod.POD_F32, max_iter=5, **KW) as ctx:
        ctx.enable_adjoint()
        ctx.run()
        T = ctx.info().iter
        draws = [ctx.indices(t, rows=True) for t in range(T)]
        L, dA = ctx.loss_grad()
    logs = [IterLog(cols=np.asarray(c, np.int64), col_counts=np.asarray(cc, np.int32),
                    rows=np.asarray(r, np.int64), row_counts=np.asarray(rc, np.int32)) for c, cc, r, rc in draws]
    prm = IsmaParams(**KW)
    ref = oracle_isma(A32.astype(np.float64), prm, n_iter=T, replay=logs, final_step=False, elem_bytes=4)
    cs, rows = adj.col_sets_of(ref.log), adj.row_sets_of(ref.log)
    Lr, Gr = adj.loss_and_grad(A32.astype(np.float64), cs, prm.k, prm.rank, row_sets=rows)
    rel = np.linalg.norm(dA.cpu().numpy() - Gr) / np.linalg.norm(Gr)
    print(f"  merges={T} fp32 loss rel={abs(L - Lr) / Lr:.2e} grad rel={rel:.2e}", flush=True)
    u32 = 2.0 ** -24
    s = np.exp(-np.arange(6) / 7.0)
    bound = 100 * u32 * s[0] ** 2 / (s[3] ** 2 - s[4] ** 2)
    assert abs(L - Lr) <= bound * Lr
    assert rel <= bound

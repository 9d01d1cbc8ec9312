"""Pins of the oracle's adjoint of row-sampled merges (ICRS, CPU only).

The draws (columns and rows) and the row scales are frozen (the scales come
from quantised row weights: piecewise constant in A).  Pins: central finite
differences of the loss through row-sampled merges with truncated blocks
(r_u < g); with every row kept at unit scale and r_u = g the merged subspace
is that of the columns, so the gradient equals the column-only one (the
eigenvector term must cancel there); the eigenvector term is large enough
elsewhere that leaving it out fails the finite differences; and the forward
of the adjoint reproduces the merges of oracle.isma's row-sampled runs."""
import numpy as np
import pytest

import snapgen
from oracle import adjoint as adj
from oracle.isma import IsmaParams, isma


def _run(row_strategy="l2", seed=2101, m=400, n=90, k=4, c=10, w=60):
    sm = snapgen.spectrum_matrix(m, n, np.exp(-np.arange(min(m, n)) / 7.0), 1e-6, seed=seed, centre=False,
                                 v_orthogonal_to_ones=False)
    prm = IsmaParams(k=k, c=c, w=w, seed=seed + 7, theta_tol=1e-8, row_strategy=row_strategy)
    ref = isma(sm.A, prm, final_step=False, n_iter=5)
    return sm.A, ref, adj.col_sets_of(ref.log), adj.row_sets_of(ref.log), prm


@pytest.fixture(scope="module")
def l2_run():
    return _run("l2")


def test_row_scales_logged_and_truncated(l2_run):
    A, ref, cs, rs_, prm = l2_run
    assert all(r is not None for r in rs_)
    assert any(r_u < len(c) for (rows, sc, r_u), c in zip(rs_, cs)), "want truncated row blocks"
    for (rows, sc, r_u) in rs_:
        assert rows.shape == sc.shape and np.all(sc > 0)


@pytest.mark.parametrize("strategy", ["l2", "ls"])
def test_forward_equals_oracle_row_merges(strategy):
    A, ref, cs, rs_, prm = _run(strategy)
    U, s, _ = adj.forward(A, cs, prm.rank, rs_)
    assert np.max(np.abs(s - ref.s_merge) / ref.s_merge) <= 1e-10
    Q = U - ref.U_merge @ (ref.U_merge.T @ U)
    assert np.linalg.norm(Q, 2) <= 1e-8


def test_row_gradient_matches_central_differences(l2_run):
    A, ref, cs, rs_, prm = l2_run
    L, G = adj.loss_and_grad(A, cs, prm.k, prm.rank, row_sets=rs_)
    rng = np.random.default_rng(11)
    for _ in range(3):
        E = rng.standard_normal(A.shape)
        fd = adj.fd_directional(A, cs, prm.k, prm.rank, E, 1e-6, row_sets=rs_)
        assert abs(fd - float(np.sum(G * E))) <= 1e-6 * abs(fd)


def test_unit_rows_full_block_equals_column_chain(l2_run):
    A, ref, cs, rs_, prm = l2_run
    m = A.shape[0]
    rows_all = [(np.arange(m), np.ones(m), len(c)) for c in cs]
    L1, G1 = adj.loss_and_grad(A, cs, prm.k, prm.rank, row_sets=rows_all)
    L0, G0 = adj.loss_and_grad(A, cs, prm.k, prm.rank)
    assert abs(L1 - L0) <= 1e-10 * L0
    assert np.max(np.abs(G1 - G0)) <= 1e-9 * np.max(np.abs(G0))


def test_eigenvector_term_is_needed(l2_run, monkeypatch):
    """Without the eigenvector path (D-bar = C-bar V_u^T only) the gradient
    misses the finite differences by far more than their error."""
    A, ref, cs, rs_, prm = l2_run
    L, G = adj.loss_and_grad(A, cs, prm.k, prm.rank, row_sets=rs_)

    def direct_only(rb, Cbar, eta):
        rows, scales, r_u, D, W, lam, V = rb
        return Cbar @ V[:, :r_u].T

    monkeypatch.setattr(adj, "_row_block_adjoint", direct_only)
    _, Gd = adj.loss_and_grad(A, cs, prm.k, prm.rank, row_sets=rs_)
    E = np.random.default_rng(12).standard_normal(A.shape)
    monkeypatch.undo()
    fd = adj.fd_directional(A, cs, prm.k, prm.rank, E, 1e-6, row_sets=rs_)
    assert abs(fd - float(np.sum(G * E))) <= 1e-6 * abs(fd)
    assert abs(fd - float(np.sum(Gd * E))) >= 1e-3 * abs(fd)

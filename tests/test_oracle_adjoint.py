"""Pins of the oracle's adjoint of the merge chain (CPU only).

Central finite differences of the loss with the sampled columns frozen
(h = 1e-6 on a 500 x 100 FP64 matrix with s_i = exp(-i/6), k = 4, c = 8,
and every entry of a small case), the closed form of the gradient when a
single merge sees every column, and the forward pass against the C oracle's
merges."""
import numpy as np
import pytest

import snapgen
from oracle import adjoint as adj
from oracle.isma import IsmaParams, isma


def _case(m, n, tau, k, c, seed, r=None):
    sm = snapgen.spectrum_matrix(m, n, np.exp(-np.arange(min(m, n)) / tau), 1e-8, seed=seed, centre=False,
                                 v_orthogonal_to_ones=False)
    prm = IsmaParams(k=k, c=c, r=r, seed=seed + 1000, theta_tol=1e-8)
    ref = isma(sm.A, prm, final_step=False)
    return sm.A, ref, adj.col_sets_of(ref.log)


@pytest.fixture(scope="module")
def fd_case():
    return _case(500, 100, 6.0, 4, 8, 1005)


def test_forward_equals_oracle_merges(fd_case):
    A, ref, cs = fd_case
    U, s, _ = adj.forward(A, cs, 4)
    assert np.max(np.abs(s - ref.s_merge) / ref.s_merge) <= 1e-12
    # same subspace
    Q = U - ref.U_merge @ (ref.U_merge.T @ U)
    assert np.linalg.norm(Q, 2) <= 1e-10


@pytest.mark.parametrize("r", [4, 8])
def test_gradient_matches_central_differences(fd_case, r):
    A, _, cs = fd_case
    L, G = adj.loss_and_grad(A, cs, 4, r)
    assert L > 0
    rng = np.random.default_rng(r)
    gn = np.linalg.norm(G)
    for _ in range(32):
        E = rng.standard_normal(A.shape)
        E /= np.linalg.norm(E)
        fd = adj.fd_directional(A, cs, 4, r, E, h=1e-6)
        an = float(np.sum(G * E))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-2 * gn), (fd, an)


def test_gradient_every_entry_small_case():
    A, _, cs = _case(40, 16, 3.0, 3, 6, 77)
    assert len(cs) >= 2
    _, G = adj.loss_and_grad(A, cs, 3, 3)
    h = 1e-6
    scale = np.max(np.abs(G))
    for i in range(A.shape[0]):
        for j in range(A.shape[1]):
            E = np.zeros_like(A)
            E[i, j] = 1.0
            fd = adj.fd_directional(A, cs, 3, 3, E, h=h)
            assert abs(fd - G[i, j]) <= 1e-6 * scale, (i, j, fd, G[i, j])


def test_closed_form_when_one_merge_sees_all_columns(fd_case):
    A, _, _ = fd_case
    n = A.shape[1]
    L, G = adj.loss_and_grad(A, [np.arange(n)], 4, 4)
    s = np.linalg.svd(A, compute_uv=False)
    assert abs(L - np.sum(s[4:] ** 2)) <= 1e-12 * np.sum(s ** 2)
    U = np.linalg.svd(A, full_matrices=False)[0][:, :4]
    Gc = 2.0 * (A - U @ (U.T @ A))
    assert np.linalg.norm(G - Gc) <= 1e-10 * np.linalg.norm(Gc)


def test_indirect_term_is_not_negligible(fd_case):
    """With several merges the gradient differs from the explicit term."""
    A, _, cs = fd_case
    _, G = adj.loss_and_grad(A, cs, 4, 4)
    U, _, _ = adj.forward(A, cs, 4)
    Uk = U[:, :4]
    Ge = 2.0 * (A - Uk @ (Uk.T @ A))
    assert np.linalg.norm(G - Ge) >= 1e-3 * np.linalg.norm(G)


def test_vjp_of_singular_values_matches_central_differences(fd_case):
    """The reverse pass from Sigma-bar alone: f(A) = <w, Sigma_k(A)>."""
    A, _, cs = fd_case
    w = np.array([1.0, -0.5, 0.25, 2.0])
    dA, _, _ = adj.vjp(A, cs, 4, 4, dsigma=w)
    rng = np.random.default_rng(5)

    def f(X):
        return float(np.dot(w, adj.forward(X, cs, 4)[1][:4]))

    for _ in range(8):
        E = rng.standard_normal(A.shape)
        E /= np.linalg.norm(E)
        fd = (f(A + 1e-6 * E) - f(A - 1e-6 * E)) / 2e-6
        an = float(np.sum(dA * E))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-2 * np.linalg.norm(dA))


def test_loss_gradient_equals_explicit_plus_vjp(fd_case):
    """loss_and_grad = 2R + vjp(U-bar = -2 R B^T): the two entry points agree."""
    A, _, cs = fd_case
    L, G = adj.loss_and_grad(A, cs, 4, 4)
    U, _, _ = adj.forward(A, cs, 4)
    Uk = U[:, :4]
    B = Uk.T @ A
    R = A - Uk @ B
    dA, _, _ = adj.vjp(A, cs, 4, 4, dU=-2.0 * R @ B.T)
    assert np.linalg.norm(G - (2.0 * R + dA)) <= 1e-13 * np.linalg.norm(G)

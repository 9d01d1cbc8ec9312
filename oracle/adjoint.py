"""Adjoint of the ISMA merge chain (TEST INFRASTRUCTURE ONLY).

Loss: L(A) = || A - U_k U_k^T A ||_F^2 with U_k the first k columns of the
basis the merges of Alg. 1 (Alg. 2, BLOCK MERGE) end with, the sampled
columns of every iteration held fixed (the draw is piecewise constant in A).

Forward: merge t forms M_t = [U_{t-1} Sigma_{t-1} | A(:, I_t)], takes its full
thin SVD M_t = U S V^T (LAPACK through numpy, a library step) and keeps
r_t = min(r, #{s_i > p u s_1}) leading pairs (the rank guard of Alg. 2).

Backward (reverse mode, every intermediate of the forward stored): the
adjoint of a thin SVD restricted to the leading r columns (Townsend 2016,
"Differentiating the Singular Value Decomposition"; Ionescu, Vantzos &
Sminchisescu 2015) with V-bar = 0:

    M-bar = U [ (F o (J - J^T)) S + diag(s-bar) ] V^T
            + (I - U U^T) U-bar S_r^-1 V_r^T,       J = U^T U-bar (p x p,
                                                     zero beyond column r),
    F_ij = d_ij / (d_ij^2 + eta^2 s_1^4), d_ij = s_j^2 - s_i^2 (i != j), F_ii = 0

(the eta term is a guard against near-equal pairs: F_ij = 1/(s_j^2 - s_i^2)
whenever |d_ij| >> eta s_1^2).  M-bar splits into the adjoint of
U_{t-1} Sigma_{t-1} -- giving U-bar_{t-1} = M-bar(:, :rs) Sigma_{t-1} and
s-bar_{t-1,i} = u_i^T M-bar(:, i) -- and that of the sampled columns, added
to dA(:, I_t).  The loss contributes 2 (A - U_k B) to dA directly and
U-bar = -2 (A - U_k B) B^T with B = U_k^T A.

Row-sampled merges (ICRS, Alg. 1 SAMPLE AND SCALE UNIQUE ROWS): the block
merged is C = D V_u with D = A(:, I_t), V_u the leading r_u eigenvectors of
G = W^T W, W = diag(s) D(I_r, :).  The draws (I_t, I_r) and the scales s
(functions of the quantised, hence piecewise constant, row weights) are held
fixed.  With C-bar the adjoint of C (the columns of M-bar beyond the basis):

    D-bar = C-bar V_u^T + [rows I_r] diag(s) W-bar,   W-bar = 2 W G-bar_s,
    G-bar = V K V^T,  K_ij = (v_i^T V-bar_j) / (lambda_j - lambda_i) (i != j,
    j < r_u; 0 otherwise),  V-bar_u = D^T C-bar,  G-bar_s = (G-bar + G-bar^T) / 2

(the first-order perturbation of the eigenvectors of a symmetric matrix,
dv_j = sum_{i != j} v_i (v_i^T dG v_j) / (lambda_j - lambda_i), with V the
full eigenbasis of G and the same eta guard on the denominators).

Pins: central finite differences of the loss, and the closed form
dL/dA = 2 (I - U_k U_k^T) A when one merge sees every column (the merge is
then the exact truncated SVD, where the indirect term vanishes).  For the rows:
finite differences with the draws and scales frozen, and, with every row kept
at unit scale and r_u = g (C = D V, V orthogonal, so the merged subspace is
that of D), the gradient of the column-only chain.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

U_F64 = 2.0 ** -53


def row_block(D, rows, scales, r_u: int):
    """The row-sampled merge input of one iteration: (C, W, lambda, V) with
    W = diag(s) D(I_r, :), G = W^T W = V diag(lambda) V^T (descending; LAPACK
    through numpy, a library step) and C = D V(:, :r_u)."""
    rows = np.asarray(rows, dtype=np.int64)
    W = np.asarray(scales, dtype=np.float64)[:, None] * D[rows, :]
    lam, V = np.linalg.eigh(W.T @ W)
    lam, V = lam[::-1], V[:, ::-1]
    return D @ V[:, :r_u], W, lam, V


def forward(A, col_sets: Sequence[np.ndarray], r: int, row_sets=None):
    """Merge chain on the fixed column sets (and, for row-sampled iterations,
    row_sets[t] = (rows, scales, r_u); None: the columns merged as drawn).
    Returns (U, s, tape)."""
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    U = np.zeros((m, 0))
    s = np.zeros(0)
    tape = []
    for t, cols in enumerate(col_sets):
        cols = np.asarray(cols, dtype=np.int64)
        D = A[:, cols]
        rb = None
        if row_sets is not None and row_sets[t] is not None:
            rows, scales, r_u = row_sets[t]
            C, W, lam, V = row_block(D, rows, scales, r_u)
            rb = (np.asarray(rows, dtype=np.int64), np.asarray(scales, dtype=np.float64), r_u, D, W, lam, V)
        else:
            C = D
        M = np.hstack([U * s[None, :], C])
        Uf, sf, Vt = np.linalg.svd(M, full_matrices=False)
        p = M.shape[1]
        rr = int(min(r, np.sum(sf > p * U_F64 * sf[0]))) if sf.size and sf[0] > 0 else 0
        tape.append((U, s, cols, Uf, sf, Vt.T, rr, rb))
        U, s = Uf[:, :rr], sf[:rr]
    return U, s, tape


def loss(A, col_sets, k: int, r: int, row_sets=None) -> float:
    A = np.asarray(A, dtype=np.float64)
    U, _, _ = forward(A, col_sets, r, row_sets)
    Uk = U[:, :k]
    R = A - Uk @ (Uk.T @ A)
    return float(np.sum(R * R))


def _reverse(tape, Ubar, sbar, dA, eta):
    """Reverse pass over the merges from the adjoints (Ubar, sbar) of the final
    state; adds the adjoint of every sampled block to dA."""
    for (U0, s0, cols, Uf, sf, V, rr, rb) in reversed(tape):
        p = sf.size
        J = np.zeros((p, p))
        J[:, :rr] = Uf.T @ Ubar
        d = sf[None, :] ** 2 - sf[:, None] ** 2
        F = d / (d * d + (eta * sf[0] ** 2) ** 2) if sf[0] > 0 else np.zeros_like(d)
        np.fill_diagonal(F, 0.0)
        K = (F * (J - J.T)) * sf[None, :]
        K[np.arange(rr), np.arange(rr)] += sbar
        Mbar = Uf @ K @ V.T
        if rr:
            Mbar += ((Ubar - Uf @ J[:, :rr]) / sf[None, :rr]) @ V[:, :rr].T
        rs = s0.size
        if rb is None:
            dA[:, cols] += Mbar[:, rs:]
        else:
            dA[:, cols] += _row_block_adjoint(rb, Mbar[:, rs:], eta)
        Ubar = Mbar[:, :rs] * s0[None, :]
        sbar = np.sum(U0 * Mbar[:, :rs], axis=0)
    return dA


def _row_block_adjoint(rb, Cbar, eta):
    """D-bar of a row-sampled merge input from C-bar (module docstring)."""
    rows, scales, r_u, D, W, lam, V = rb
    g = V.shape[0]
    Dbar = Cbar @ V[:, :r_u].T
    Vbar = D.T @ Cbar                                   # g x r_u
    d = lam[None, :] - lam[:, None]                     # d_ij = lambda_j - lambda_i
    scale = eta * max(abs(lam[0]), 0.0) if g else 0.0
    F = d / (d * d + scale * scale) if scale > 0 else np.where(d != 0, 1.0 / np.where(d != 0, d, 1.0), 0.0)
    np.fill_diagonal(F, 0.0)
    K = np.zeros((g, g))
    K[:, :r_u] = (V.T @ Vbar) * F[:, :r_u]
    Gbar = V @ K @ V.T
    Gs = 0.5 * (Gbar + Gbar.T)
    Wbar = 2.0 * W @ Gs
    np.add.at(Dbar, rows, scales[:, None] * Wbar)
    return Dbar


def loss_and_grad(A, col_sets, k: int, r: int, eta: float = 1e-12, row_sets=None):
    """(L, dL/dA) by the reverse pass described in the module docstring."""
    A = np.asarray(A, dtype=np.float64)
    U, s, tape = forward(A, col_sets, r, row_sets)
    kk = min(k, U.shape[1])
    Uk = U[:, :kk]
    B = Uk.T @ A
    R = A - Uk @ B
    L = float(np.sum(R * R))
    Ubar = np.zeros_like(U)
    Ubar[:, :kk] = -2.0 * R @ B.T
    dA = _reverse(tape, Ubar, np.zeros(U.shape[1]), 2.0 * R, eta)
    return L, dA


def vjp(A, col_sets, k: int, r: int, dU=None, dsigma=None, eta: float = 1e-12, row_sets=None):
    """dA for the adjoints dU (m x k) and dsigma (k) of the first k merged
    modes and singular values (U_k, Sigma_k).  Returns (dA, U_k, Sigma_k)."""
    A = np.asarray(A, dtype=np.float64)
    U, s, tape = forward(A, col_sets, r, row_sets)
    kk = min(k, U.shape[1])
    Ubar = np.zeros_like(U)
    sbar = np.zeros(U.shape[1])
    if dU is not None:
        Ubar[:, :kk] = np.asarray(dU, dtype=np.float64)[:, :kk]
    if dsigma is not None:
        sbar[:kk] = np.asarray(dsigma, dtype=np.float64)[:kk]
    dA = _reverse(tape, Ubar, sbar, np.zeros_like(A), eta)
    return dA, U[:, :kk], s[:kk]


def col_sets_of(logs) -> List[np.ndarray]:
    """The column sets of a run's iteration logs (oracle.isma's IterLog)."""
    return [np.asarray(lg.cols, dtype=np.int64) for lg in logs]


def row_sets_of(logs):
    """The row sets (rows, scales, r_u) of a run's iteration logs (None for an
    iteration without rows)."""
    return [None if lg.rows is None else (np.asarray(lg.rows, dtype=np.int64), np.asarray(lg.row_scales), int(lg.r_u))
            for lg in logs]


def fd_directional(A, col_sets, k: int, r: int, E, h: float = 1e-6, row_sets=None) -> float:
    """Central difference (L(A + h E) - L(A - h E)) / (2 h)."""
    return (loss(A + h * E, col_sets, k, r, row_sets) - loss(A - h * E, col_sets, k, r, row_sets)) / (2.0 * h)

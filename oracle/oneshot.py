"""One-shot sampled SVDs of Appendix A (TEST INFRASTRUCTURE ONLY).

Alg. 4 (LTSVD) and Alg. 5 (CTSVD), the column / column-and-row norm sampled
SVDs the paper evaluates before proposing ISMA, and the SVD-A^T A truth of
Sec. 4 (Table 1), in FP64 on top of the C primitives of ``pod_oracle.c``.

Readings shared with the iterative driver (``isma.py``):
  * the probabilities p_j of Eq. (LTSVD_prob) are the integer sampling
    weights w_j / W the Philox draw actually uses (key (seed, 0), counter
    (0, d/4, block, 0)); rows (Alg. 5) use key (seed, 1);
  * draws with replacement are folded into their distinct indices: a column
    drawn t_j times enters once, scaled by sqrt(t_j / (c p_j)) instead of
    t_j copies scaled by 1/sqrt(c p_j).  C C^T is unchanged (sum over the draws
    of a a^T / (c p)), so are the left singular vectors, the singular values
    and u~_i = C v~_i / sigma~_i (the right factors differ only by a matrix
    with orthonormal rows); likewise for the rows of W (the identity of SAMPLE
    AND SCALE UNIQUE ROWS);
  * the scale is evaluated as sqrt((t_j W) / (c w_j)) with t_j, W, c and w_j
    converted to FP64.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import col_sqnorms, draw, jacobi_eig, quantize, row_sqnorms, unique

U_F64 = 2.0 ** -53


@dataclass
class OneShot:
    U: np.ndarray          # m x l (u~_i = C v~_i / sigma~_i)
    sigma: np.ndarray      # l
    cols: np.ndarray       # distinct sampled columns (ascending)
    col_counts: np.ndarray
    col_scale: np.ndarray  # sqrt(t_j / (c p_j)) per distinct column
    rows: Optional[np.ndarray] = None
    row_counts: Optional[np.ndarray] = None
    row_scale: Optional[np.ndarray] = None
    l: int = 0


def _scaled_columns(X, c, seed, block, elem_bytes):
    """The first loop of Alg. 4 / Alg. 5: c draws of columns with the norm
    probabilities of Eq. (LTSVD_prob), folded into the distinct columns, each
    scaled by sqrt(t_j / (c p_j))."""
    nu = col_sqnorms(X, elem_bytes)
    wq = quantize(nu)
    draws, W = draw(wq, c, seed, 0, 0, block)
    if W == 0:
        raise ValueError("every column has zero norm")
    cols, cnt = unique(draws)
    scale = np.array([np.sqrt((float(int(t)) * float(W)) / (float(c) * float(int(wq[j]))))
                      for j, t in zip(cols, cnt)])
    C = np.asfortranarray(X[:, cols] * scale[None, :])
    return C, cols, cnt, scale


def _left_vectors(C, G, l):
    """Step of Alg. 4 / Alg. 5: V~ Sigma~^2 V~^T = SVD(G) (G = C^T C or W^T W;
    Jacobi eigen-decomposition, descending), u~_i = C v~_i / sigma~_i."""
    ev, V = jacobi_eig(G)
    sig = np.sqrt(np.maximum(ev[:l], 0.0))
    U = np.asfortranarray(C @ V[:, :l] / sig[None, :]) if l else np.zeros((C.shape[0], 0))
    return U, sig, ev


def ltsvd(A, k: int, c: int, seed: int, block: int = 0, elem_bytes: Optional[int] = None) -> OneShot:
    """Alg. 4 (LTSVD): l = min(k, rank C) left singular pairs of the scaled
    column sample C.  Reading: rank C = #{lambda_i > g u lambda_1} of the
    eigenvalues of C^T C (g = distinct columns)."""
    if elem_bytes is None:
        elem_bytes = np.asarray(A).dtype.itemsize
    X = np.asfortranarray(np.asarray(A, dtype=np.float64))
    C, cols, cnt, scale = _scaled_columns(X, c, seed, block, elem_bytes)
    G = C.T @ C
    ev, _ = jacobi_eig(G)
    g = C.shape[1]
    rank = int(np.sum(ev > g * U_F64 * max(ev[0], 0.0))) if g else 0
    l = min(int(k), rank)
    U, sig, _ = _left_vectors(C, G, l)
    return OneShot(U, sig, cols, cnt, scale, l=l)


def ctsvd(A, k: int, c: int, w: int, eps: float, seed: int, block: int = 0,
          elem_bytes: Optional[int] = None) -> OneShot:
    """Alg. 5 (CTSVD): columns as in Alg. 4; row probabilities
    q_i = |c^i|^2 / |C|_F^2 of the scaled sample (Eq. CTSVD_prob_col); w row
    draws folded into the distinct rows, each scaled by sqrt(t^_i / (w q_i));
    V~ Sigma~^2 V~^T = SVD(W^T W); gamma = eps / (100 k);
    l = min(k, max{r : sigma~_r^2 >= gamma |W|_F^2}); u~_i = C v~_i / sigma~_i.
    The u~_i are not orthonormal in general."""
    if elem_bytes is None:
        elem_bytes = np.asarray(A).dtype.itemsize
    X = np.asfortranarray(np.asarray(A, dtype=np.float64))
    C, cols, cnt, scale = _scaled_columns(X, c, seed, block, elem_bytes)
    wr = quantize(row_sqnorms(C))
    rdraws, Om = draw(wr, w, seed, 1, 0, block)
    if Om == 0:
        raise ValueError("every sampled row has zero norm")
    rows, rcnt = unique(rdraws)
    rscale = np.array([np.sqrt((float(int(t)) * float(Om)) / (float(w) * float(int(wr[i]))))
                       for i, t in zip(rows, rcnt)])
    W = C[rows, :] * rscale[:, None]
    G = W.T @ W
    ev, _ = jacobi_eig(G)
    wf2 = float(np.sum(W * W))
    gamma = float(eps) / (100.0 * float(k))
    keep = np.flatnonzero(ev >= gamma * wf2)
    l = min(int(k), int(keep[-1]) + 1 if keep.size else 0)
    U, sig, _ = _left_vectors(C, G, l)
    return OneShot(U, sig, cols, cnt, scale, rows, rcnt, rscale, l)


def svd_ata(A, k: int):
    """The SVD-A^T A truth of Sec. 4: eigen-decomposition of A^T A (LAPACK
    through numpy, a library step), descending, and U_k = A V_k Sigma_k^-1."""
    X = np.asarray(A, dtype=np.float64)
    ev, V = np.linalg.eigh(X.T @ X)
    order = np.argsort(ev)[::-1][:k]
    sig = np.sqrt(np.maximum(ev[order], 0.0))
    U = X @ V[:, order] / sig[None, :]
    return U, sig

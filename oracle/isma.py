"""ISMA driver of the oracle (TEST INFRASTRUCTURE ONLY).

Follows the paper's Alg. 1 (ISMA with GET UPDATE and SAMPLE AND SCALE UNIQUE
ROWS), Alg. 2 (BLOCK MERGE) and Alg. 3 (incremental POD) step by step, in FP64,
on top of the C primitives of ``pod_oracle.c``.  Readings of passages where the
paper is silent or ambiguous are marked "Reading:".
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

from . import (col_sqnorms, draw, jacobi_eig, merge, project, quantize, row_sqnorms,
               subspace_sines, unique)

U_F64 = 2.0 ** -53
# ORT residuals at or below this fraction of |a_i|^2 count as zero (FP64 runs)
ORT_FLOOR_F64 = 1e-12


@dataclass
class IsmaParams:
    """Inputs of Alg. 1: ISMA(A, p, k, c, w, r, tau, rows).

    rows = 1 in the paper  <=>  w > 0 here.  The tolerance is an angle:
    the iteration stops when the largest angle between successive estimates
    is below ``theta_tol`` (the paper's tau is its cosine, tau = 0.99 in its
    experiments).  ``r`` defaults to k.  ``r_update`` > 0 truncates each new
    block to its top r_update right singular directions before the merge
    (the paper's GET UPDATE without rows); 0 merges the distinct columns as
    they are.  Reading: merging [U S | D] equals the paper's merge with the
    block's full SVD, since an orthogonal right factor changes neither the
    left singular vectors nor the singular values."""
    k: int
    c: int
    w: int = 0
    r: Optional[int] = None
    theta_tol: float = 1e-10
    col_strategy: str = "l2n"      # "l2n" | "unf" | "ort"
    row_strategy: str = "l2"       # "l2" | "ls"
    criterion: str = "subspace"    # "subspace" | "mode"
    max_iter: int = 1 << 30
    seed: int = 0
    r_update: int = 0
    block: int = 0

    @property
    def rank(self) -> int:
        return self.r if self.r else self.k


@dataclass
class IterLog:
    cols: np.ndarray
    col_counts: np.ndarray
    rows: Optional[np.ndarray] = None
    row_counts: Optional[np.ndarray] = None
    row_scales: Optional[np.ndarray] = None   # sqrt(t_hat_i / (w q_i)) of the kept rows
    r_u: int = 0
    rank: int = 0
    sin_theta: float = float("nan")
    sigma: Optional[np.ndarray] = None


@dataclass
class IsmaResult:
    U: np.ndarray            # m x k after the final step (Rayleigh-Ritz)
    sigma: np.ndarray        # k
    V: Optional[np.ndarray]  # n x k
    U_merge: np.ndarray      # m x r' state at the end of the iteration
    s_merge: np.ndarray
    log: List[IterLog] = field(default_factory=list)
    converged: bool = False
    exhausted: bool = False


def sample_size_ltsvd(k: int, eps: float, delta: float) -> int:
    """Eq. (c_LTSVD): c = 4k (1 + sqrt(8 ln(1/delta)))^2 / eps^2, rounded up."""
    return int(math.ceil(4.0 * k * (1.0 + math.sqrt(8.0 * math.log(1.0 / delta))) ** 2 / eps ** 2))


def sample_size_ctsvd(k: int, eps: float, delta: float) -> int:
    """Eq. (c_w_CTSVD): c = w = k^2 (1 + sqrt(ln(2/delta)))^2 / eps^4, rounded up."""
    return int(math.ceil(k * k * (1.0 + math.sqrt(math.log(2.0 / delta))) ** 2 / eps ** 4))


def sign_normalise(U, V=None):
    """Reading: each u_i is flipped so that its largest-magnitude entry is
    positive (lowest index on ties); v_i gets the same flip."""
    U = np.array(U, dtype=np.float64, order="F", copy=True)
    V = None if V is None else np.array(V, dtype=np.float64, order="F", copy=True)
    for i in range(U.shape[1]):
        j = int(np.argmax(np.abs(U[:, i])))
        if U[j, i] < 0:
            U[:, i] = -U[:, i]
            if V is not None:
                V[:, i] = -V[:, i]
    return U, V


def mode_sines(Uold, Unew):
    """The "mode" convergence criterion of Alg. 1 (xi_i = u~_i^T u^_i): the sine
    of the angle between u_old,i and u_new,i for each mode i, measured sign
    free as |u_new,i - u_old,i (u_old,i^T u_new,i)| (both unit vectors).
    Reading: sines rather than the paper's cosines, which cannot resolve
    angles below ~1e-8 in FP64."""
    out = np.zeros(Uold.shape[1])
    for i in range(Uold.shape[1]):
        a, b = Uold[:, i], Unew[:, i]
        d = b - a * float(a @ b)
        out[i] = float(np.sqrt(d @ d))
    return out


def center_rows(A):
    """Row centring of the snapshot matrix (Sec. 1: the POD is taken of the
    mean-subtracted snapshots).  mean_i = (sum_j a_ij) / n, summed in FP64 in
    column order; returns (A - mean 1^T rounded to A's dtype, mean)."""
    A = np.asarray(A)
    X = np.asarray(A, dtype=np.float64)
    m, n = X.shape
    mean = np.zeros(m)
    for j in range(n):
        mean += X[:, j]
    mean /= float(n)
    out = np.asfortranarray((X - mean[:, None]).astype(A.dtype))
    return out, mean


def ls_row_weights(U_state, k: int):
    """Leverage-score row weights of GET UPDATE (Alg. 1, rows branch, second
    iteration on): q_i proportional to |u^i|^2, the squared norm of row i of
    the current first k modes U~_k (the paper's q_i = |u^i|^2 / k, whose
    normalisation the integer weights absorb).  Columns beyond the k-th of the
    state do not enter."""
    kk = min(int(k), U_state.shape[1])
    return row_sqnorms(np.asfortranarray(U_state[:, :kk]))


def ort_col_weights(X, U_state, inS, rel_floor: float = ORT_FLOOR_F64):
    """ORT column weights of Alg. 1 (Sec. "Column sampling" (c)):
    p_i proportional to |a_i - U~ U~^T a_i|^2 over the unsampled set S, with U~
    the whole current state (r' columns), the residual formed explicitly in
    FP64.  Columns outside S get 0.  Readings: a residual at or below
    rel_floor |a_i|^2 is zero (the column lies in the current subspace to
    working accuracy; without this floor rounding noise would decide the
    draw), and the weights are quantised after this masking (their maximum is
    taken over S)."""
    X = np.asarray(X, dtype=np.float64)
    U = np.asarray(U_state, dtype=np.float64)
    rho = np.zeros(X.shape[1])
    for i in np.flatnonzero(inS):
        a = X[:, i]
        res = a - U @ (U.T @ a)
        v = float(res @ res)
        rho[i] = v if v > rel_floor * float(a @ a) else 0.0
    return rho


def sample_and_scale_unique_rows(D, wr, w, seed, it, block=0, forced=None):
    """SAMPLE AND SCALE UNIQUE ROWS of Alg. 1: draw w row indices with
    Pr[i] = q_i = wr_i / sum(wr) (Philox stream 1), keep the distinct rows
    I_r with their multiplicities t_hat, and scale row i by
    sqrt(t_hat_i / (w q_i)).  Returns (I_r, t_hat, W)."""
    Omega = float(int(np.asarray(wr, dtype=np.uint64).astype(object).sum()))
    if forced is not None:
        rows, rcnt = forced
    else:
        if Omega == 0.0:
            raise ValueError("row weights are all zero")
        rdraws, _ = draw(wr, w, seed, 1, it, block)
        rows, rcnt = unique(rdraws)
    q = np.asarray(wr)[rows].astype(np.float64) / Omega
    scale = np.sqrt(rcnt.astype(np.float64) / (float(w) * q))
    W = np.asarray(D)[rows, :] * scale[:, None]
    return rows, rcnt, W


def get_update(X, prm: IsmaParams, it: int, inS: np.ndarray, wq: np.ndarray, U_state,
               replay: Optional[IterLog] = None):
    """GET UPDATE of Alg. 1.  Returns (C, IterLog) or (None, None) when no
    column of S can be drawn (S empty, or every weight in S is zero).

    Column weights: L2N every iteration; UNF uniform over S from the second
    iteration; ORT the squared residuals of the columns of S against the
    current state from the second iteration (Table of sampling strategies,
    Sec. "Column sampling").  Rows (w > 0): L2 norms of the
    rows of D, or, from the second iteration, leverage scores |u^i|^2 of the
    current U_k (LS)."""
    n = X.shape[1]
    r = prm.rank
    if replay is not None:
        cols, ccnt = np.asarray(replay.cols, np.int64), np.asarray(replay.col_counts, np.int32)
    else:
        if prm.col_strategy == "unf" and it > 0:
            wcol = inS.astype(np.uint64)
        elif prm.col_strategy == "ort" and it > 0 and U_state.shape[1] > 0:
            wcol = quantize(ort_col_weights(X, U_state, inS))
        else:
            wcol = np.where(inS, wq, np.uint64(0)).astype(np.uint64)
        if int(wcol.astype(object).sum()) == 0:
            return None, None
        draws_, _ = draw(wcol, prm.c, prm.seed, 0, it, prm.block)
        cols, ccnt = unique(draws_)
    inS[cols] = False
    D = np.asfortranarray(X[:, cols])
    g = D.shape[1]
    log = IterLog(cols=cols, col_counts=ccnt)
    if prm.w > 0:
        if prm.row_strategy == "ls" and it > 0:
            rho = ls_row_weights(U_state, prm.k)
        else:
            rho = row_sqnorms(D)
        wr = quantize(rho)
        forced = None
        if replay is not None and replay.rows is not None:
            forced = (np.asarray(replay.rows, np.int64), np.asarray(replay.row_counts, np.int32))
        rows, rcnt, W = sample_and_scale_unique_rows(D, wr, prm.w, prm.seed, it, prm.block, forced)
        Omega = float(int(np.asarray(wr, dtype=np.uint64).astype(object).sum()))
        log.row_scales = np.sqrt(rcnt.astype(np.float64) / (float(prm.w) * (wr[rows].astype(np.float64) / Omega)))
        G = W.T @ W
        ev, Vt = jacobi_eig(G)
        h = rows.shape[0]
        # Reading: only directions with a non-zero singular value of W are
        # kept (the paper divides by sigma~_i); r_u = min(r, g, rank(W)).
        nz = int(np.sum(ev > g * U_F64 * max(ev[0], 0.0))) if g else 0
        r_u = min(r, g, h, nz)
        C = np.asfortranarray(D @ Vt[:, :r_u])
        log.rows, log.row_counts, log.r_u = rows, rcnt, r_u
    elif prm.r_update > 0:
        G = D.T @ D
        ev, Vt = jacobi_eig(G)
        nz = int(np.sum(ev > g * U_F64 * max(ev[0], 0.0))) if g else 0
        r_u = min(prm.r_update, g, nz)
        C = np.asfortranarray(D @ Vt[:, :r_u])
        log.r_u = r_u
    else:
        C = D
        log.r_u = g
    return C, log


def isma(A, prm: IsmaParams, elem_bytes: Optional[int] = None, n_iter: Optional[int] = None,
         replay: Optional[List[IterLog]] = None, final_step: bool = True, want_v: bool = True) -> IsmaResult:
    """Alg. 1.  A is m x n (any float dtype; computed in FP64).

    ``elem_bytes`` is the storage width of A on the device (sets the norm
    summation order); defaults to A's dtype.  ``n_iter`` forces the number of
    merges (parity replay of the iteration count); ``replay`` forces the
    sampled indices of each iteration (for strategies whose indices depend
    on computed modes)."""
    if elem_bytes is None:
        elem_bytes = np.asarray(A).dtype.itemsize
    X = np.asfortranarray(np.asarray(A, dtype=np.float64))
    m, n = X.shape
    k, r = prm.k, prm.rank
    if not (1 <= k <= r):
        raise ValueError("need 1 <= k <= r")
    nu = col_sqnorms(X, elem_bytes)
    wq = quantize(nu)
    inS = np.ones(n, dtype=bool)
    U = np.zeros((m, 0), order="F")
    s = np.zeros(0)
    logs: List[IterLog] = []
    converged = exhausted = False
    it = 0
    sin_tol = math.sin(min(prm.theta_tol, math.pi / 2))
    while True:
        if n_iter is not None and it >= n_iter:
            break
        rp = replay[it] if replay is not None and it < len(replay) else None
        C, log = get_update(X, prm, it, inS, wq, U, rp)
        if C is None:
            exhausted = True
            break
        Unew, snew = merge(U, s, C, r)
        if it > 0 and U.shape[1] > 0 and Unew.shape[1] > 0:
            kk = min(k, U.shape[1], Unew.shape[1])
            if prm.criterion == "mode":
                log.sin_theta = float(np.max(mode_sines(U[:, :kk], Unew[:, :kk])))
            else:
                log.sin_theta = float(np.max(subspace_sines(U[:, :kk], Unew[:, :kk])))
        log.rank = Unew.shape[1]
        log.sigma = snew.copy()
        logs.append(log)
        U, s = Unew, snew
        it += 1
        if n_iter is not None:
            continue
        if it > 1 and log.sin_theta < sin_tol:
            converged = True
            break
        if it >= prm.max_iter:
            break
        if not inS.any():
            exhausted = True
            break
    if final_step and U.shape[1] > 0:
        Uf, sf, Vf = project(X, U, want_v=want_v)
        kk = min(k, Uf.shape[1])
        Uk, Vk = sign_normalise(Uf[:, :kk], None if Vf is None else Vf[:, :kk])
        return IsmaResult(Uk, sf[:kk].copy(), Vk, U, s, logs, converged, exhausted)
    kk = min(k, U.shape[1])
    Uk, _ = sign_normalise(U[:, :kk])
    return IsmaResult(Uk, s[:kk].copy(), None, U, s, logs, converged, exhausted)


def block_bounds(n: int, t: Optional[int] = None, width: Optional[int] = None):
    """Column blocks of Alg. 3.  Reading: 0-based half-open blocks
    [floor(i n / t), floor((i+1) n / t)) for t blocks, or consecutive blocks of
    ``width`` columns with a shorter last block."""
    if width is not None:
        return [(j, min(j + width, n)) for j in range(0, n, width)]
    return [((i * n) // t, ((i + 1) * n) // t) for i in range(t)]


def incremental(A, prm: IsmaParams, blocks, elem_bytes: Optional[int] = None, block_final_step: bool = True):
    """Alg. 3: ISMA on each column block, then BLOCK MERGE into the running
    (U, Sigma).  Block b uses Philox counter word 2 = b.  Reading: each
    block's ISMA ends with its own final step (Alg. 1) and hands its r
    leading pairs to the merge.  Returns (U_k, sigma_k, U_r, s_r)."""
    U = s = None
    r = prm.rank
    for b, (j0, j1) in enumerate(blocks):
        res = isma(np.asarray(A)[:, j0:j1], replace(prm, block=b, k=min(prm.k, r)), elem_bytes=elem_bytes,
                   final_step=False)
        Ub, sb = res.U_merge, res.s_merge
        if block_final_step:
            Ub, sb, _ = project(np.asarray(A)[:, j0:j1], Ub, want_v=False)
        if U is None:
            U, s = Ub[:, :r], sb[:r]
        else:
            U, s = merge(U, s, Ub[:, :r] * sb[None, :r], r)
    kk = min(prm.k, U.shape[1])
    Uk, _ = sign_normalise(U[:, :kk])
    return Uk, s[:kk].copy(), U, s

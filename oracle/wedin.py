"""Quality measure of converged POD modes (TEST INFRASTRUCTURE ONLY).

Sec. "Quality of converged solution", Eq. (ang_meas): with the top k
singular triplets (U_k, Sigma_k, V_k) of the final estimate,

    R = A V_k - U_k Sigma_k,    S = A^T U_k - V_k Sigma_k,

Wedin's theorem bounds the sines of the principal angles between the exact
and the estimated dominant left and right subspaces:

    sqrt(||sin Theta||_F^2 + ||sin Phi||_F^2) <= sqrt(||R||_F^2 + ||S||_F^2) / omega,

omega = min(min_j |sigma~_k - sigma_{k+j}|, sigma~_k).  The exact singular
values being unknown, the paper estimates omega from the (k+1)-th estimated
value: omega^ = min(|sigma~_k - sigma~_{k+1}|, sigma~_k), which needs r > k.
Plain FP64, the definition written out.
"""
from __future__ import annotations

import math

import numpy as np


def wedin_measure(A, Uk, sk, Vk, s_next):
    """Returns (||R||_F, ||S||_F, omega^, bound) of Eq. (ang_meas) with the
    paper's estimate omega^ = min(|s_k - s_{k+1}|, s_k).  A is m x n, Uk m x k,
    Vk n x k, sk the k estimated singular values, s_next the (k+1)-th."""
    X = np.asarray(A, dtype=np.float64)
    U = np.asarray(Uk, dtype=np.float64)
    V = np.asarray(Vk, dtype=np.float64)
    s = np.asarray(sk, dtype=np.float64)
    R = X @ V - U * s[None, :]
    S = X.T @ U - V * s[None, :]
    rn = float(np.sqrt(np.sum(R * R)))
    sn = float(np.sqrt(np.sum(S * S)))
    omega = min(abs(float(s[-1]) - float(s_next)), float(s[-1]))
    bound = math.sqrt(rn * rn + sn * sn) / omega if omega > 0.0 else math.inf
    return rn, sn, omega, bound

"""FP64 CPU oracle for the iterative sample-and-merge POD (ISMA).

TEST INFRASTRUCTURE ONLY.  The oracle is the parity reference for the HIP
library in ``paper_1905_05107_amd``.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.
It shares no code with the GPU path and never calls it; the product path
never calls the oracle.

The numerical primitives live in ``pod_oracle.c`` (plain C, FP64, no
BLAS/LAPACK; OpenMP splits only loops over independent columns, so every
result is bitwise the same for any thread count); ``isma.py`` strings them together in the order of
the paper's Alg. 1 (ISMA, with the UNF / L2N / ORT column and L2 / LS row
strategies and the optional row centring), Alg. 2 (BLOCK MERGE) and Alg. 3
(incremental POD); ``oneshot.py`` follows Alg. 4 (LTSVD) and Alg. 5 (CTSVD) of
Appendix A; ``adjoint.py`` the reverse pass of the merge chain; ``wedin.py``
the quality measure of Eq. (ang_meas).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pod_oracle.c")
_LIB = os.path.join(_HERE, "_pod_oracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile pod_oracle.c into _pod_oracle.so with gcc (FP contraction off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-Wall", "-shared", "-fPIC",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i64, i32, u64 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
        pd, pu64, pi64, pi32 = P(d), P(u64), P(i64), P(i32)
        sig = {
            "or_philox4x64_10": (None, [pu64, pu64, pu64]),
            "or_col_sqnorms": (None, [pd, i64, i64, i64, ctypes.c_int, pd]),
            "or_row_sqnorms": (None, [pd, i64, i64, pd]),
            "or_quantize": (ctypes.c_int, [pd, i64, pu64]),
            "or_draw": (u64, [pu64, i64, i32, u64, u64, u64, u64, pi64]),
            "or_unique": (i32, [pi64, i32, pi64, pi32]),
            "or_householder_qr": (None, [pd, i64, i64, pd, pd]),
            "or_jacobi_svd": (ctypes.c_int, [pd, i64, i64, pd, pd, pd, ctypes.c_int]),
            "or_jacobi_eig": (ctypes.c_int, [pd, i64, pd, pd, ctypes.c_int]),
            "or_merge": (i32, [pd, pd, i64, i32, pd, i32, i32, pd, pd]),
            "or_subspace_sines": (ctypes.c_int, [pd, pd, i64, i32, pd]),
            "or_project": (ctypes.c_int, [pd, i64, i64, i64, pd, i32, pd, pd, pd]),
            "or_set_threads": (None, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _f64(a):
    """Column-major FP64 copy (values of FP32 inputs are represented exactly)."""
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def set_threads(n: int) -> None:
    """Threads of the C oracle's column-parallel loops (results do not depend
    on it: only independent columns are split between threads)."""
    lib().or_set_threads(int(n))


# ---------------------------------------------------------------- primitives

def philox4x64_10(counter, key):
    """One Philox-4x64-10 block: 4 counter words, 2 key words -> 4 words."""
    c = np.asarray(counter, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_10(_p(c, ctypes.c_uint64), _p(k, ctypes.c_uint64), _p(out, ctypes.c_uint64))
    return out


def col_sqnorms(A, elem_bytes=None):
    """|a_j|^2 in the fixed summation order (see pod_oracle.c).

    ``elem_bytes`` is the storage width of A (4 for FP32, 8 for FP64); it sets
    the vector width of the summation order.  Defaults to A's own dtype."""
    if elem_bytes is None:
        elem_bytes = np.asarray(A).dtype.itemsize
    X = _f64(A)
    m, n = X.shape
    nu = np.zeros(n)
    lib().or_col_sqnorms(_p(X, ctypes.c_double), m, n, m, int(elem_bytes), _p(nu, ctypes.c_double))
    return nu


def row_sqnorms(D):
    X = _f64(D)
    m, g = X.shape
    rho = np.zeros(m)
    lib().or_row_sqnorms(_p(X, ctypes.c_double), m, g, _p(rho, ctypes.c_double))
    return rho


def quantize(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    w = np.zeros(v.shape[0], dtype=np.uint64)
    rc = lib().or_quantize(_p(v, ctypes.c_double), v.shape[0], _p(w, ctypes.c_uint64))
    if rc != 0:
        raise ValueError("sampling weights are not finite and non-negative")
    return w


def draw(w, cnt, seed, stream, it, block=0):
    """cnt draws with replacement; returns (indices int64[cnt], W)."""
    w = np.ascontiguousarray(w, dtype=np.uint64)
    out = np.zeros(max(cnt, 1), dtype=np.int64)
    W = lib().or_draw(_p(w, ctypes.c_uint64), w.shape[0], int(cnt), int(seed) & (2**64 - 1),
                      int(stream), int(it), int(block), _p(out, ctypes.c_int64))
    return out[:cnt], int(W)


def unique(draws):
    d = np.ascontiguousarray(draws, dtype=np.int64)
    n = d.shape[0]
    u = np.zeros(max(n, 1), dtype=np.int64)
    c = np.zeros(max(n, 1), dtype=np.int32)
    g = lib().or_unique(_p(d, ctypes.c_int64), n, _p(u, ctypes.c_int64), _p(c, ctypes.c_int32))
    return u[:g].copy(), c[:g].copy()


def householder_qr(X):
    X = _f64(X)
    m, p = X.shape
    R = np.zeros((p, p), order="F")
    Q = np.zeros((m, p), order="F")
    lib().or_householder_qr(_p(X, ctypes.c_double), m, p, _p(R, ctypes.c_double), _p(Q, ctypes.c_double))
    return Q, R


def jacobi_svd(X, want_v=True, max_sweeps=100):
    """One-sided Jacobi SVD: returns (U, sigma, V) with X V = U diag(sigma)."""
    X = _f64(X)
    rows, cols = X.shape
    s = np.zeros(cols)
    U = np.zeros((rows, cols), order="F")
    V = np.zeros((cols, cols), order="F") if want_v else None
    sw = lib().or_jacobi_svd(_p(X, ctypes.c_double), rows, cols, _p(s, ctypes.c_double),
                             _p(U, ctypes.c_double),
                             _p(V, ctypes.c_double) if want_v else None, max_sweeps)
    if sw < 0:
        raise RuntimeError("one-sided Jacobi SVD did not converge")
    return U, s, V


def jacobi_eig(G, max_sweeps=100):
    G = _f64(G)
    n = G.shape[0]
    ev = np.zeros(n)
    V = np.zeros((n, n), order="F")
    sw = lib().or_jacobi_eig(_p(G, ctypes.c_double), n, _p(ev, ctypes.c_double), _p(V, ctypes.c_double),
                             max_sweeps)
    if sw < 0:
        raise RuntimeError("Jacobi eigensolver did not converge")
    return ev, V


def merge(U1, s1, C, r):
    """Alg. 2 BLOCK MERGE of (U1, s1) with the block C = U2 S2; truncate to r."""
    C = _f64(C)
    m, g = C.shape
    if U1 is None or np.asarray(U1).shape[1] == 0:
        U1 = np.zeros((m, 0), order="F")
        s1 = np.zeros(0)
    U1 = _f64(U1)
    s1 = np.ascontiguousarray(s1, dtype=np.float64)
    r1 = U1.shape[1]
    Uo = np.zeros((m, max(r, 1)), order="F")
    so = np.zeros(max(r, 1))
    rr = lib().or_merge(_p(U1, ctypes.c_double) if r1 else None, _p(s1, ctypes.c_double) if r1 else None,
                        m, r1, _p(C, ctypes.c_double), g, int(r), _p(Uo, ctypes.c_double),
                        _p(so, ctypes.c_double))
    if rr < 0:
        raise RuntimeError("merge: Jacobi SVD did not converge")
    return np.asfortranarray(Uo[:, :rr]), so[:rr].copy()


def subspace_sines(Ua, Ub):
    Ua, Ub = _f64(Ua), _f64(Ub)
    m, k = Ua.shape
    s = np.zeros(k)
    if lib().or_subspace_sines(_p(Ua, ctypes.c_double), _p(Ub, ctypes.c_double), m, k,
                               _p(s, ctypes.c_double)) != 0:
        raise RuntimeError("subspace sines: Jacobi SVD did not converge")
    return s


def project(A, U, want_v=True):
    """Final step of Alg. 1 (QR of A^T U, SVD of R, rotation): (U, sigma, V)."""
    A = _f64(A)
    U = _f64(U)
    m, n = A.shape
    r = U.shape[1]
    Uo = np.zeros((m, r), order="F")
    s = np.zeros(r)
    V = np.zeros((n, r), order="F") if want_v else None
    rc = lib().or_project(_p(A, ctypes.c_double), m, n, m, _p(U, ctypes.c_double), r,
                          _p(Uo, ctypes.c_double), _p(s, ctypes.c_double),
                          _p(V, ctypes.c_double) if want_v else None)
    if rc != 0:
        raise RuntimeError("project: Jacobi SVD did not converge")
    return Uo, s, V

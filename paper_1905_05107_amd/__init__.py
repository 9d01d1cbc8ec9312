"""MI355X (gfx950) iterative sample-and-merge POD (ISMA, arXiv 1905.05107).

Thin ctypes binding of ``libpod.so`` (declared in ``include/pod.h``): argument
marshalling only.  Every step of the method runs in the library's HIP kernels;
PyTorch supplies device memory and the stream.  There is no CPU fallback: if
the library is not built this module raises on first use.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpod.so")

POD_OK, POD_EINVAL, POD_ENOMEM, POD_EHIP, POD_ENOTPD, POD_ESTATE, POD_EXHAUSTED, POD_ENONFINITE, POD_ENOCONV = range(9)
POD_F64, POD_F32, POD_BF16_REFINE = 0, 1, 2
POD_COL_L2N, POD_COL_UNF, POD_COL_ORT = 0, 1, 2
POD_ROW_L2, POD_ROW_LS = 0, 1
POD_CRIT_SUBSPACE, POD_CRIT_MODE = 0, 1
POD_STOP_NONE, POD_STOP_NONFINITE, POD_STOP_CONVERGED, POD_STOP_EXHAUSTED, POD_STOP_MAX_ITER, POD_STOP_BREAKDOWN = \
    range(6)
STOP_NAMES = {POD_STOP_NONE: "running", POD_STOP_NONFINITE: "nonfinite", POD_STOP_CONVERGED: "converged",
              POD_STOP_EXHAUSTED: "exhausted", POD_STOP_MAX_ITER: "max_iter", POD_STOP_BREAKDOWN: "breakdown"}

# every symbol include/pod.h declares
EXPORTS = ["pod_init", "pod_sample", "pod_merge", "pod_converged", "pod_project", "pod_wedin_bound", "pod_get_basis", "pod_get_info",
           "pod_get_indices", "pod_get_col_sqnorms", "pod_col_sqnorms", "pod_sample_size", "pod_destroy",
           "pod_status_str", "pod_profile_enable", "pod_profile_read", "pod_inc_init", "pod_inc_add_block",
           "pod_inc_add_host_blocks", "pod_inc_result", "pod_inc_get_info", "pod_inc_destroy", "pod_batch_init",
           "pod_batch_autotune", "pod_batch_run", "pod_batch_project", "pod_batch_get_info", "pod_batch_destroy",
           "pod_enable_adjoint", "pod_backward", "pod_loss_grad", "pod_batch_enable_adjoint", "pod_batch_loss_grad", "pod_batch_loss_grad_all",
           "pod_run", "pod_set_indices", "pod_center_rows", "pod_center_rows_noalloc",
           "pod_oneshot"]


class PodError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_str(status)} (status {status})")
        self.status = status


class pod_params(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
        ("a_dtype", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("k", ctypes.c_int32), ("r", ctypes.c_int32), ("c", ctypes.c_int32), ("w", ctypes.c_int32),
        ("r_update", ctypes.c_int32), ("col_strategy", ctypes.c_int32), ("row_strategy", ctypes.c_int32),
        ("criterion", ctypes.c_int32), ("center_rows", ctypes.c_int32), ("max_iter", ctypes.c_int32),
        ("theta_tol", ctypes.c_double), ("seed", ctypes.c_uint64), ("block", ctypes.c_uint64),
    ]


class pod_info(ctypes.Structure):
    _fields_ = [
        ("iter", ctypes.c_int32), ("rank", ctypes.c_int32), ("g", ctypes.c_int32), ("h", ctypes.c_int32),
        ("exhausted", ctypes.c_int32), ("flags", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
        ("total_sweeps", ctypes.c_int32), ("sin_theta", ctypes.c_double),
        ("stop_reason", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class pod_inc_info(ctypes.Structure):
    _fields_ = [
        ("blocks", ctypes.c_int32), ("columns", ctypes.c_int64), ("host_bytes", ctypes.c_double),
        ("copy_ms", ctypes.c_double), ("wall_ms", ctypes.c_double),
    ]


_lib = None


def lib():
    """Load libpod.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1905_05107_amd.build` first")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER
        sig = {
            "pod_init": (i32, [P(vp), P(pod_params), vp, vp]),
            "pod_sample": (i32, [vp, P(i32), P(i32)]),
            "pod_merge": (i32, [vp]),
            "pod_converged": (i32, [vp, P(i32), P(d)]),
            "pod_run": (i32, [vp, i32, i32, i32, P(d), P(i32), P(i32)]),
            "pod_project": (i32, [vp, vp, vp, vp]),
            "pod_wedin_bound": (i32, [vp, vp, vp, P(d)]),
            "pod_get_basis": (i32, [vp, vp, vp, P(i32)]),
            "pod_get_info": (i32, [vp, P(pod_info)]),
            "pod_get_indices": (i32, [vp, i32, P(i32), P(i32), P(i32), P(i32), P(i32), P(i32)]),
            "pod_set_indices": (i32, [vp, i32, P(i32), P(i32), i32, P(i32), P(i32), i32]),
            "pod_get_col_sqnorms": (i32, [vp, vp]),
            "pod_col_sqnorms": (i32, [vp, i32, i64, i64, i64, vp, vp]),
            "pod_center_rows": (i32, [vp, i32, i64, i64, i64, vp]),
            "pod_oneshot": (i32, [P(pod_params), vp, d, vp, vp, P(i32), vp]),
            "pod_center_rows_noalloc": (i32, [vp, i32, i64, i64, i64, vp]),
            "pod_sample_size": (i64, [i32, i32, d, d]),
            "pod_destroy": (None, [vp]),
            "pod_status_str": (ctypes.c_char_p, [i32]),
            "pod_profile_enable": (i32, [i32]),
            "pod_profile_read": (i32, [P(i64), P(d)]),
            "pod_inc_init": (i32, [P(vp), P(pod_params), vp]),
            "pod_inc_add_block": (i32, [vp, vp, i64, i64]),
            "pod_inc_add_host_blocks": (i32, [vp, P(vp), P(i64), i32]),
            "pod_inc_result": (i32, [vp, vp, vp, P(i32)]),
            "pod_inc_get_info": (i32, [vp, P(pod_inc_info)]),
            "pod_inc_destroy": (None, [vp]),
            "pod_batch_init": (i32, [P(vp), i32, P(pod_params), P(vp)]),
            "pod_batch_autotune": (i32, [vp, P(i32)]),
            "pod_batch_run": (i32, [vp, i32, i32, P(i32)]),
            "pod_batch_project": (i32, [vp, i32, vp, vp, vp]),
            "pod_batch_get_info": (i32, [vp, i32, P(pod_info), P(i32)]),
            "pod_batch_destroy": (None, [vp]),
            "pod_enable_adjoint": (i32, [vp]),
            "pod_backward": (i32, [vp, vp, vp, vp]),
            "pod_loss_grad": (i32, [vp, vp, P(d)]),
            "pod_batch_enable_adjoint": (i32, [vp]),
            "pod_batch_loss_grad": (i32, [vp, i32, vp, P(d)]),
            "pod_batch_loss_grad_all": (i32, [vp, P(vp), P(d)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_str(s: int) -> str:
    return lib().pod_status_str(int(s)).decode()


def _check(s: int, what: str, ok=(POD_OK,)):
    if s not in ok:
        raise PodError(s, what)
    return s


def sample_size(kind: str, k: int, eps: float, delta: float) -> int:
    """Eq. (c_LTSVD) for kind 'ltsvd', Eq. (c_w_CTSVD) for 'ctsvd'."""
    return int(lib().pod_sample_size(0 if kind == "ltsvd" else 1, int(k), float(eps), float(delta)))


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _a_layout(A):
    """(ptr, m, n, lda, dtype code) of a column-major device matrix.

    Accepts an m x n tensor whose columns are contiguous (A.stride(0) == 1),
    e.g. the transpose of an (n, m) contiguous tensor."""
    import torch
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    if A.dim() != 2 or (A.shape[0] > 1 and A.stride(0) != 1):
        raise ValueError("A must be m x n with contiguous columns (stride(0) == 1)")
    if A.dtype == torch.float64:
        code = POD_F64
    elif A.dtype == torch.float32:
        code = POD_F32
    else:
        raise ValueError("A must be float32 or float64")
    m, n = A.shape
    lda = A.stride(1) if n > 1 else m
    return A.data_ptr(), m, n, max(lda, m), code


@dataclass
class Result:
    U: "object"            # m x k device tensor
    sigma: "object"        # k (float64 device tensor)
    V: Optional["object"]  # n x k device tensor
    iters: int
    sin_theta: List[float]
    exhausted: bool
    converged: bool
    flags: int
    stopped_by: str = "running"


class PodContext:
    """One ISMA run on one device matrix (pod_init ... pod_destroy)."""

    def __init__(self, A, k: int, c: int, r: int = 0, w: int = 0, precision: int = POD_F64,
                 theta_tol: float = 1e-10, col_strategy: int = POD_COL_L2N, row_strategy: int = POD_ROW_L2,
                 criterion: int = POD_CRIT_SUBSPACE, max_iter: Optional[int] = None, seed: int = 0,
                 block: int = 0, r_update: int = 0, center_rows: bool = False, stream=None):
        ptr, m, n, lda, code = _a_layout(A)
        self.A = A
        self.m, self.n = m, n
        self.k = k
        self.precision = precision
        p = pod_params()
        p.m, p.n, p.lda, p.a_dtype, p.precision = m, n, lda, code, precision
        p.k, p.r, p.c, p.w, p.r_update = k, r, c, w, r_update
        p.col_strategy, p.row_strategy, p.criterion = col_strategy, row_strategy, criterion
        p.center_rows = 1 if center_rows else 0
        p.max_iter = int(max_iter if max_iter is not None else n + 1)
        p.theta_tol = float(theta_tol)
        p.seed = int(seed) & (2**64 - 1)
        p.block = int(block)
        self.params = p
        self.stream = _stream_handle(stream)
        h = ctypes.c_void_p()
        _check(lib().pod_init(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p(ptr), self.stream), "pod_init")
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().pod_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- steps
    def sample(self, want_counts: bool = False):
        """GET UPDATE; returns True if a draw was made (False: S exhausted)."""
        if want_counts:
            g, h = ctypes.c_int32(), ctypes.c_int32()
            s = lib().pod_sample(self.h, ctypes.byref(g), ctypes.byref(h))
            _check(s, "pod_sample", ok=(POD_OK, POD_EXHAUSTED))
            return (s == POD_OK, g.value, h.value)
        s = lib().pod_sample(self.h, None, None)
        _check(s, "pod_sample", ok=(POD_OK, POD_EXHAUSTED))
        return s == POD_OK

    def merge(self):
        _check(lib().pod_merge(self.h), "pod_merge")

    def converged(self):
        done, sn = ctypes.c_int32(), ctypes.c_double()
        _check(lib().pod_converged(self.h, ctypes.byref(done), ctypes.byref(sn)), "pod_converged")
        return bool(done.value), sn.value

    def info(self) -> pod_info:
        inf = pod_info()
        _check(lib().pod_get_info(self.h, ctypes.byref(inf)), "pod_get_info")
        return inf

    def _out_dtype(self):
        import torch
        return torch.float64 if self.precision == POD_F64 else torch.float32

    def project(self, want_v: bool = True):
        import torch
        inf = self.info()
        k = min(self.k, inf.rank)
        dev = self.A.device
        Ut = torch.empty((k, self.m), dtype=self._out_dtype(), device=dev)
        sig = torch.empty(k, dtype=torch.float64, device=dev)
        Vt = torch.empty((k, self.n), dtype=self._out_dtype(), device=dev) if want_v else None
        _check(lib().pod_project(self.h, ctypes.c_void_p(Ut.data_ptr()), ctypes.c_void_p(sig.data_ptr()),
                                 ctypes.c_void_p(Vt.data_ptr()) if want_v else None), "pod_project")
        self._proj_k = k
        return Ut.T, sig, (Vt.T if want_v else None)

    def wedin_bound(self, U, V):
        """Quality measure of Eq. (ang_meas) for the pairs the last project()
        returned: (||R||_F, ||S||_F, omega^, bound).  Needs r > k."""
        k = getattr(self, "_proj_k", None)
        if k is None:
            raise ValueError("wedin_bound needs the pairs of a project() call")
        check_pairs(U, V, self.m, self.n, k, self._out_dtype(), self.A.device)
        Ut, Vt = U.T, V.T
        out = (ctypes.c_double * 4)()
        _check(lib().pod_wedin_bound(self.h, ctypes.c_void_p(Ut.data_ptr()), ctypes.c_void_p(Vt.data_ptr()), out),
               "pod_wedin_bound")
        return tuple(out)

    def basis(self):
        import torch
        inf = self.info()
        rk = inf.rank
        dev = self.A.device
        Ut = torch.empty((max(rk, 1), self.m), dtype=self._out_dtype(), device=dev)
        sig = torch.empty(max(rk, 1), dtype=torch.float64, device=dev)
        r = ctypes.c_int32()
        _check(lib().pod_get_basis(self.h, ctypes.c_void_p(Ut.data_ptr()), ctypes.c_void_p(sig.data_ptr()),
                                   ctypes.byref(r)), "pod_get_basis")
        return Ut[:r.value].T, sig[:r.value]

    def indices(self, it: int, rows: bool = False):
        """Distinct columns and their multiplicities drawn at merge `it`;
        with rows=True also the distinct rows and their multiplicities."""
        import numpy as np
        c, w = self.params.c, self.params.w
        cols = np.zeros(max(c, 1), dtype=np.int32)
        cnt = np.zeros(max(c, 1), dtype=np.int32)
        rws = np.zeros(max(w, 1), dtype=np.int32)
        rcnt = np.zeros(max(w, 1), dtype=np.int32)
        g, h = ctypes.c_int32(), ctypes.c_int32()
        P = ctypes.POINTER(ctypes.c_int32)
        _check(lib().pod_get_indices(self.h, int(it), cols.ctypes.data_as(P), cnt.ctypes.data_as(P),
                                     ctypes.byref(g), rws.ctypes.data_as(P), rcnt.ctypes.data_as(P),
                                     ctypes.byref(h)), "pod_get_indices")
        if rows:
            return cols[:g.value].copy(), cnt[:g.value].copy(), rws[:h.value].copy(), rcnt[:h.value].copy()
        return cols[:g.value].copy(), cnt[:g.value].copy()

    def set_indices(self, it: int, cols, col_counts=None, rows=None, row_counts=None):
        """Replay: the next draw (that of merge `it`) takes these distinct
        columns (ascending; multiplicities optional) and, with row sampling,
        these distinct rows and multiplicities instead of drawing."""
        import numpy as np
        P = ctypes.POINTER(ctypes.c_int32)
        c = np.ascontiguousarray(cols, dtype=np.int32)
        cc = None if col_counts is None else np.ascontiguousarray(col_counts, dtype=np.int32)
        rw = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
        rc = None if row_counts is None else np.ascontiguousarray(row_counts, dtype=np.int32)
        if cc is not None and cc.shape != c.shape or (rw is None) != (rc is None) or \
                (rw is not None and rw.shape != rc.shape):
            raise ValueError("indices and their counts must have the same length")
        _check(lib().pod_set_indices(self.h, int(it), c.ctypes.data_as(P),
                                     cc.ctypes.data_as(P) if cc is not None else None, int(c.shape[0]),
                                     rw.ctypes.data_as(P) if rw is not None else None,
                                     rc.ctypes.data_as(P) if rc is not None else None,
                                     int(rw.shape[0]) if rw is not None else 0), "pod_set_indices")

    def replay(self, draws):
        """Merges with given draws: ``draws`` is a list of (cols, col_counts)
        or (cols, col_counts, rows, row_counts) per iteration, e.g. from a
        reference run.  Returns the convergence sines (NaN for the first)."""
        sines = []
        for d in draws:
            self.set_indices(self.info().iter, *d)
            if not self.sample():
                break
            self.merge()
            _, sn = self.converged()
            sines.append(sn)
        return sines

    # -- reverse mode
    def enable_adjoint(self):
        """Keep the per-merge checkpoints of the reverse pass (call first)."""
        _check(lib().pod_enable_adjoint(self.h), "pod_enable_adjoint")

    def _dA(self):
        import torch
        dt = torch.float64 if self.precision == POD_F64 else torch.float32
        return torch.zeros((self.n, self.m), dtype=dt, device=self.A.device)

    def loss_grad(self):
        """(L, dL/dA) for L = |A - U_k U_k^T A|_F^2 of the merged modes."""
        dAt = self._dA()
        L = ctypes.c_double()
        _check(lib().pod_loss_grad(self.h, ctypes.c_void_p(dAt.data_ptr()), ctypes.byref(L)), "pod_loss_grad")
        return L.value, dAt.T

    def backward(self, dU=None, dsigma=None, dA=None):
        """dA += adjoint of (U_k, Sigma_k) for the output adjoints dU, dsigma."""
        import torch
        dAt = self._dA() if dA is None else dA.T
        if dA is not None and not dAt.is_contiguous():
            raise ValueError("dA must have contiguous columns (ld = m)")
        dUt = None
        if dU is not None:
            dt = torch.float64 if self.precision == POD_F64 else torch.float32
            dUt = dU.T.to(dt).contiguous()
        ds = dsigma.to(torch.float64).contiguous() if dsigma is not None else None
        _check(lib().pod_backward(self.h, ctypes.c_void_p(dUt.data_ptr()) if dUt is not None else None,
                                  ctypes.c_void_p(ds.data_ptr()) if ds is not None else None,
                                  ctypes.c_void_p(dAt.data_ptr())), "pod_backward")
        return dAt.T

    def col_sqnorms(self):
        import numpy as np
        nu = np.zeros(self.n, dtype=np.float64)
        _check(lib().pod_get_col_sqnorms(self.h, ctypes.c_void_p(nu.ctypes.data)), "pod_get_col_sqnorms")
        return nu

    def run(self, n_iter: Optional[int] = None, chunk: int = 8, stepwise: bool = False):
        """Alg. 1: sample/merge until converged, S is exhausted, max_iter
        merges were done, or (when given) n_iter merges were done.  Returns
        the convergence sines of the merges (NaN for the first).  The loop runs
        on the device (pod_run, one sync per `chunk` iterations) unless
        stepwise, which drives pod_sample / pod_merge / pod_converged."""
        if not stepwise:
            cap = int(n_iter) if n_iter is not None else min(int(self.params.max_iter), self.n)
            buf = (ctypes.c_double * max(cap, 1))()
            merged, done = ctypes.c_int32(), ctypes.c_int32()
            _check(lib().pod_run(self.h, cap, 1 if n_iter is None else 0, int(chunk), buf, ctypes.byref(merged),
                                 ctypes.byref(done)), "pod_run")
            return [buf[i] for i in range(merged.value)]
        sines = []
        while n_iter is None or len(sines) < n_iter:
            if not self.sample():
                break
            before = len(sines)
            self.merge()
            done, sn = self.converged()
            if done and self.info().iter == before:   # the draw found S exhausted: no merge happened
                break
            sines.append(sn)
            if done and n_iter is None:
                break
        return sines


def check_pairs(U, V, m: int, n: int, k: int, dtype, device):
    """The kernels behind wedin_bound read k columns of m (U) and n (V) rows
    in the context's output type: refuse anything else before the call."""
    for name, X, rows in (("U", U, m), ("V", V, n)):
        if tuple(X.shape) != (rows, k):
            raise ValueError(f"{name} must be {rows} x {k} (the pairs of the last project()), got {tuple(X.shape)}")
        if X.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {X.dtype}")
        if X.device != device:
            raise ValueError(f"{name} must live on {device}, got {X.device}")
        if not X.T.is_contiguous():
            raise ValueError(f"{name} must have contiguous columns (ld = {rows})")


def isma(A, k: int, c: int, want_v: bool = True, n_iter: Optional[int] = None, **kw) -> Result:
    """Run Alg. 1 on the device matrix A (m x n, contiguous columns) and the
    final projection; returns the first k modes."""
    with PodContext(A, k, c, **kw) as ctx:
        sines = ctx.run(n_iter=n_iter)
        inf = ctx.info()
        U, sig, V = ctx.project(want_v=want_v)
        return Result(U, sig, V, inf.iter, sines, bool(inf.exhausted), inf.stop_reason == POD_STOP_CONVERGED,
                      inf.flags, STOP_NAMES.get(inf.stop_reason, "unknown"))


class Incremental:
    """Alg. 3 over column blocks (pod_inc_*): ISMA on each block, BLOCK MERGE
    of its leading pairs into the running (U, Sigma).

    ``m``, ``max_block`` (largest block width) and the ISMA parameters are
    fixed at construction; ``dtype`` is the storage of the blocks."""

    def __init__(self, m: int, max_block: int, k: int, c: int, dtype="float32", r: int = 0, w: int = 0,
                 precision: int = POD_F32, theta_tol: float = 1e-10, col_strategy: int = POD_COL_L2N,
                 row_strategy: int = POD_ROW_L2, criterion: int = POD_CRIT_SUBSPACE,
                 max_iter: Optional[int] = None, seed: int = 0, r_update: int = 0, stream=None):
        import torch
        code = POD_F64 if str(dtype).endswith("float64") else POD_F32
        p = pod_params()
        p.m, p.n, p.lda, p.a_dtype, p.precision = m, max_block, m, code, precision
        p.k, p.r, p.c, p.w, p.r_update = k, r, c, w, r_update
        p.col_strategy, p.row_strategy, p.criterion = col_strategy, row_strategy, criterion
        p.center_rows = 0
        p.max_iter = int(max_iter if max_iter is not None else max_block + 1)
        p.theta_tol = float(theta_tol)
        p.seed = int(seed) & (2**64 - 1)
        self.params = p
        self.m, self.k = m, k
        self.code = code
        self.precision = precision
        self._torch_dtype = torch.float64 if code == POD_F64 else torch.float32
        self.stream = _stream_handle(stream)
        h = ctypes.c_void_p()
        _check(lib().pod_inc_init(ctypes.byref(h), ctypes.byref(p), self.stream), "pod_inc_init")
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().pod_inc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def add_block(self, B):
        """A device block (m x nb, contiguous columns)."""
        ptr, m, nb, ldb, code = _a_layout(B)
        if m != self.m or code != self.code:
            raise ValueError("block shape or dtype does not match")
        _check(lib().pod_inc_add_block(self.h, ctypes.c_void_p(ptr), nb, ldb), "pod_inc_add_block")

    def add_host_blocks(self, blocks):
        """Host blocks: CPU tensors of shape (nb, m) (row j = column j of the
        block), contiguous, ideally pinned; streamed through the device."""
        ptrs = (ctypes.c_void_p * len(blocks))()
        nbs = (ctypes.c_int64 * len(blocks))()
        for i, b in enumerate(blocks):
            if b.is_cuda or not b.is_contiguous() or b.dim() != 2 or b.shape[1] != self.m or b.dtype != self._torch_dtype:
                raise ValueError("host blocks must be contiguous CPU tensors of shape (nb, m)")
            ptrs[i] = b.data_ptr()
            nbs[i] = b.shape[0]
        _check(lib().pod_inc_add_host_blocks(self.h, ptrs, nbs, len(blocks)), "pod_inc_add_host_blocks")

    def result(self):
        import torch
        dt = torch.float64 if self.precision == POD_F64 else torch.float32
        Ut = torch.empty((self.k, self.m), dtype=dt, device="cuda")
        sig = torch.empty(self.k, dtype=torch.float64, device="cuda")
        kk = ctypes.c_int32()
        _check(lib().pod_inc_result(self.h, ctypes.c_void_p(Ut.data_ptr()), ctypes.c_void_p(sig.data_ptr()),
                                    ctypes.byref(kk)), "pod_inc_result")
        return Ut[:kk.value].T, sig[:kk.value]

    def info(self) -> pod_inc_info:
        inf = pod_inc_info()
        _check(lib().pod_inc_get_info(self.h, ctypes.byref(inf)), "pod_inc_get_info")
        return inf


def _params(A, k, c, r=0, w=0, precision=POD_F64, theta_tol=1e-10, col_strategy=POD_COL_L2N,
            row_strategy=POD_ROW_L2, criterion=POD_CRIT_SUBSPACE, max_iter=None, seed=0, block=0, r_update=0,
            center_rows=False):
    ptr, m, n, lda, code = _a_layout(A)
    p = pod_params()
    p.m, p.n, p.lda, p.a_dtype, p.precision = m, n, lda, code, precision
    p.k, p.r, p.c, p.w, p.r_update = k, r, c, w, r_update
    p.col_strategy, p.row_strategy, p.criterion = col_strategy, row_strategy, criterion
    p.center_rows = 1 if center_rows else 0
    p.max_iter = int(max_iter if max_iter is not None else n + 1)
    p.theta_tol = float(theta_tol)
    p.seed = int(seed) & (2**64 - 1)
    p.block = int(block)
    return p, ptr


class Batch:
    """Many ISMA runs advanced together (pod_batch_*).  ``mats`` is a list of
    device matrices (m_i x n_i, contiguous columns), ``params`` a list of
    keyword dicts (k, c, seed, ...) or one dict for all."""

    def __init__(self, mats, params):
        if isinstance(params, dict):
            params = [params] * len(mats)
        self.mats = list(mats)
        self.kw = [dict(p) for p in params]
        arr = (pod_params * len(mats))()
        ptrs = (ctypes.c_void_p * len(mats))()
        for i, (A, kw) in enumerate(zip(mats, self.kw)):
            arr[i], ptrs[i] = _params(A, **kw)
        h = ctypes.c_void_p()
        _check(lib().pod_batch_init(ctypes.byref(h), len(mats), arr, ptrs), "pod_batch_init")
        self.h = h
        self.params = arr

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().pod_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def autotune(self) -> int:
        n = ctypes.c_int32()
        _check(lib().pod_batch_autotune(self.h, ctypes.byref(n)), "pod_batch_autotune")
        return n.value

    def run(self, use_graph: bool = True, max_rounds: int = 1 << 20) -> int:
        r = ctypes.c_int32()
        _check(lib().pod_batch_run(self.h, 1 if use_graph else 0, int(max_rounds), ctypes.byref(r)), "pod_batch_run")
        return r.value

    def enable_adjoint(self):
        _check(lib().pod_batch_enable_adjoint(self.h), "pod_batch_enable_adjoint")

    def loss_grad(self, i: int):
        """(L_i, dL_i/dA_i) for L_i = |A_i - U_k U_k^T A_i|_F^2 of matrix i."""
        import torch
        p = self.params[i]
        dt = torch.float64 if p.precision == POD_F64 else torch.float32
        dAt = torch.zeros((p.n, p.m), dtype=dt, device=self.mats[i].device)
        L = ctypes.c_double()
        _check(lib().pod_batch_loss_grad(self.h, int(i), ctypes.c_void_p(dAt.data_ptr()), ctypes.byref(L)),
               "pod_batch_loss_grad")
        return L.value, dAt.T

    def loss_grad_all(self):
        """[(L_i, dL_i/dA_i)] for every matrix, the reverse steps of all matrices
        launched together (equal to loss_grad(i) bit for bit)."""
        import torch
        dAts = []
        for i, p in enumerate(self.params):
            dt = torch.float64 if p.precision == POD_F64 else torch.float32
            dAts.append(torch.zeros((p.n, p.m), dtype=dt, device=self.mats[i].device))
        ptrs = (ctypes.c_void_p * len(dAts))(*[t.data_ptr() for t in dAts])
        losses = (ctypes.c_double * len(dAts))()
        _check(lib().pod_batch_loss_grad_all(self.h, ptrs, losses), "pod_batch_loss_grad_all")
        return [(losses[i], dAts[i].T) for i in range(len(dAts))]

    def info(self, i: int):
        inf = pod_info()
        nb = ctypes.c_int32()
        _check(lib().pod_batch_get_info(self.h, int(i), ctypes.byref(inf), ctypes.byref(nb)), "pod_batch_get_info")
        return inf, nb.value

    def project(self, i: int, want_v: bool = False):
        import torch
        A = self.mats[i]
        p = self.params[i]
        inf, _ = self.info(i)
        k = min(p.k, inf.rank)
        dt = torch.float64 if p.precision == POD_F64 else torch.float32
        Ut = torch.empty((k, p.m), dtype=dt, device=A.device)
        sig = torch.empty(k, dtype=torch.float64, device=A.device)
        Vt = torch.empty((k, p.n), dtype=dt, device=A.device) if want_v else None
        _check(lib().pod_batch_project(self.h, int(i), ctypes.c_void_p(Ut.data_ptr()), ctypes.c_void_p(sig.data_ptr()),
                                       ctypes.c_void_p(Vt.data_ptr()) if want_v else None), "pod_batch_project")
        return Ut.T, sig, (Vt.T if want_v else None)


def _podfunction():
    import torch

    class PODFunction(torch.autograd.Function):
        """(U_k, Sigma_k) of the merge chain of Alg. 1 as a differentiable
        function of A; backward runs pod_backward (the sampled columns are
        constants).  U_k is the basis before the final step."""

        @staticmethod
        def forward(fctx, A, k, c, kw):
            pc = PodContext(A.detach(), k, c, **kw)
            pc.enable_adjoint()
            pc.run()
            U, s = pc.basis()
            kk = min(k, U.shape[1])
            fctx.pc = pc
            return U[:, :kk].clone(), s[:kk].clone()

        @staticmethod
        def backward(fctx, dU, dsigma):
            pc = fctx.pc
            dA = pc.backward(dU, dsigma)
            pc.close()
            return dA, None, None, None

    return PODFunction


def pod_function(A, k: int, c: int, **kw):
    """Differentiable (U_k, Sigma_k) = ISMA merge chain of A (see PODFunction)."""
    return _podfunction().apply(A, k, c, kw)


POD_K = dict(colnorms=0, draw=1, gram=2, gram_reduce=3, chol=4, tall=5, svd=6, project=7, rr=8, sign=9)


def profile_enable(kclass):
    """Time every launch of one kernel class with HIP events (None disables)."""
    code = -1 if kclass is None else (POD_K[kclass] if isinstance(kclass, str) else int(kclass))
    _check(lib().pod_profile_enable(code), "pod_profile_enable")


def profile_read():
    """(launches, total ms) of the enabled class since the last read."""
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(lib().pod_profile_read(ctypes.byref(n), ctypes.byref(ms)), "pod_profile_read")
    return n.value, ms.value


def oneshot(A, k: int, c: int, w: int = 0, eps: float = 0.6, seed: int = 0, precision: int = POD_F64,
            block: int = 0, center_rows: bool = False, stream=None):
    """One-shot sampled SVD of Appendix A on the device matrix A: Alg. 4
    (LTSVD) for w = 0, Alg. 5 (CTSVD) for w > 0.  Returns (U (m x k), sigma (k),
    l): the first l columns and values are the method's output, the rest zero."""
    import torch
    p, ptr = _params(A, k, c, w=w, precision=precision, seed=seed, block=block, center_rows=center_rows)
    dt = torch.float64 if precision == POD_F64 else torch.float32
    Ut = torch.empty((k, p.m), dtype=dt, device=A.device)
    sig = torch.empty(k, dtype=torch.float64, device=A.device)
    l = ctypes.c_int32()
    _check(lib().pod_oneshot(ctypes.byref(p), ctypes.c_void_p(ptr), float(eps), ctypes.c_void_p(Ut.data_ptr()),
                             ctypes.c_void_p(sig.data_ptr()), ctypes.byref(l), _stream_handle(stream)), "pod_oneshot")
    return Ut.T, sig, l.value


def center_rows(A, stream=None):
    """Subtract the FP64 row means of the device matrix A (m x n, contiguous
    columns) in place (pod_center_rows)."""
    ptr, m, n, lda, code = _a_layout(A)
    _check(lib().pod_center_rows(ctypes.c_void_p(ptr), code, m, n, lda, _stream_handle(stream)), "pod_center_rows")
    return A


def center_rows_noalloc(A, stream=None):
    """center_rows without any device allocation (the library's own device
    scratch, m <= 4,194,304 rows); stream-ordered, no sync."""
    ptr, m, n, lda, code = _a_layout(A)
    _check(lib().pod_center_rows_noalloc(ctypes.c_void_p(ptr), code, m, n, lda, _stream_handle(stream)),
           "pod_center_rows_noalloc")
    return A


def col_sqnorms(A, stream=None):
    """Column squared norms of a device matrix in the library's fixed order."""
    import torch
    ptr, m, n, lda, code = _a_layout(A)
    nu = torch.empty(n, dtype=torch.float64, device=A.device)
    _check(lib().pod_col_sqnorms(ctypes.c_void_p(ptr), code, m, n, lda, ctypes.c_void_p(nu.data_ptr()),
                                 _stream_handle(stream)), "pod_col_sqnorms")
    return nu

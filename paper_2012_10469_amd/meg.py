"""ctypes binding of the MI355X low-rank MEG library (include/meg.h).

The functions here marshal arguments only; every step of the method runs in
the HIP kernels of ``libmeg.so``.  Importing this module loads the library and
fails loudly if it has not been built (``python -m paper_2012_10469_amd.build``).

Low-level names mirror the C ABI (``meg_init``, ``meg_step``, ``meg_solve``,
``meg_certificate``, ...).  ``LowRankMEG`` is a thin convenience wrapper that
keeps the borrowed device arrays alive for the context's lifetime.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Any, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmeg.so")

# ---- enums (include/meg.h) -------------------------------------------------
MEG_OK = 0
MEG_ERR_INVALID_ARG = 1
MEG_ERR_OUT_OF_MEMORY = 2
MEG_ERR_DEVICE = 3
MEG_ERR_NUMERIC = 4
MEG_ERR_NOT_CONVERGED = 5
MEG_ERR_STATE = 6
MEG_ERR_UNSUPPORTED = 7

MEG_PREC_F64 = 0
MEG_PREC_F32 = 1
MEG_PREC_F32_BF16X3 = 2

MEG_GRAD_LINEAR_DENSE = 0
MEG_GRAD_DENOISE_DENSE = 1
MEG_GRAD_LINEAR_CSR = 2
MEG_GRAD_MASKED_CSR = 3
MEG_GRAD_QUADMEAS = 4
MEG_GRAD_EXTERNAL = 5
MEG_GRAD_BILINEAR = 6

MEG_FLAG_STRICT = 1
MEG_FLAG_NO_LDS_CACHE = 2
MEG_FLAG_NO_EXTRAPOLATE = 4
MEG_FLAG_NO_CHEBYSHEV = 8
MEG_FLAG_DUAL_AVERAGE = 16
MEG_SERVER_FLAG_GRAPH = 1

EXPORTED = [
    "meg_block_size", "meg_init", "meg_step", "meg_solve", "meg_certificate", "meg_objective_value",
    "meg_get_iterate", "meg_set_iterate", "meg_get_state", "meg_set_state", "meg_profile_step", "meg_destroy",
    "meg_status_str", "meg_get_counters", "meg_step_external", "meg_dual_gap", "meg_solve_to_gap",
    "meg_trace_exp", "meg_certificate_full", "meg_dual_gap_static", "meg_certificate_bound",
    "meg_exact_create", "meg_exact_step", "meg_exact_get", "meg_exact_bregman", "meg_exact_destroy",
    "meg_server_create", "meg_server_submit", "meg_server_run", "meg_server_query", "meg_server_result",
    "meg_server_release", "meg_server_team", "meg_server_get_stats", "meg_server_destroy",
]


class MegParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("r", ctypes.c_int32), ("oversample", ctypes.c_int32),
        ("prec", ctypes.c_int32), ("min_inner", ctypes.c_int32), ("max_inner", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("eta", ctypes.c_double), ("eps_scale", ctypes.c_double),
        ("eps_c", ctypes.c_double), ("eps_pow", ctypes.c_double), ("inner_tol", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("cert_tol", ctypes.c_double),
    ]


class MegObjective(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("dense", ctypes.c_void_p), ("dense_lo", ctypes.c_void_p), ("ld", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p), ("nnz", ctypes.c_int64),
        ("A", ctypes.c_void_p), ("lda", ctypes.c_int64), ("b", ctypes.c_void_p), ("m", ctypes.c_int64),
        ("batch_idx", ctypes.c_void_p), ("batch_steps", ctypes.c_int64),
    ]


class MegStart(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("V0", ctypes.POINTER(ctypes.c_double)), ("lambda0", ctypes.POINTER(ctypes.c_double))]


class MegStepInfo(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_int64), ("f", ctypes.c_double), ("eps_t", ctypes.c_double), ("cert_L", ctypes.c_double),
        ("cert_bound", ctypes.c_double), ("cert_holds", ctypes.c_int32), ("inner_iters", ctypes.c_int32),
        ("ritz_gap", ctypes.c_double), ("resid_max", ctypes.c_double), ("mu_r1", ctypes.c_double),
        ("sigma", ctypes.c_double), ("converged", ctypes.c_int32), ("cert_resolved", ctypes.c_int32),
        ("resid_r1", ctypes.c_double), ("cert_L_up", ctypes.c_double), ("mu_r1_up", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class MegKernelTimes(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("prep_ms", ctypes.c_double), ("apply_ms", ctypes.c_double * 64),
                ("small_ms", ctypes.c_double * 64), ("finalize_ms", ctypes.c_double),
                ("sweeps_active", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("wg_apply_ms", (ctypes.c_double * 3) * 2), ("wg_skew_ms", ctypes.c_double * 2),
                ("reduce_ms", ctypes.c_double * 2), ("rr_ms", ctypes.c_double * 3), ("rr_tail_ms", ctypes.c_double),
                ("jacobi_sweeps", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class MegCounters(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("iterations", ctypes.c_int64), ("applies", ctypes.c_int64),
                ("workgroups", ctypes.c_int32), ("jacobi_sweeps", ctypes.c_int32), ("kernel_ms", ctypes.c_double),
                ("extrapolated", ctypes.c_int64), ("unconverged", ctypes.c_int64)]


class MegCertBoundInfo(ctypes.Structure):
    _fields_ = [("mu_up", ctypes.c_double), ("lambda_min_defl", ctypes.c_double), ("resid", ctypes.c_double),
                ("t", ctypes.c_int64), ("steps", ctypes.c_int32), ("converged", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class MegExactInfo(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("f", ctypes.c_double)]


class MegDualGapInfo(ctypes.Structure):
    _fields_ = [("gap", ctypes.c_double), ("x_dot_g", ctypes.c_double), ("lambda_min", ctypes.c_double),
                ("resid", ctypes.c_double), ("t", ctypes.c_int64), ("steps", ctypes.c_int32),
                ("converged", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class MegTraceInfo(ctypes.Structure):
    _fields_ = [("log_b", ctypes.c_double), ("log_b_defl", ctypes.c_double), ("log_b_tail", ctypes.c_double),
                ("tail_rel_stderr", ctypes.c_double), ("t", ctypes.c_int64), ("kd", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("converged", ctypes.c_int32), ("batches", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class MegServerParams(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("launch_steps", ctypes.c_int32),
                ("max_resident", ctypes.c_int32), ("flags", ctypes.c_uint32), ("fixed_team", ctypes.c_int32)]


class MegRequest(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("r", ctypes.c_int32), ("n", ctypes.c_int64), ("M", ctypes.c_void_p),
        ("ld", ctypes.c_int64), ("q", ctypes.c_int32), ("max_iters", ctypes.c_int32),
        ("V0", ctypes.POINTER(ctypes.c_double)), ("lambda0", ctypes.POINTER(ctypes.c_double)),
        ("eta", ctypes.c_double), ("eps_scale", ctypes.c_double), ("eps_c", ctypes.c_double),
        ("eps_pow", ctypes.c_double), ("tol", ctypes.c_double), ("oversample", ctypes.c_int32),
        ("max_inner", ctypes.c_int32), ("seed", ctypes.c_uint64),
    ]


class MegRequestStatus(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("iterations", ctypes.c_int64),
                ("submit_ms", ctypes.c_double), ("admit_ms", ctypes.c_double), ("done_ms", ctypes.c_double),
                ("team", ctypes.c_int32), ("reserved", ctypes.c_int32), ("last", MegStepInfo),
                ("applies", ctypes.c_int64)]


class MegServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("iterations", ctypes.c_int64), ("kernel_ms", ctypes.c_double),
                ("resident", ctypes.c_int32), ("queued", ctypes.c_int32), ("capacity_wg", ctypes.c_int32),
                ("graph_node", ctypes.c_int32), ("arena_bytes", ctypes.c_int64), ("arena_used", ctypes.c_int64),
                ("arena_peak", ctypes.c_int64)]


_lib: Optional[ctypes.CDLL] = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmeg.so and declare the C signatures (raises if missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libmeg.so not built: {path} (run python -m paper_2012_10469_amd.build)")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    sig = {
        "meg_block_size": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32]),
        "meg_init": (ctypes.c_int, [P(vp), P(MegParams), P(MegObjective), P(MegStart), vp]),
        "meg_step": (ctypes.c_int, [vp, P(MegStepInfo)]),
        "meg_step_external": (ctypes.c_int, [vp, P(MegObjective), P(MegStepInfo)]),
        "meg_solve": (ctypes.c_int, [vp, ctypes.c_int64, ctypes.c_double, P(MegStepInfo)]),
        "meg_certificate": (ctypes.c_int, [vp, P(MegStepInfo)]),
        "meg_objective_value": (ctypes.c_int, [vp, P(ctypes.c_double)]),
        "meg_get_iterate": (ctypes.c_int, [vp, P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double),
                                           P(ctypes.c_int64)]),
        "meg_set_iterate": (ctypes.c_int, [vp, P(ctypes.c_double), ctypes.c_int32, P(ctypes.c_double),
                                           ctypes.c_double, ctypes.c_int64]),
        "meg_get_state": (ctypes.c_int, [vp, vp, P(ctypes.c_size_t)]),
        "meg_set_state": (ctypes.c_int, [vp, vp, ctypes.c_size_t]),
        "meg_profile_step": (ctypes.c_int, [vp, P(MegKernelTimes)]),
        "meg_get_counters": (ctypes.c_int, [vp, P(MegCounters), ctypes.c_int32]),
        "meg_dual_gap": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_double, P(MegDualGapInfo)]),
        "meg_dual_gap_static": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_double, P(MegDualGapInfo)]),
        "meg_certificate_bound": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_double, P(MegCertBoundInfo)]),
        "meg_trace_exp": (ctypes.c_int, [vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                         P(MegTraceInfo)]),
        "meg_certificate_full": (ctypes.c_int, [vp, P(MegTraceInfo), P(ctypes.c_double), P(ctypes.c_int32)]),
        "meg_solve_to_gap": (ctypes.c_int, [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, P(MegStepInfo),
                                            P(MegDualGapInfo)]),
        "meg_destroy": (None, [vp]),
        "meg_exact_create": (ctypes.c_int, [P(vp), P(MegParams), P(MegObjective), P(MegStart), vp]),
        "meg_exact_step": (ctypes.c_int, [vp, P(MegExactInfo)]),
        "meg_exact_get": (ctypes.c_int, [vp, P(ctypes.c_double), P(ctypes.c_int64)]),
        "meg_exact_bregman": (ctypes.c_int, [vp, P(ctypes.c_double), ctypes.c_int32, P(ctypes.c_double),
                                             ctypes.c_double, P(ctypes.c_double)]),
        "meg_exact_destroy": (None, [vp]),
        "meg_status_str": (ctypes.c_char_p, [ctypes.c_int]),
        "meg_server_create": (ctypes.c_int, [P(vp), P(MegServerParams), vp]),
        "meg_server_submit": (ctypes.c_int, [vp, P(MegRequest), P(ctypes.c_int64)]),
        "meg_server_run": (ctypes.c_int, [vp, ctypes.c_int32, P(ctypes.c_int32)]),
        "meg_server_query": (ctypes.c_int, [vp, ctypes.c_int64, P(MegRequestStatus)]),
        "meg_server_result": (ctypes.c_int, [vp, ctypes.c_int64, P(ctypes.c_double), P(ctypes.c_double),
                                             P(ctypes.c_double)]),
        "meg_server_release": (ctypes.c_int, [vp, ctypes.c_int64]),
        "meg_server_team": (ctypes.c_int, [vp, ctypes.c_int64, P(ctypes.c_int32), P(ctypes.c_int32)]),
        "meg_server_get_stats": (ctypes.c_int, [vp, P(MegServerStats)]),
        "meg_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MegError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load_library()
        super().__init__(f"{where}: {lib.meg_status_str(status).decode()} (status {status})")
        self.status = status


def _check(status: int, where: str) -> None:
    if status != MEG_OK:
        raise MegError(status, where)


def _dptr(t: Any) -> Optional[int]:
    """Device pointer of a torch tensor (or an int address, or None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _dblp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---- thin wrappers with the C names ----------------------------------------
def meg_block_size(r: int, oversample: int) -> int:
    return int(load_library().meg_block_size(r, oversample))


def meg_status_str(status: int) -> str:
    return load_library().meg_status_str(status).decode()


def make_params(n, r, prec=MEG_PREC_F32, eta=1.0, oversample=4, eps=(0.8, 10.0, 2.0), min_inner=1,
                max_inner=12, inner_tol=0.0, seed=0, flags=0, cert_tol=0.0) -> MegParams:
    return MegParams(n=n, r=r, oversample=oversample, prec=prec, min_inner=min_inner, max_inner=max_inner,
                     flags=flags, eta=eta, eps_scale=eps[0], eps_c=eps[1], eps_pow=eps[2], inner_tol=inner_tol,
                     seed=seed, cert_tol=cert_tol)


def meg_init(params: MegParams, obj: MegObjective, V0, lam0, stream: Optional[int] = None):
    """Returns (status, ctx_handle).  V0 is n x q (host), lam0 length q."""
    lib = load_library()
    V0 = np.asarray(V0, dtype=np.float64)
    if V0.ndim == 1:
        V0 = V0[:, None]
    Vc = np.asfortranarray(V0)  # n x q column-major
    lam = _f64(lam0)
    start = MegStart(q=Vc.shape[1], reserved=0, V0=Vc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     lambda0=_dblp(lam))
    ctx = ctypes.c_void_p()
    st = lib.meg_init(ctypes.byref(ctx), ctypes.byref(params), ctypes.byref(obj), ctypes.byref(start),
                      ctypes.c_void_p(stream) if stream else None)
    return st, ctx


class ExactMEG:
    """Exact MEG (Algorithm 1) on the GPU: dense FP64 iterates W_t from the
    low-rank method's first iterate for the same start (meg_exact_*).
    ``dense`` is the float64 device matrix C (linear) or M (denoising)."""

    def __init__(self, n: int, kind: int, V0, lam0, dense, *, eta: float = 1.0, eps=(0.8, 10.0, 2.0),
                 stream: Optional[int] = None):
        import torch

        self._lib = load_library()
        self._keep = [dense]
        self.n = int(n)
        obj = MegObjective(kind=kind, dense=_dptr(dense), ld=int(dense.stride(0)))
        params = make_params(n, 1, MEG_PREC_F64, eta, 0, eps, 1, 1, 0.0, 0, 0, 0.0)
        V0 = np.asarray(V0, dtype=np.float64)
        if V0.ndim == 1:
            V0 = V0[:, None]
        Vc = np.asfortranarray(V0)
        lam = _f64(lam0)
        start = MegStart(q=Vc.shape[1], reserved=0, V0=Vc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         lambda0=_dblp(lam))
        if stream is None:
            self._torch_stream = torch.cuda.Stream()
            stream = self._torch_stream.cuda_stream
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _check(self._lib.meg_exact_create(ctypes.byref(h), ctypes.byref(params), ctypes.byref(obj),
                                          ctypes.byref(start), ctypes.c_void_p(stream)), "meg_exact_create")
        self._h = h

    def step(self) -> dict:
        out = MegExactInfo()
        _check(self._lib.meg_exact_step(self._h, ctypes.byref(out)), "meg_exact_step")
        return {"t": out.t, "f": out.f}

    def get(self):
        W = np.empty((self.n, self.n), dtype=np.float64)
        t = ctypes.c_int64()
        _check(self._lib.meg_exact_get(self._h, W.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       ctypes.byref(t)), "meg_exact_get")
        return W, t.value

    def bregman(self, V, d, alpha) -> float:
        """B(W_t, X) for the factored X = alpha I + V diag(d) V^T."""
        Vc = np.asfortranarray(np.asarray(V, dtype=np.float64))
        dd = _f64(d)
        out = ctypes.c_double()
        _check(self._lib.meg_exact_bregman(self._h, Vc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           int(Vc.shape[1]), _dblp(dd), float(alpha), ctypes.byref(out)),
               "meg_exact_bregman")
        return out.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.meg_exact_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LowRankMEG:
    """One low-rank MEG problem instance on the current HIP stream.

    Device arrays (torch tensors) are borrowed by the library and referenced
    here until ``close()``.  Dense data: ``dense`` (n x n, float64 for F64,
    float32 for F32; for F32_BF16X3 the bf16 hi plane as a 16-bit tensor,
    with ``dense_lo`` the lo plane, rows of ``ld`` elements).  CSR data:
    ``row_ptr``/``col`` int32, ``val``.
    """

    def __init__(self, n: int, r: int, kind: int, V0, lam0, *, prec: int = MEG_PREC_F32, eta: float = 1.0,
                 dense=None, dense_lo=None, row_ptr=None, col=None, val=None, A=None, b=None, batch_idx=None,
                 oversample: int = 4, eps=(0.8, 10.0, 2.0), min_inner: int = 1, max_inner: int = 12,
                 inner_tol: float = 0.0, seed: int = 0, flags: int = 0, cert_tol: float = 0.0,
                 stream: Optional[int] = None, meas_rank: int = 1):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("LowRankMEG needs a visible GPU")
        self._lib = load_library()
        self._keep = [dense, dense_lo, row_ptr, col, val, A, b, batch_idx]
        self.n, self.r = int(n), int(r)
        self.kind = kind
        # quadratic measurements: A is m x lda (row i = a_i), batch_idx int32
        # batch_steps x L (step t uses row (t - 1) mod batch_steps); bilinear
        # measurements: A is 2mp x lda (columns of A_1..A_m, then of B_1..B_m),
        # b holds y, meas_rank = p
        if kind == MEG_GRAD_BILINEAR and A is not None:
            m = int(A.shape[0]) // (2 * max(1, meas_rank))
        else:
            m = 0 if A is None else int(A.shape[0])
        batch = int(batch_idx.shape[1]) if batch_idx is not None else (int(meas_rank) if kind == MEG_GRAD_BILINEAR
                                                                      else 0)
        obj = MegObjective(kind=kind, batch=batch,
                           dense=_dptr(dense), dense_lo=_dptr(dense_lo),
                           ld=int(dense.stride(0)) if dense is not None else 0,
                           row_ptr=_dptr(row_ptr), col=_dptr(col), val=_dptr(val),
                           nnz=int(col.numel()) if col is not None else 0,
                           A=_dptr(A), lda=int(A.stride(0)) if A is not None else 0, b=_dptr(b),
                           m=m, batch_idx=_dptr(batch_idx),
                           batch_steps=int(batch_idx.shape[0]) if batch_idx is not None else 0)
        params = make_params(n, r, prec, eta, oversample, eps, min_inner, max_inner, inner_tol, seed, flags,
                             cert_tol)
        if stream is None:
            # a dedicated (default-priority) stream: graph capture needs a
            # stream other than the legacy null stream
            self._torch_stream = torch.cuda.Stream()
            stream = self._torch_stream.cuda_stream
        torch.cuda.synchronize()  # uploads on other streams are complete
        self.stream = stream
        st, ctx = meg_init(params, obj, V0, lam0, stream)
        _check(st, "meg_init")
        self._ctx = ctx
        self.k = meg_block_size(r, oversample)

    # -- C ABI calls --
    def step(self, info: bool = True) -> Optional[dict]:
        if not info:
            _check(self._lib.meg_step(self._ctx, None), "meg_step")
            return None
        out = MegStepInfo()
        _check(self._lib.meg_step(self._ctx, ctypes.byref(out)), "meg_step")
        return out.as_dict()

    def step_external(self, dense=None, row_ptr=None, col=None, val=None, info: bool = True) -> Optional[dict]:
        """One step with the caller's gradient G_t at the current iterate
        (context created with kind MEG_GRAD_EXTERNAL): dense n x n, or CSR
        (row_ptr, col, val), device tensors in the state's type."""
        if dense is not None:
            g = MegObjective(kind=MEG_GRAD_LINEAR_DENSE, dense=_dptr(dense), ld=int(dense.stride(0)))
        else:
            g = MegObjective(kind=MEG_GRAD_LINEAR_CSR, row_ptr=_dptr(row_ptr), col=_dptr(col), val=_dptr(val),
                             nnz=int(col.numel()))
        out = MegStepInfo()
        _check(self._lib.meg_step_external(self._ctx, ctypes.byref(g), ctypes.byref(out) if info else None),
               "meg_step_external")
        return out.as_dict() if info else None

    def solve(self, max_iters: int, tol: float = 0.0) -> dict:
        out = MegStepInfo()
        _check(self._lib.meg_solve(self._ctx, int(max_iters), float(tol), ctypes.byref(out)), "meg_solve")
        return out.as_dict()

    def certificate(self) -> dict:
        out = MegStepInfo()
        _check(self._lib.meg_certificate(self._ctx, ctypes.byref(out)), "meg_certificate")
        return out.as_dict()

    def objective(self) -> float:
        f = ctypes.c_double()
        _check(self._lib.meg_objective_value(self._ctx, ctypes.byref(f)), "meg_objective_value")
        return f.value

    def get_iterate(self):
        """Returns (V n x r float64, d r, alpha, t)."""
        V = np.zeros((self.r, self.n), dtype=np.float64)  # column-major n x r == row-major r x n
        d = np.zeros(self.r)
        a = ctypes.c_double()
        t = ctypes.c_int64()
        _check(self._lib.meg_get_iterate(self._ctx, _dblp(V), _dblp(d), ctypes.byref(a), ctypes.byref(t)),
               "meg_get_iterate")
        return V.T.copy(), d, a.value, t.value

    def set_iterate(self, V, d, alpha: float, t: int) -> None:
        V = np.asarray(V, dtype=np.float64)
        Vc = np.asfortranarray(V)
        dd = _f64(d)
        _check(self._lib.meg_set_iterate(self._ctx, Vc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         int(Vc.shape[1]), _dblp(dd), float(alpha), int(t)), "meg_set_iterate")

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        _check(self._lib.meg_get_state(self._ctx, None, ctypes.byref(n)), "meg_get_state")
        buf = ctypes.create_string_buffer(n.value)
        _check(self._lib.meg_get_state(self._ctx, buf, ctypes.byref(n)), "meg_get_state")
        return buf.raw[: n.value]

    def set_state(self, blob: bytes) -> None:
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self._lib.meg_set_state(self._ctx, buf, len(blob)), "meg_set_state")

    def profile_step(self) -> dict:
        """Run one step: HIP-event time of the step kernel and its phase times
        from the kernel's own wall-clock stamps (milliseconds)."""
        out = MegKernelTimes()
        _check(self._lib.meg_profile_step(self._ctx, ctypes.byref(out)), "meg_profile_step")
        a = out.sweeps_active
        return {"kernel_ms": out.kernel_ms, "prep_ms": out.prep_ms, "apply_ms": list(out.apply_ms[:a]),
                "small_ms": list(out.small_ms[:a]), "finalize_ms": out.finalize_ms, "sweeps_active": a,
                "workgroups": out.workgroups,
                "wg_apply_ms": [list(out.wg_apply_ms[s]) for s in range(min(a, 2))],
                "wg_skew_ms": list(out.wg_skew_ms[:min(a, 2)]), "reduce_ms": list(out.reduce_ms[:min(a, 2)]),
                "rr_ms": list(out.rr_ms) + [out.rr_tail_ms], "jacobi_sweeps": out.jacobi_sweeps}

    def counters(self, reset: bool = False) -> dict:
        """Step-kernel launches, iterations, operator applies, Jacobi sweeps and
        their summed HIP-event GPU time (ms) since init or the last reset;
        synchronises."""
        out = MegCounters()
        _check(self._lib.meg_get_counters(self._ctx, ctypes.byref(out), 1 if reset else 0), "meg_get_counters")
        return {"launches": out.launches, "iterations": out.iterations, "applies": out.applies,
                "workgroups": out.workgroups, "jacobi_sweeps": out.jacobi_sweeps, "kernel_ms": out.kernel_ms,
                "extrapolated": out.extrapolated, "unconverged": out.unconverged}

    def dual_gap(self, max_steps: int = 128, tol: float = 1e-10) -> dict:
        """Dual gap <X_t, G> - lambda_min(G) at the current iterate (G its
        gradient), with the Lanczos run's step count and residual; synchronises."""
        out = MegDualGapInfo()
        _check(self._lib.meg_dual_gap(self._ctx, int(max_steps), float(tol), ctypes.byref(out)), "meg_dual_gap")
        return out.as_dict()

    def dual_gap_static(self, max_steps: int = 128, tol: float = 1e-10) -> dict:
        """dual_gap through the allocation-free entry point (the library's fixed
        device workspace, a fresh start vector every call)."""
        out = MegDualGapInfo()
        _check(self._lib.meg_dual_gap_static(self._ctx, int(max_steps), float(tol), ctypes.byref(out)),
               "meg_dual_gap_static")
        return out.as_dict()

    def certificate_bound(self, max_steps: int = 128, tol: float = 1e-10) -> dict:
        """Upper bound of mu_{r+1} for the next step (armed for it); synchronises."""
        out = MegCertBoundInfo()
        _check(self._lib.meg_certificate_bound(self._ctx, int(max_steps), float(tol), ctypes.byref(out)),
               "meg_certificate_bound")
        return out.as_dict()

    def trace_exp(self, probes=None, weight: Optional[float] = None, max_steps: int = 64, tol: float = 1e-10):
        """Estimate of b_n = tr exp(M_t) for the current iterate (the matrix the
        next step decomposes): the solver block's span exactly, the rest from
        the probes (a float64 device tensor n x p, probe j = probes[:, j]; the
        library reads it column by column, so it is passed as its transpose's
        contiguous copy).  weight defaults to 1/p.  Returns the info dict and
        the MegTraceInfo for certificate_full."""
        p = 0 if probes is None else int(probes.shape[1])
        ptr = None
        if p > 0:
            import torch

            if probes.dtype != torch.float64 or not probes.is_cuda or probes.dim() != 2:
                raise ValueError("probes must be a 2-D float64 device tensor (n x p)")
            pt = probes.t().contiguous()
            self._keep_probe = pt
            ptr = _dptr(pt)
        w = (1.0 / p if p > 0 else 1.0) if weight is None else float(weight)
        out = MegTraceInfo()
        _check(self._lib.meg_trace_exp(self._ctx, ptr, p, w, int(max_steps), float(tol), ctypes.byref(out)),
               "meg_trace_exp")
        self._keep_probe = None
        return out.as_dict(), out

    def certificate_full(self, trace: "MegTraceInfo") -> tuple:
        """(L_full, holds) of the most recent step from a trace estimate taken
        at the iterate that step started from."""
        L, h = ctypes.c_double(), ctypes.c_int32()
        _check(self._lib.meg_certificate_full(self._ctx, ctypes.byref(trace), ctypes.byref(L), ctypes.byref(h)),
               "meg_certificate_full")
        return L.value, h.value

    def solve_to_gap(self, max_iters: int, tol: float, check_every: int = 8) -> tuple:
        """Iterate until the dual gap is <= tol (checked every check_every
        iterations) or max_iters; returns (last step info, last gap)."""
        info, gap = MegStepInfo(), MegDualGapInfo()
        _check(self._lib.meg_solve_to_gap(self._ctx, int(max_iters), float(tol), int(check_every), ctypes.byref(info),
                                          ctypes.byref(gap)), "meg_solve_to_gap")
        return info.as_dict(), gap.as_dict()

    def close(self) -> None:
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self._lib.meg_destroy(self._ctx)
            self._ctx = None
        self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class MegServer:
    """Batched server (meg_server_* of the C ABI) on its own HIP stream.

    ``submit`` takes a device FP32 matrix (torch tensor, n x n, row-major),
    borrowed until the request is admitted; the start (V0, lam0) is host
    data.  ``run(rounds)`` performs scheduling rounds (retire, admit, one
    launch of the batched kernel) and returns the number of pending requests.
    """

    def __init__(self, budget_bytes: int = 0, launch_steps: int = 8, max_resident: int = 256,
                 graph: bool = False, fixed_team: int = 0, stream: Optional[int] = None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("MegServer needs a visible GPU")
        self._lib = load_library()
        if stream is None:
            self._torch_stream = torch.cuda.Stream()
            stream = self._torch_stream.cuda_stream
        self.stream = stream
        p = MegServerParams(budget_bytes=int(budget_bytes), launch_steps=int(launch_steps),
                            max_resident=int(max_resident), flags=MEG_SERVER_FLAG_GRAPH if graph else 0,
                            fixed_team=int(fixed_team))
        h = ctypes.c_void_p()
        _check(self._lib.meg_server_create(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p(stream)),
               "meg_server_create")
        self._h = h
        self._keep = {}

    def submit(self, M, V0, lam0, r: int, *, kind: int = MEG_GRAD_DENOISE_DENSE, eta: float = 1.0,
               eps=(0.8, 10.0, 2.0), tol: float = 0.0, max_iters: int = 300, max_inner: int = 12,
               oversample: int = 4, seed: int = 0) -> int:
        V0 = np.asarray(V0, dtype=np.float64)
        if V0.ndim == 1:
            V0 = V0[:, None]
        Vc = np.asfortranarray(V0)
        lam = _f64(lam0)
        n = int(M.shape[0])
        req = MegRequest(kind=kind, r=int(r), n=n, M=_dptr(M), ld=int(M.stride(0)), q=int(Vc.shape[1]),
                         max_iters=int(max_iters), V0=Vc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         lambda0=_dblp(lam), eta=float(eta), eps_scale=eps[0], eps_c=eps[1], eps_pow=eps[2],
                         tol=float(tol), oversample=int(oversample), max_inner=int(max_inner), seed=int(seed))
        rid = ctypes.c_int64()
        _check(self._lib.meg_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)), "meg_server_submit")
        self._keep[rid.value] = M  # borrowed until admitted
        return rid.value

    def run(self, rounds: int = 1) -> int:
        pend = ctypes.c_int32()
        _check(self._lib.meg_server_run(self._h, int(rounds), ctypes.byref(pend)), "meg_server_run")
        for rid in list(self._keep):
            if self.query(rid)["state"] >= 1:
                del self._keep[rid]
        return pend.value

    def query(self, rid: int) -> dict:
        st = MegRequestStatus()
        _check(self._lib.meg_server_query(self._h, int(rid), ctypes.byref(st)), "meg_server_query")
        out = {name: getattr(st, name) for name, _ in st._fields_ if name not in ("reserved", "last")}
        out["last"] = st.last.as_dict()
        return out

    def result(self, rid: int, n: int, r: int):
        """(V n x r, d, alpha) of a done request."""
        V = np.zeros((r, n), dtype=np.float64)
        d = np.zeros(r)
        a = ctypes.c_double()
        _check(self._lib.meg_server_result(self._h, int(rid), _dblp(V), _dblp(d), ctypes.byref(a)),
               "meg_server_result")
        return V.T.copy(), d, a.value

    def release(self, rid: int) -> None:
        _check(self._lib.meg_server_release(self._h, int(rid)), "meg_server_release")

    def team(self, n: int) -> tuple:
        """(latency, throughput) team sizes for dimension n (autotuned on first use)."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.meg_server_team(self._h, int(n), ctypes.byref(a), ctypes.byref(b)), "meg_server_team")
        return a.value, b.value

    def stats(self) -> dict:
        st = MegServerStats()
        _check(self._lib.meg_server_get_stats(self._h, ctypes.byref(st)), "meg_server_get_stats")
        return {name: getattr(st, name) for name, _ in st._fields_ if name != "reserved"}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.meg_server_destroy(self._h)
            self._h = None
        self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

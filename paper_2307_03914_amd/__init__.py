"""BSPAI-GMRES-IR on MI355X: Python binding of ``libbspai.so``.

Argument marshalling only: every step of the method runs in the HIP library
(``csrc/``); PyTorch provides device memory and the current stream.  The
functions mirror the C interface in ``include/bspai.h``:

* :func:`build` / :func:`import_m` -> :class:`Handle` (``bspai_build`` /
  ``bspai_import``): SPAI of A on a pattern (FP64 Householder least squares,
  run on A^T and transposed), then bucketing of its entries by magnitude.
* :func:`apply` / :func:`apply_T` (``bspai_apply`` / ``bspai_apply_T``).
* :func:`solve` (``gmres_ir_solve``): GMRES-based iterative refinement, one
  or up to 64 right-hand sides.
* :class:`MultiPlan` (``bspai_multi_*``): many independent systems in one
  persistent launch, replayed from a captured HIP graph.
* :class:`BSPAISolve`: ``torch.autograd.Function`` whose backward solves the
  adjoint system with the transposed bucketed preconditioner.

The library must be built (``__graft_entry__.build()``); importing this
package without it raises ImportError — there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import sys
from typing import Dict, List, Optional, Sequence, Tuple

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libbspai.so")

FP64, FP32, FP16, BF16, FP8_E4M3, DROP = 0, 1, 2, 3, 4, 5
PREC = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16, "fp8": FP8_E4M3, "fp8_e4m3": FP8_E4M3,
        "drop": DROP}
OK, EINVAL, ENOMEM, EHIP, EZEROROW, ERANK, ENOCONV, ENAN, ESTAG = 0, -1, -2, -3, -4, -5, -6, -7, -8
_ERRNAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP", EZEROROW: "EZEROROW", ERANK: "ERANK",
             ENOCONV: "ENOCONV", ENAN: "ENAN", ESTAG: "ESTAG"}
# statuses of a solve that ended without meeting a tolerance but left a valid x
NOT_CONVERGED = (ENOCONV, ESTAG)

if not os.path.exists(LIBPATH):
    raise ImportError(f"{LIBPATH} is missing: build the HIP library first (__graft_entry__.build())")


class _CSR(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p)]


class _Pattern(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("build_T", C.c_int), ("keep_fp64_M", C.c_int), ("scale", C.c_int), ("u_f", C.c_int)]


class _Tol(C.Structure):
    _fields_ = [("u_g", C.c_int), ("ur_dd", C.c_int), ("tau", C.c_double), ("tol_rr", C.c_double),
                ("tol_be", C.c_double), ("i_max", C.c_int), ("gmres_max", C.c_int), ("x0_mode", C.c_int),
                ("trans", C.c_int), ("stag_ratio", C.c_double), ("orth", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("steps", C.c_int), ("its_total", C.c_int), ("stop_reason", C.c_int), ("status", C.c_int),
                ("its", C.c_int * 64), ("eta", C.c_double * 65), ("relres", C.c_double * 65)]


class _BStats(C.Structure):
    _fields_ = [("n", C.c_int32), ("q", C.c_int32), ("nnz", C.c_int64), ("precs", C.c_int * 6),
                ("count", C.c_int64 * 6), ("threshold", C.c_double * 6), ("scale", C.c_double * 6),
                ("norm_inf", C.c_double), ("eps_b", C.c_double), ("bytes_values", C.c_int64),
                ("bytes_indices", C.c_int64), ("storage_pct", C.c_double), ("ell_width", C.c_int32 * 6),
                ("col_bytes", C.c_int32 * 6), ("apply_kind", C.c_int32 * 2)]


class _System(C.Structure):
    _fields_ = [("A", _CSR), ("b", C.c_void_p), ("x", C.c_void_p), ("M", C.c_void_p)]


_lib = C.CDLL(LIBPATH)
_vp = C.c_void_p
_lib.bspai_build.argtypes = [C.POINTER(_CSR), C.POINTER(_Pattern), C.c_double, C.POINTER(C.c_int), C.c_int,
                             C.POINTER(_Opts), C.POINTER(_vp), _vp]
_lib.bspai_import.argtypes = [C.POINTER(_CSR), C.c_double, C.POINTER(C.c_int), C.c_int, C.POINTER(_Opts),
                              C.POINTER(_vp), _vp]
_lib.bspai_apply.argtypes = [_vp, _vp, _vp, C.c_int, C.c_int64, C.c_int, _vp]
_lib.bspai_apply_T.argtypes = [_vp, _vp, _vp, C.c_int, C.c_int64, C.c_int, _vp]
_lib.gmres_ir_solve.argtypes = [C.POINTER(_CSR), _vp, _vp, C.POINTER(_Tol), _vp, C.c_int, C.POINTER(_Stats), _vp]
_lib.gmres_ir_solve_ab.argtypes = [C.POINTER(_CSR), _vp, _vp, _vp, C.POINTER(_Tol), _vp, C.c_int, C.POINTER(_Stats),
                                   _vp]
_lib.bspai_stats.argtypes = [_vp, C.POINTER(_BStats)]
_lib.bspai_export.argtypes = [_vp, _vp, _vp, _vp]
_lib.bspai_free.argtypes = [_vp]
_lib.bspai_free.restype = None
_lib.bspai_last_error.restype = C.c_char_p
_lib.bspai_set_profiling.argtypes = [C.c_int]
_lib.bspai_set_profiling.restype = None
_lib.bspai_last_solve_kernel_ms.restype = C.c_double
_lib.bspai_set_apply_kind.argtypes = [_vp, C.c_int, C.c_int]
_lib.bspai_set_apply_kind.restype = C.c_int
_lib.bspai_tune_apply.argtypes = [_vp, _vp]
_lib.bspai_tune_apply.restype = C.c_int
_lib.bspai_exchange_latency.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_double), _vp]
_lib.bspai_exchange_latency.restype = C.c_int
_lib.bspai_solve_blocks.argtypes = [C.c_int]
_lib.bspai_solve_blocks.restype = C.c_int
_lib.bspai_multi_plan.argtypes = [C.POINTER(_System), C.c_int, C.POINTER(_Tol), C.c_int, C.c_int, C.POINTER(_vp),
                                  _vp]
_lib.bspai_multi_launch.argtypes = [_vp, _vp]
_lib.bspai_multi_poll.argtypes = [_vp]
_lib.bspai_multi_wait.argtypes = [_vp, C.POINTER(_Stats), _vp]
_lib.bspai_multi_group_blocks.argtypes = [_vp]
_lib.bspai_multi_free.argtypes = [_vp]
_lib.bspai_multi_free.restype = None
_lib.bspai_release_workspace.argtypes = []
_lib.bspai_release_workspace.restype = C.c_int
for _f in ("bspai_build", "bspai_import", "bspai_apply", "bspai_apply_T", "gmres_ir_solve", "gmres_ir_solve_ab",
           "bspai_stats",
           "bspai_export", "bspai_multi_plan", "bspai_multi_launch", "bspai_multi_poll", "bspai_multi_wait",
           "bspai_multi_group_blocks"):
    getattr(_lib, _f).restype = C.c_int

SYMBOLS = ("bspai_build", "bspai_import", "bspai_apply", "bspai_apply_T", "gmres_ir_solve", "bspai_stats",
           "bspai_export", "bspai_free", "bspai_last_error", "bspai_grad_vals", "bspai_set_profiling",
           "bspai_last_solve_kernel_ms", "bspai_multi_plan", "bspai_multi_launch", "bspai_multi_poll",
           "bspai_multi_wait", "bspai_multi_free", "bspai_multi_group_blocks", "bspai_exchange_latency",
           "bspai_solve_blocks", "bspai_set_apply_kind", "bspai_tune_apply", "bspai_build_adaptive",
           "bspai_export_pattern", "gmres_ir_solve_ab", "bspai_release_workspace", "gmres_ir_solve_noalloc", "bspai_exchange_latency_placed",
           "bspai_batched_mgs_profile", "bspai_set_batch_mode")


def set_profiling(on: bool) -> None:
    """Time the solver kernel of each gmres_ir_solve with HIP events."""
    _lib.bspai_set_profiling(int(on))


def exchange_latency_us(G: int, iters: int = 20000, stream=None) -> float:
    """Average time of one grid-wide all-reduction of the persistent solver
    with G blocks (bspai_exchange_latency)."""
    out = C.c_double(0.0)
    _check(_lib.bspai_exchange_latency(int(G), int(iters), C.byref(out), _stream(stream)))
    return out.value


_lib.bspai_exchange_latency_placed.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double), _vp, _vp]
_lib.bspai_exchange_latency_placed.restype = C.c_int


def exchange_latency_placed_us(G: int, one_xcd: bool, iters: int = 20000, stream=None):
    """(microseconds per all-reduction, XCD of each participating block) for
    G blocks spread by the dispatcher or kept on one XCD
    (bspai_exchange_latency_placed)."""
    import numpy as np

    out = C.c_double(0.0)
    xcd = np.zeros(G, dtype=np.int32)
    _check(_lib.bspai_exchange_latency_placed(int(G), int(iters), int(one_xcd), C.byref(out),
                                              xcd.ctypes.data_as(C.c_void_p), _stream(stream)))
    return out.value, xcd.tolist()


def solve_blocks(n: int) -> int:
    """Blocks of the persistent solver for n rows (bspai_solve_blocks)."""
    return _check_int(_lib.bspai_solve_blocks(int(n)))


def last_solve_kernel_ms() -> float:
    return _lib.bspai_last_solve_kernel_ms()


_lib.bspai_batched_mgs_profile.argtypes = [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_longlong),
                                           C.POINTER(C.c_double), C.POINTER(C.c_longlong)]
_lib.bspai_batched_mgs_profile.restype = None
_lib.bspai_set_batch_mode.argtypes = [C.c_int]
_lib.bspai_set_batch_mode.restype = C.c_int


def batched_mgs_profile(reset: bool = False) -> Dict:
    """Totals of the one-launch MGS kernel while profiling is on
    (bspai_batched_mgs_profile): ms, launches and algorithmic bytes of the
    timed launches (one in seven), and all_launches."""
    ms, n, by, al = C.c_double(0), C.c_longlong(0), C.c_double(0), C.c_longlong(0)
    _lib.bspai_batched_mgs_profile(int(reset), C.byref(ms), C.byref(n), C.byref(by), C.byref(al))
    return dict(ms=ms.value, launches=n.value, bytes=by.value, all_launches=al.value)


BATCH_AUTO, BATCH_ALL_COLUMNS, BATCH_GROUPS = 0, 1, 2


def set_batch_mode(mode: int) -> None:
    """How solves with several right-hand sides run their columns
    (bspai_set_batch_mode): 0 automatic, 1 all columns in each pass kernel,
    2 column groups with the one-launch MGS."""
    _check(_lib.bspai_set_batch_mode(int(mode)))


class BSPAIError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


def _check(code: int, allow=()):
    if code != OK and code not in allow:
        raise BSPAIError(code, _lib.bspai_last_error().decode(errors="replace"))
    return code


def _check_int(value: int) -> int:
    """Calls that return a count on success and a negative status on failure."""
    if value < 0:
        raise BSPAIError(value, _lib.bspai_last_error().decode(errors="replace"))
    return value


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _prec_ids(precs: Sequence) -> Tuple:
    ids = [PREC[p] if isinstance(p, str) else int(p) for p in precs]
    return (C.c_int * len(ids))(*ids), len(ids)


class CSRMatrix:
    """Square CSR matrix on the GPU: int32 row_ptr/col, float64 values."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, val: Optional[torch.Tensor], n: int):
        self.row_ptr = row_ptr.to(dtype=torch.int32).contiguous()
        self.col = col.to(dtype=torch.int32).contiguous()
        self.val = None if val is None else val.to(dtype=torch.float64).contiguous()
        self.n = int(n)
        for t in (self.row_ptr, self.col) + (() if self.val is None else (self.val,)):
            if not t.is_cuda:
                raise ValueError("CSRMatrix tensors must live on the GPU")

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @classmethod
    def from_host(cls, A, device="cuda") -> "CSRMatrix":
        """From any object with n, row_ptr, col, val NumPy arrays (e.g. workloads.CSR)."""
        val = None if A.val is None else torch.as_tensor(A.val, dtype=torch.float64, device=device)
        return cls(torch.as_tensor(A.row_ptr, device=device), torch.as_tensor(A.col, device=device), val, A.n)

    def _c(self) -> _CSR:
        return _CSR(self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                    self.val.data_ptr() if self.val is not None else None)

    def _p(self) -> _Pattern:
        return _Pattern(self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr())


class Handle:
    """Owns a ``bspai_handle`` (bucketed M on the GPU)."""

    def __init__(self, ptr: int, n: int, nnz: int):
        self._ptr = ptr
        self.n = n
        self.nnz = nnz

    @property
    def ptr(self) -> int:
        if not self._ptr:
            raise ValueError("handle already freed")
        return self._ptr

    def free(self):
        if self._ptr:
            _lib.bspai_free(self._ptr)
            self._ptr = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # during interpreter shutdown the HIP runtime may already be torn
        # down: free nothing then (call free() before exiting instead); the
        # check is bound at definition, as module globals may be gone by then
        if _finalizing():
            return
        try:
            self.free()
        except Exception:
            pass

    def stats(self) -> Dict:
        s = _BStats()
        _check(_lib.bspai_stats(self.ptr, C.byref(s)))
        q = s.q
        return dict(n=s.n, q=q, nnz=s.nnz, precs=list(s.precs[:q]), count=list(s.count[:q]),
                    threshold=list(s.threshold[:q]), scale=list(s.scale[:q]), norm_inf=s.norm_inf, eps_b=s.eps_b,
                    bytes_values=s.bytes_values, bytes_indices=s.bytes_indices, storage_pct=s.storage_pct,
                    ell_width=list(s.ell_width[:q]), col_bytes=list(s.col_bytes[:q]),
                    apply_kind=list(s.apply_kind))

    def export_pattern(self):
        """M's CSR pattern (row_ptr, col) as numpy int32 arrays."""
        import numpy as np

        rp = np.zeros(self.n + 1, dtype=np.int32)
        col = np.zeros(max(self.nnz, 1), dtype=np.int32)
        _check(_lib.bspai_export_pattern(self.ptr, rp.ctypes.data_as(C.c_void_p), col.ctypes.data_as(C.c_void_p)))
        return rp, col[: self.nnz]

    def set_apply_kind(self, kind: int, trans: bool = False) -> None:
        """Kernel of apply (trans False) or apply_T: 0 automatic, 1 padded
        copies, 2 LDS tiles, 3 two rows per thread, 4 lanes per row,
        5 entry-balanced tiles (long rows summed by a wavefront)."""
        _check(_lib.bspai_set_apply_kind(self.ptr, int(trans), int(kind)))

    def tune_apply(self, stream=None) -> None:
        """Time every available apply kernel and keep the fastest."""
        _check(_lib.bspai_tune_apply(self.ptr, _stream(stream)))

    def export(self, fp64: bool = True) -> Dict:
        import numpy as np

        bk = np.zeros(self.nnz, dtype=np.int8)
        st = np.zeros(self.nnz, dtype=np.float64)
        m64 = np.zeros(self.nnz, dtype=np.float64) if fp64 else None
        _check(_lib.bspai_export(self.ptr, bk.ctypes.data, st.ctypes.data,
                                 m64.ctypes.data if m64 is not None else None))
        return dict(bucket=bk, stored=st, m64=m64)


def _opts(build_T, keep_fp64_M, scale, u_f="fp64"):
    if u_f not in ("fp64", "fp32", "fp16"):
        raise ValueError("u_f must be 'fp64', 'fp32' or 'fp16'")
    return _Opts(int(build_T), int(keep_fp64_M), int(scale), PREC[u_f])


def build(A: CSRMatrix, P: Optional[CSRMatrix] = None, eps: float = 1e-4, precs: Sequence = ("fp64",),
          build_T: bool = True, keep_fp64_M: bool = True, scale: bool = False, u_f: str = "fp64",
          stream=None) -> Handle:
    """SPAI of A on the pattern P (None: A's), bucketed (bspai_build).  u_f:
    precision of the least squares ("fp64", "fp32" or "fp16"; use scale=True
    below fp64)."""
    out = _vp()
    pids, q = _prec_ids(precs)
    a = A._c()
    p = P._p() if P is not None else None
    _check(_lib.bspai_build(C.byref(a), C.byref(p) if p is not None else None, float(eps), pids, q,
                            C.byref(_opts(build_T, keep_fp64_M, scale, u_f)), C.byref(out), _stream(stream)))
    return Handle(out.value, A.n, P.nnz if P is not None else A.nnz)


class _AdOpts(C.Structure):
    _fields_ = [("alpha", C.c_int), ("beta", C.c_int), ("eps", C.c_double)]


_lib.bspai_build_adaptive.argtypes = [C.POINTER(_CSR), C.POINTER(_Pattern), C.POINTER(_AdOpts), C.c_double,
                                      C.POINTER(C.c_int), C.c_int, C.POINTER(_Opts), C.POINTER(_vp), _vp, _vp]
_lib.bspai_build_adaptive.restype = C.c_int
_lib.bspai_export_pattern.argtypes = [_vp, _vp, _vp]
_lib.bspai_export_pattern.restype = C.c_int


def build_adaptive(A: CSRMatrix, J0: Optional[CSRMatrix] = None, alpha: int = 5, beta: int = 8,
                   eps_spai: float = 0.4, eps: float = 1e-4, precs: Sequence = ("fp64",), build_T: bool = True,
                   keep_fp64_M: bool = True, u_f: str = "fp64", scale: bool = False, stream=None):
    """SPAI with Algorithm 1's augmentation loop (bspai_build_adaptive), then
    bucketing.  J0 None: identity start.  u_f: precision of the least squares
    solves ("fp64", "fp32", "fp16"; use scale=True below fp64).  Returns
    (Handle, steps per row)."""
    import numpy as np

    ids, q = _prec_ids(precs)
    o = _opts(build_T, keep_fp64_M, scale, u_f)
    ad = _AdOpts(int(alpha), int(beta), float(eps_spai))
    out = _vp()
    steps = np.zeros(A.n, dtype=np.int32)
    a = A._c()
    p = J0._p() if J0 is not None else None
    _check(_lib.bspai_build_adaptive(C.byref(a), C.byref(p) if p is not None else None, C.byref(ad), float(eps),
                                     ids, q, C.byref(o), C.byref(out), steps.ctypes.data_as(C.c_void_p),
                                     _stream(stream)))
    st = _BStats()
    _check(_lib.bspai_stats(out.value, C.byref(st)))
    return Handle(out.value, A.n, st.nnz), steps


def import_m(M: CSRMatrix, eps: float, precs: Sequence, build_T: bool = True, keep_fp64_M: bool = True,
             stream=None) -> Handle:
    out = _vp()
    pids, q = _prec_ids(precs)
    m = M._c()
    _check(_lib.bspai_import(C.byref(m), float(eps), pids, q, C.byref(_opts(build_T, keep_fp64_M, False)),
                             C.byref(out), _stream(stream)))
    return Handle(out.value, M.n, M.nnz)


def bucket_a(A: CSRMatrix, eps: float, precs: Sequence, build_T: bool = False, keep_fp64: bool = False,
             stream=None) -> Handle:
    """A split into buckets by Algorithm 2's rule (thresholds fl(eps ||A||_inf)
    / u_k), for the GMRES products of :func:`solve` (``A_b``); build_T for the
    adjoint (trans) solve; keep_fp64 keeps a copy of A's FP64 values (needed
    by Handle.export only)."""
    return import_m(A, eps, precs, build_T=build_T, keep_fp64_M=keep_fp64, stream=stream)


def _apply(fn, h: Handle, x: torch.Tensor, out: Optional[torch.Tensor], stream):
    if x.dtype not in (torch.float32, torch.float64) or not x.is_cuda:
        raise ValueError("x must be a float32/float64 CUDA tensor")
    x = x.contiguous()
    nrhs = 1 if x.dim() == 1 else x.shape[1]
    if x.shape[0] != h.n:
        raise ValueError(f"x has {x.shape[0]} rows, M is {h.n} x {h.n}")
    y = torch.empty_like(x) if out is None else out
    _check(fn(h.ptr, x.data_ptr(), y.data_ptr(), nrhs, nrhs, FP64 if x.dtype == torch.float64 else FP32,
              _stream(stream)))
    return y


def apply(h: Handle, x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """y = M_b x (x: [n] or [n, nrhs] float32/float64 on the GPU)."""
    return _apply(_lib.bspai_apply, h, x, out, stream)


def apply_T(h: Handle, x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """y = M_b^T x."""
    return _apply(_lib.bspai_apply_T, h, x, out, stream)


def _stats_dict(s: _Stats) -> Dict:
    k = s.steps
    return dict(steps=k, its=list(s.its[:k]), its_total=s.its_total, eta=list(s.eta[:k + 1]),
                relres=list(s.relres[:k + 1]), stop_reason=s.stop_reason, status=s.status)


def _stag(r: Optional[float]) -> float:
    """stag_ratio for the C struct: None switches the stagnation stop off."""
    if r is None:
        return -1.0
    if r <= 0:
        raise ValueError("stag_ratio must be positive (None: no stagnation stop)")
    return float(r)


def solve(A: CSRMatrix, b: torch.Tensor, h: Handle, u_g: str = "fp32", ur_dd: bool = True, tau: float = 1e-4,
          tol_rr: float = 1e-10, tol_be: float = 0.0, i_max: int = 20, gmres_max: int = 150, x0_mode: int = 0,
          trans: bool = False, x: Optional[torch.Tensor] = None, stream=None, raise_noconv: bool = False,
          stag_ratio: Optional[float] = 0.5, A_b: Optional[Handle] = None, orth: str = "mgs"):
    """BSPAI-GMRES-IR.  b: [n] or [n, nrhs] (1 <= nrhs <= 64, row-major)
    float64 on the GPU.  Returns (x, stats): one stats dict for a 1-D b, a
    list of them (one per column) for a 2-D b.  A solve that met neither
    tolerance (ENOCONV: i_max reached; ESTAG: the corrections stagnated
    first) is reported in the stats' status unless raise_noconv, which
    raises BSPAIError instead.  stag_ratio: stop when a correction's
    ||d||/||x|| exceeds stag_ratio times the previous one (None: never).
    A_b: A bucketed (:func:`bucket_a`) for the products inside GMRES
    (``gmres_ir_solve_ab``); None: A rounded to u_g.  orth: "mgs" (the
    paper's modified Gram-Schmidt) or "cgs2" (classical Gram-Schmidt twice,
    two grid-wide reductions per Arnoldi step; one right-hand side)."""
    if b.dtype != torch.float64 or not b.is_cuda or b.dim() not in (1, 2):
        raise ValueError("b must be a 1-D or 2-D float64 CUDA tensor")
    b = b.contiguous()
    nrhs = 1 if b.dim() == 1 else b.shape[1]
    if not 1 <= nrhs <= 64:
        raise ValueError("b must have between 1 and 64 columns")
    if x is None:
        x = torch.zeros_like(b) if x0_mode == 3 else torch.empty_like(b)
    elif x.shape != b.shape or x.dtype != torch.float64 or not x.is_contiguous():
        raise ValueError("x must be a contiguous float64 tensor shaped like b")
    if orth not in ("mgs", "cgs2"):
        raise ValueError("orth must be 'mgs' or 'cgs2'")
    tol = _Tol(PREC[u_g], int(ur_dd), float(tau), float(tol_rr), float(tol_be), int(i_max), int(gmres_max),
               int(x0_mode), int(trans), _stag(stag_ratio), 0 if orth == "mgs" else 1)
    st = (_Stats * nrhs)()
    a = A._c()
    allow = () if raise_noconv else NOT_CONVERGED
    if A_b is None:
        rc = _lib.gmres_ir_solve(C.byref(a), b.data_ptr(), h.ptr, C.byref(tol), x.data_ptr(), nrhs, st,
                                 _stream(stream))
    else:
        rc = _lib.gmres_ir_solve_ab(C.byref(a), A_b.ptr, b.data_ptr(), h.ptr, C.byref(tol), x.data_ptr(), nrhs, st,
                                    _stream(stream))
    _check(rc, allow=allow)
    if b.dim() == 1:
        return x, _stats_dict(st[0])
    return x, [_stats_dict(q) for q in st]


_lib.gmres_ir_solve_noalloc.argtypes = [C.POINTER(_CSR), _vp, _vp, C.POINTER(_Tol), _vp, C.POINTER(_Stats), _vp]
_lib.gmres_ir_solve_noalloc.restype = C.c_int


def solve_noalloc(A: CSRMatrix, b: torch.Tensor, h: Handle, x: torch.Tensor, u_g: str = "fp32", ur_dd: bool = True,
                  tau: float = 1e-4, tol_rr: float = 1e-10, tol_be: float = 0.0, i_max: int = 20,
                  gmres_max: int = 150, x0_mode: int = 0, stream=None, raise_noconv: bool = False,
                  stag_ratio: Optional[float] = 0.5, orth: str = "mgs") -> Dict:
    """gmres_ir_solve_noalloc: one right-hand side, workspace in the library's
    static device scratch (nothing allocated by the library).  b, x: 1-D
    float64 CUDA tensors of length n; x is written (and read for x0_mode 3).
    Returns the stats dict."""
    if b.dtype != torch.float64 or not b.is_cuda or b.dim() != 1 or not b.is_contiguous():
        raise ValueError("b must be a contiguous 1-D float64 CUDA tensor")
    if x.shape != b.shape or x.dtype != torch.float64 or not x.is_contiguous():
        raise ValueError("x must be a contiguous float64 tensor shaped like b")
    if orth not in ("mgs", "cgs2"):
        raise ValueError("orth must be 'mgs' or 'cgs2'")
    tol = _Tol(PREC[u_g], int(ur_dd), float(tau), float(tol_rr), float(tol_be), int(i_max), int(gmres_max),
               int(x0_mode), 0, _stag(stag_ratio), 0 if orth == "mgs" else 1)
    st = _Stats()
    a = A._c()
    rc = _lib.gmres_ir_solve_noalloc(C.byref(a), b.data_ptr(), h.ptr, C.byref(tol), x.data_ptr(), C.byref(st),
                                     _stream(stream))
    _check(rc, allow=() if raise_noconv else NOT_CONVERGED)
    return _stats_dict(st)


class MultiPlan:
    """Independent systems solved in one persistent launch replayed from a
    captured HIP graph (``bspai_multi_*``).  ``systems``: list of
    (CSRMatrix A, b tensor, Handle M[, x tensor]); b and x are 1-D float64
    CUDA tensors that the plan keeps referenced (each launch reads b and
    writes x).  group_blocks: blocks per group (0 automatic, -1 autotuned by
    timing one launch per candidate size).  orth: "mgs" or "cgs2", as in
    :func:`solve`."""

    def __init__(self, systems, u_g: str = "fp32", ur_dd: bool = True, tau: float = 1e-4, tol_rr: float = 1e-10,
                 tol_be: float = 0.0, i_max: int = 20, gmres_max: int = 150, x0_mode: int = 0, trans: bool = False,
                 group_blocks: int = 0, max_groups: int = 0, stream=None, stag_ratio: Optional[float] = 0.5,
                 orth: str = "mgs"):
        self._ptr = None
        self.A, self.b, self.x, self.M = [], [], [], []
        arr = (_System * len(systems))()
        for k, item in enumerate(systems):
            A, b, M = item[0], item[1], item[2]
            x = item[3] if len(item) > 3 else None
            if b.dtype != torch.float64 or not b.is_cuda or b.dim() != 1 or b.shape[0] != A.n:
                raise ValueError("each b must be a 1-D float64 CUDA tensor of length n")
            b = b.contiguous()
            if x is None:
                x = torch.zeros_like(b)
            self.A.append(A), self.b.append(b), self.x.append(x), self.M.append(M)
            arr[k].A = A._c()
            arr[k].b = b.data_ptr()
            arr[k].x = x.data_ptr()
            arr[k].M = M.ptr
        if orth not in ("mgs", "cgs2"):
            raise ValueError("orth must be 'mgs' or 'cgs2'")
        self.tol = _Tol(PREC[u_g], int(ur_dd), float(tau), float(tol_rr), float(tol_be), int(i_max),
                        int(gmres_max), int(x0_mode), int(trans), _stag(stag_ratio), 0 if orth == "mgs" else 1)
        out = _vp()
        _check(_lib.bspai_multi_plan(arr, len(systems), C.byref(self.tol), int(group_blocks), int(max_groups),
                                     C.byref(out), _stream(stream)))
        self._ptr = out.value
        self.nsys = len(systems)
        self.group_blocks = _lib.bspai_multi_group_blocks(self._ptr)

    def launch(self, stream=None) -> None:
        _check(_lib.bspai_multi_launch(self._ptr, _stream(stream)))

    def poll(self) -> bool:
        return bool(_lib.bspai_multi_poll(self._ptr))

    def wait(self, stream=None, raise_noconv: bool = False) -> List[Dict]:
        st = (_Stats * self.nsys)()
        allow = () if raise_noconv else NOT_CONVERGED
        _check(_lib.bspai_multi_wait(self._ptr, st, _stream(stream)), allow=allow)
        return [_stats_dict(q) for q in st]

    def free(self) -> None:
        if self._ptr:
            _lib.bspai_multi_free(self._ptr)
            self._ptr = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


def release_workspace() -> None:
    """Free the solvers' cached device workspaces, single-system and column
    groups (bspai_release_workspace); the next solve allocates them again."""
    _check(_lib.bspai_release_workspace())


from .autograd import BSPAISolve  # noqa: E402  (needs the names above)

__all__ = ["CSRMatrix", "Handle", "build", "build_adaptive", "import_m", "apply", "apply_T", "solve", "MultiPlan",
           "BSPAISolve", "BSPAIError", "SYMBOLS", "PREC", "release_workspace", "NOT_CONVERGED", "solve_noalloc"]

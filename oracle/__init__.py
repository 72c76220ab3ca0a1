"""CPU oracle for BSPAI-GMRES-IR — TEST INFRASTRUCTURE.

A plain, slow, obviously-correct reference for the method of Khan & Carson
(arXiv 2307.03914), written in C (``oracle.c``) and wrapped here with ctypes and
NumPy.  Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package; the product path never does.  It
shares no code with the HIP implementation.

Parity status per function (the pins live in ``tests/test_oracle_*.py``):

* ``round_to`` / ``encode`` / ``decode``  pinned: exhaustive code round trips,
  NumPy float16/float32 and torch bfloat16/float8_e4m3fn casts, hand-made ties.
* ``householder_ls`` / ``spai``  pinned: NumPy ``lstsq``, full pattern gives the
  dense inverse, diagonal and block-diagonal closed forms, LS optimality.  In
  a lower u_f: Householder's backward-stability and forward-error bounds,
  rounding placement against IEEE float16/float32 scalars, fp16 overflow
  without Section 4's scaling.
* ``bucketize``  pinned: hand-computed bucket ids at the interval ends of
  eq. (nint), invariants (counts, monotonicity in eps, limits).
* ``storage_pct``  pinned: the "str." column of Tables 3 and 4.
* ``apply`` / ``apply_T`` / ``apply_paper``  pinned: exact rational products,
  the error bound of Theorem 3.1 as quoted in Section 2.3.
* ``residual``  pinned: exact rational residual (double-double error bound).
* ``gmres`` / ``gmres_ir``  pinned: termination in <= n steps, Arnoldi relation,
  closed-form spectra, dense solves, backward error reaching O(u).  Their
  bucketed-A option (``Ab``): a one-bucket A_b reproduces the u_p path bit for
  bit, the first Arnoldi step by hand, the per-row product bound.  Their
  CGS2 option (``orth``): Arnoldi relation, full orthogonality where MGS
  loses it, Krylov termination facts, the first fp32 step by hand.
* ``gradient``  pinned: dense ``numpy.linalg.solve`` adjoint and finite differences.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liboracle.so")

FP64, FP32, FP16, BF16, FP8, DROP = 0, 1, 2, 3, 4, 5
OK, EINVAL, ENOMEM, EZEROROW, ERANK, ENOCONV, ENAN, ESTAG = 0, -1, -2, -4, -5, -6, -7, -8

_lib = None

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")


class GmresOpts(C.Structure):
    _fields_ = [("ug", C.c_int), ("up", C.c_int), ("tau", C.c_double), ("max_it", C.c_int), ("trans", C.c_int),
                ("dot64", C.c_int), ("arp_b", C.c_void_p), ("aci_b", C.c_void_p), ("at_b", C.c_void_p),
                ("ab_b", C.c_void_p), ("qa", C.c_int), ("orth", C.c_int)]


class IROpts(C.Structure):
    _fields_ = [("ug", C.c_int), ("up", C.c_int), ("ur_dd", C.c_int), ("tau", C.c_double),
                ("tol_rr", C.c_double), ("tol_be", C.c_double), ("i_max", C.c_int),
                ("gmres_max", C.c_int), ("x0_mode", C.c_int), ("trans", C.c_int), ("dot64", C.c_int),
                ("stag", C.c_double), ("arp_b", C.c_void_p), ("aci_b", C.c_void_p), ("at_b", C.c_void_p),
                ("ab_b", C.c_void_p), ("qa", C.c_int), ("orth", C.c_int)]


class IRStats(C.Structure):
    _fields_ = [("steps", C.c_int), ("its_total", C.c_int), ("stop_reason", C.c_int), ("pad", C.c_int),
                ("its", C.c_int * 64), ("eta", C.c_double * 65), ("relres", C.c_double * 65)]


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH) or os.path.getmtime(LIBPATH) < os.path.getmtime(os.path.join(HERE, "oracle.c")):
        from . import build as _b
        _b.build()
    L = C.CDLL(LIBPATH)
    L.orc_num_threads.argtypes = [C.c_int]
    L.orc_num_threads.restype = C.c_int
    L.orc_unit_roundoff.argtypes = [C.c_int]
    L.orc_unit_roundoff.restype = C.c_double
    L.orc_round.argtypes = [C.c_int, C.c_double]
    L.orc_round.restype = C.c_double
    L.orc_round_array.argtypes = [C.c_int, C.c_int64, _f64p, _f64p]
    L.orc_encode_array.argtypes = [C.c_int, C.c_int64, _f64p, _u32p]
    L.orc_decode_array.argtypes = [C.c_int, C.c_int64, _u32p, _f64p]
    L.orc_storage_pct.argtypes = [_i64p, _i32p, C.c_int, C.c_double, C.c_int]
    L.orc_storage_pct.restype = C.c_double
    L.orc_householder_ls.argtypes = [C.c_int, C.c_int, _f64p, _f64p, _f64p]
    L.orc_householder_ls_prec.argtypes = [C.c_int, C.c_int, _f64p, _f64p, _f64p, C.c_int]
    L.orc_spai_prec.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, C.c_void_p, C.c_int, C.c_int,
                                C.c_int, C.POINTER(C.c_int)]
    L.orc_spai.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, C.c_void_p, C.c_int, C.c_int,
                           C.POINTER(C.c_int)]
    L.orc_spai_adaptive.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, C.c_void_p, C.c_void_p, C.c_int,
                                    C.c_int, C.c_double, C.c_int, _i32p, _i32p, _f64p, _i32p, C.POINTER(C.c_int)]
    L.orc_spai_adaptive_prec.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, C.c_void_p, C.c_void_p,
                                         C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, _i32p, _i32p,
                                         _f64p, _i32p, C.POINTER(C.c_int)]
    L.orc_norm_inf.argtypes = [C.c_int, _i32p, _f64p]
    L.orc_norm_inf.restype = C.c_double
    L.orc_bucketize.argtypes = [C.c_int, _i32p, _f64p, C.c_double, _i32p, C.c_int, _i8p, _f64p, _f64p, _f64p, _i64p]
    L.orc_apply.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i8p, C.c_int, _f64p, _f64p, C.c_int]
    L.orc_apply_paper.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i8p, _i32p, C.c_int, _f64p, _f64p]
    L.orc_transpose.argtypes = [C.c_int, _i32p, _i32p, C.c_void_p, C.c_void_p, _i32p, _i32p, C.c_void_p, C.c_void_p]
    L.orc_spmv.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, _f64p, _f64p, C.c_int]
    L.orc_residual.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, C.c_int]
    L.orc_gmres.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _i8p, C.c_int, _f64p, _f64p,
                            C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(GmresOpts), C.c_void_p, C.c_void_p]
    L.orc_gmres_ir.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _i8p,
                               C.c_int, _f64p, _f64p, C.POINTER(IROpts), C.POINTER(IRStats)]
    _lib = L
    return L


def num_threads(req: int = 0) -> int:
    return lib().orc_num_threads(req)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------- formats

def unit_roundoff(prec: int) -> float:
    return lib().orc_unit_roundoff(prec)


def round_to(prec: int, x) -> np.ndarray:
    x = _f64(np.atleast_1d(x))
    y = np.empty_like(x)
    lib().orc_round_array(prec, x.size, x, y)
    return y


def encode(prec: int, x) -> np.ndarray:
    x = _f64(np.atleast_1d(x))
    c = np.empty(x.size, dtype=np.uint32)
    lib().orc_encode_array(prec, x.size, x, c)
    return c


def decode(prec: int, codes) -> np.ndarray:
    c = np.ascontiguousarray(np.atleast_1d(codes), dtype=np.uint32)
    x = np.empty(c.size, dtype=np.float64)
    lib().orc_decode_array(prec, c.size, c, x)
    return x


def storage_pct(counts: Sequence[int], precs: Sequence[int], drop_bytes: float = 0.0,
                with_index: bool = False) -> float:
    c = np.ascontiguousarray(counts, dtype=np.int64)
    p = _i32(precs)
    return lib().orc_storage_pct(c, p, len(p), float(drop_bytes), int(with_index))


# ---------------------------------------------------------------- SPAI

def householder_ls(A: np.ndarray, b: np.ndarray, prec: int = FP64):
    """(status, x) for min ||b - A x||_2 (dense, m >= n); prec: every
    operation rounded to that precision (A and b must hold its numbers)."""
    A = np.asfortranarray(A, dtype=np.float64)
    m, n = A.shape
    a = _f64(A.reshape(-1, order="F"))
    bb = _f64(b).copy()
    x = np.zeros(n)
    if prec == FP64:
        st = lib().orc_householder_ls(m, n, a, bb, x)
    else:
        st = lib().orc_householder_ls_prec(m, n, a, bb, x, int(prec))
    return st, x


def spai(A, P, rows: Optional[np.ndarray] = None, scale: bool = False, uf: int = FP64):
    """(status, M values on P's CSR, bad_row).  A, P: workloads.CSR.  uf: the
    construction precision u_f (FP64, FP32 or FP16)."""
    Mv = np.zeros(P.nnz, dtype=np.float64)
    bad = C.c_int(-1)
    if rows is not None:
        rr = _i32(rows)
        rptr, nr = rr.ctypes.data_as(C.c_void_p), rr.size
    else:
        rr, rptr, nr = None, None, 0
    st = lib().orc_spai_prec(A.n, _i32(A.row_ptr), _i32(A.col), _f64(A.val), _i32(P.row_ptr), _i32(P.col), Mv,
                             rptr, nr, int(scale), int(uf), C.byref(bad))
    return st, Mv, bad.value


def spai_adaptive(A, alpha: int = 5, beta: int = 8, eps: float = 0.4, J0=None, uf: int = FP64,
                  scale: bool = False) -> Dict:
    """Adaptive SPAI (Algorithm 1 with augmentation, on A^T).  J0: initial
    pattern (workloads.CSR; None: the identity).  uf: precision of the least
    squares solves, scale: column scaling of A^T (as :func:`spai`).  Returns
    dict(status, M (workloads.CSR with each row's columns ascending), steps
    (solves per row), bad_row)."""
    import workloads as W
    n = A.n
    AT = transpose_csr(A)
    j0max = 1 if J0 is None else int(np.diff(J0.row_ptr).max(initial=0))
    jmax = max(1, j0max + alpha * beta)
    cnt = np.zeros(n, dtype=np.int32)
    cols = np.zeros(n * jmax, dtype=np.int32)
    vals = np.zeros(n * jmax)
    steps = np.zeros(n, dtype=np.int32)
    bad = C.c_int(-1)
    keep = []
    if J0 is not None:
        jr, jc = _i32(J0.row_ptr), _i32(J0.col)
        keep = [jr, jc]
        jrp, jcp = jr.ctypes.data_as(C.c_void_p), jc.ctypes.data_as(C.c_void_p)
    else:
        jrp = jcp = None
    st = lib().orc_spai_adaptive_prec(n, _i32(A.row_ptr), _i32(A.col), _f64(A.val), _i32(AT.row_ptr),
                                      _i32(AT.col), jrp, jcp, int(alpha), int(beta), float(eps), int(jmax),
                                      int(scale), int(uf), cnt, cols, vals, steps, C.byref(bad))
    del keep
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(cnt)
    sel = (np.arange(jmax)[None, :] < cnt[:, None]).reshape(-1)
    M = W.CSR(n, rp, cols[sel].astype(np.int32), vals[sel])
    return dict(status=st, M=M, steps=steps, bad_row=bad.value)


def norm_inf(M) -> float:
    return lib().orc_norm_inf(M.n, _i32(M.row_ptr), _f64(M.val))


# ---------------------------------------------------------------- buckets

class Bucketed:
    """Bucketed M: CSR structure + per-entry bucket id and stored value."""

    def __init__(self, M, eps: float, precs: Sequence[int]):
        self.n = M.n
        self.row_ptr = _i32(M.row_ptr)
        self.col = _i32(M.col)
        self.val = _f64(M.val)
        self.precs = _i32(precs)
        self.q = len(precs)
        self.eps = float(eps)
        nnz = M.nnz
        self.bucket = np.zeros(nnz, dtype=np.int8)
        self.mt = np.zeros(nnz, dtype=np.float64)
        self.t = np.zeros(self.q)
        self.s = np.zeros(self.q)
        self.counts = np.zeros(self.q, dtype=np.int64)
        st = lib().orc_bucketize(M.n, self.row_ptr, self.val, self.eps, self.precs, self.q, self.bucket,
                                 self.mt, self.t, self.s, self.counts)
        if st != OK:
            raise ValueError(f"orc_bucketize failed: {st}")
        self.normM = norm_inf(M)

    def transpose(self) -> "Bucketed":
        T = object.__new__(Bucketed)
        n, nnz = self.n, int(self.row_ptr[-1])
        T.n, T.precs, T.q, T.eps, T.t, T.s, T.counts, T.normM = (self.n, self.precs, self.q, self.eps, self.t,
                                                                 self.s, self.counts, self.normM)
        T.row_ptr = np.zeros(n + 1, dtype=np.int32)
        T.col = np.zeros(nnz, dtype=np.int32)
        T.val = np.zeros(nnz)
        T.mt = np.zeros(nnz)
        T.bucket = np.zeros(nnz, dtype=np.int8)
        _transpose(n, self.row_ptr, self.col, self.val, T.row_ptr, T.col, T.val)
        _transpose(n, self.row_ptr, self.col, self.mt, T.row_ptr, T.col, T.mt)
        L = lib()
        L.orc_transpose(n, self.row_ptr, self.col, None, self.bucket.ctypes.data_as(C.c_void_p), T.row_ptr,
                        T.col, None, T.bucket.ctypes.data_as(C.c_void_p))
        return T

    def storage_pct(self, drop_bytes=0.0, with_index=False):
        return storage_pct(self.counts, self.precs, drop_bytes, with_index)


def _transpose(n, rp, ci, v, trp, tci, tv):
    lib().orc_transpose(n, rp, ci, v.ctypes.data_as(C.c_void_p), None, trp, tci, tv.ctypes.data_as(C.c_void_p),
                        None)


def transpose_csr(A):
    """CSR of A^T (values kept)."""
    import workloads as W
    n, nnz = A.n, A.nnz
    trp = np.zeros(n + 1, dtype=np.int32)
    tci = np.zeros(nnz, dtype=np.int32)
    tv = np.zeros(nnz)
    _transpose(n, _i32(A.row_ptr), _i32(A.col), _f64(A.val), trp, tci, tv)
    return W.CSR(n, trp, tci, tv)


def apply(Mb: Bucketed, x, out_prec: int = FP64) -> np.ndarray:
    x = _f64(x)
    y = np.zeros(Mb.n)
    lib().orc_apply(Mb.n, Mb.row_ptr, Mb.col, Mb.mt, Mb.bucket, Mb.q, x, y, out_prec)
    return y


def apply_T(Mb: Bucketed, x, out_prec: int = FP64) -> np.ndarray:
    return apply(Mb.transpose(), x, out_prec)


def apply_paper(Mb: Bucketed, x) -> np.ndarray:
    x = _f64(x)
    y = np.zeros(Mb.n)
    lib().orc_apply_paper(Mb.n, Mb.row_ptr, Mb.col, Mb.mt, Mb.bucket, Mb.precs, Mb.q, x, y)
    return y


def spmv(A, x, val_prec: int = FP64, out_prec: int = FP64) -> np.ndarray:
    y = np.zeros(A.n)
    lib().orc_spmv(A.n, _i32(A.row_ptr), _i32(A.col), _f64(A.val), val_prec, _f64(x), y, out_prec)
    return y


def residual(A, b, x, dd: bool = True) -> np.ndarray:
    r = np.zeros(A.n)
    lib().orc_residual(A.n, _i32(A.row_ptr), _i32(A.col), _f64(A.val), _f64(b), _f64(x), r, int(dd))
    return r


def backward_error(A, b, x, dd: bool = True) -> float:
    """eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)."""
    r = residual(A, b, x, dd)
    nA = norm_inf(A)
    return float(np.abs(r).max() / (nA * np.abs(x).max() + np.abs(b).max()))


# ---------------------------------------------------------------- Krylov

def _orth(name: str) -> int:
    if name not in ("mgs", "cgs2"):
        raise ValueError("orth must be 'mgs' or 'cgs2'")
    return 0 if name == "mgs" else 1


def _set_ab(o, Ab, trans):
    """Point the option struct at the bucketed A (A^T when trans); returns the
    object that owns the arrays, to be kept alive over the call."""
    if Ab is None:
        return None
    Aop_b = Ab.transpose() if trans else Ab
    o.arp_b, o.aci_b = Aop_b.row_ptr.ctypes.data, Aop_b.col.ctypes.data
    o.at_b, o.ab_b, o.qa = Aop_b.mt.ctypes.data, Aop_b.bucket.ctypes.data, Aop_b.q
    return Aop_b


def gmres(A, Mb: Bucketed, r, tau: float = 1e-4, ug: int = FP32, up: int = FP32, max_it: Optional[int] = None,
          trans: bool = False, want_basis: bool = False, dot64: bool = False,
          Ab: Optional[Bucketed] = None, orth: str = "mgs") -> Dict:
    """One preconditioned MGS-GMRES solve (left: M A d = M r; trans: A^T M^T).
    dot64: dots and norms accumulated in FP64 over u_g data (the default sums
    sequentially in u_g).  Ab: A applied bucketed (eqs. (nbe2), (fe2)).
    orth: "mgs" (the paper's) or "cgs2" (classical Gram-Schmidt twice)."""
    n = A.n
    m = min(n, max_it if max_it is not None else n)
    o = GmresOpts(ug, up, float(tau), m, int(trans), int(dot64))
    o.orth = _orth(orth)
    Aop_b = _set_ab(o, Ab, trans)
    d = np.zeros(n)
    its = C.c_int(0)
    rel = C.c_double(0)
    V = np.zeros((m + 1) * n) if want_basis else None
    H = np.zeros((m + 1) * m) if want_basis else None
    if trans:
        At = transpose_csr(A)
        Mt = Mb.transpose()
        ops = (At, Mt)
    else:
        ops = (A, Mb)
    Aop, Mop = ops
    st = lib().orc_gmres(n, _i32(Aop.row_ptr), _i32(Aop.col), _f64(Aop.val), Mop.row_ptr, Mop.col, Mop.mt,
                         Mop.bucket, Mop.q, _f64(r), d, C.byref(its), C.byref(rel), C.byref(o),
                         V.ctypes.data_as(C.c_void_p) if V is not None else None,
                         H.ctypes.data_as(C.c_void_p) if H is not None else None)
    out = dict(status=st, d=d, its=its.value, relres=rel.value)
    if want_basis:
        k = its.value
        out["V"] = V.reshape(m + 1, n)[: k + 1].T.copy()
        out["H"] = H.reshape(m, m + 1).T[: k + 1, :k].copy()
    return out


def gmres_ir(A, M, Mb: Bucketed, b, ug: int = FP32, up: int = FP32, ur_dd: bool = True, tau: float = 1e-4,
             tol_rr: float = 1e-10, tol_be: float = 0.0, i_max: int = 20, gmres_max: Optional[int] = None,
             x0_mode: int = 0, trans: bool = False, dot64: bool = False, stag_ratio: Optional[float] = 0.5,
             Ab: Optional["Bucketed"] = None, orth: str = "mgs", x0=None) -> Dict:
    """BSPAI-GMRES-IR (Algorithm 4).  M: FP64 SPAI as workloads.CSR (for x_0).
    dot64 as in :func:`gmres`; stag_ratio None: no stagnation stop; Ab: A
    bucketed (Bucketed of A) to apply A inside GMRES as well (eqs. (nbe2),
    (fe2)); None: A rounded to u_p.  orth: Gram-Schmidt of GMRES ("mgs" or
    "cgs2").  x0: the starting vector for x0_mode 3 (Algorithm 4's x_0 given by
    the caller)."""
    n = A.n
    if (x0 is not None) != (x0_mode == 3):
        raise ValueError("x0 is given exactly when x0_mode is 3")
    gm = min(n, gmres_max if gmres_max is not None else n)
    o = IROpts(ug, up, int(ur_dd), float(tau), float(tol_rr), float(tol_be), int(i_max), gm, int(x0_mode),
               int(trans), int(dot64), -1.0 if stag_ratio is None else float(stag_ratio))
    o.orth = _orth(orth)
    Aop_b = _set_ab(o, Ab, trans)
    st = IRStats()
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    if trans:
        Aop, Fop, Mop = transpose_csr(A), transpose_csr(M), Mb.transpose()
    else:
        Aop, Fop, Mop = A, M, Mb
    status = lib().orc_gmres_ir(n, _i32(Aop.row_ptr), _i32(Aop.col), _f64(Aop.val), _i32(Fop.row_ptr),
                                _i32(Fop.col), _f64(Fop.val), Mop.row_ptr, Mop.col, Mop.mt, Mop.bucket, Mop.q,
                                _f64(b), x, C.byref(o), C.byref(st))
    steps = st.steps
    return dict(status=status, x=x, steps=steps, its=list(st.its[:steps]), its_total=st.its_total,
                eta=list(st.eta[: steps + 1]), relres=list(st.relres[: steps + 1]), stop_reason=st.stop_reason)


def gradient_direct(A, x, g) -> Dict:
    """The adjoint gradient by its plain definition: lambda solves
    A^T lambda = g, here by a sparse LU factorisation (a library step, FP64),
    then dL/db = lambda and dL/da_ij = -lambda_i x_j.  The reference for
    systems too large for the iterative oracle to finish in seconds; the
    preconditioner only changes how lambda is found, not lambda."""
    import scipy.sparse.linalg as spla

    lam = spla.splu(A.to_scipy().T.tocsc()).solve(np.asarray(g, dtype=np.float64))
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    return dict(grad_b=lam, grad_vals=-lam[rows] * np.asarray(x)[A.col])


def gradient(A, M, Mb: Bucketed, x, g, **kw) -> Dict:
    """Adjoint of A x = b: lambda solves A^T lambda = g (transposed IR with M_b^T
    as right preconditioner); dL/db = lambda, dL/da_ij = -lambda_i x_j."""
    res = gmres_ir(A, M, Mb, g, trans=True, **kw)
    lam = res["x"]
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    return dict(grad_b=lam, grad_vals=-lam[rows] * np.asarray(x)[A.col], adjoint=res)

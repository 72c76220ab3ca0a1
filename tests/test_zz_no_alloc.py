"""gmres_ir_solve_noalloc (the solve for callers that cannot allocate) against
gmres_ir_solve, through the C interface: two calls in a row, the second on a
smaller system, each equal bit for bit to the allocating entry point (the
same kernels on the same row split), and a system beyond the scratch limit is
rejected with EINVAL."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _solve_noalloc(B, A, b, h, **kw):
    import torch

    B._lib.gmres_ir_solve_noalloc.argtypes = [C.POINTER(B._CSR), C.c_void_p, C.c_void_p, C.POINTER(B._Tol),
                                             C.c_void_p, C.POINTER(B._Stats), C.c_void_p]
    B._lib.gmres_ir_solve_noalloc.restype = C.c_int
    tol = B._Tol(B.PREC[kw.get("u_g", "fp32")], 1, kw["tau"], kw["tol_rr"], kw.get("tol_be", 0.0), kw["i_max"],
                 kw["gmres_max"], 0, 0, 0.5, 0)
    x = torch.empty_like(b)
    st = B._Stats()
    a = A._c()
    rc = B._lib.gmres_ir_solve_noalloc(C.byref(a), b.data_ptr(), h.ptr, C.byref(tol), x.data_ptr(), C.byref(st),
                                       B._stream(None))
    torch.cuda.synchronize()
    return rc, x, B._stats_dict(st)


def test_noalloc_matches_allocating_solve():
    import torch

    import paper_2307_03914_amd as B

    torch.cuda.set_device(0)
    kw = dict(tau=1e-4, tol_rr=1e-10, gmres_max=150, i_max=20)
    # the larger system first, then a smaller one: the scratch keeps the
    # first call's contents, which the second must not read
    for key in ("2s", "1"):
        small = key.endswith("s")
        c = W.config(key[:-1] if small else key, small=small)
        A, P = c["A"], c["P"]
        print("noalloc", key, "n", A.n, flush=True)
        Ad = B.CSRMatrix.from_host(A)
        h = B.build(Ad, B.CSRMatrix.from_host(P), eps=c["eps"][0], precs=c["precs"])
        b = torch.as_tensor(np.ascontiguousarray(c["b"]), device="cuda")
        x0, st0 = B.solve(Ad, b, h, **kw)
        torch.cuda.synchronize()
        rc, x1, st1 = _solve_noalloc(B, Ad, b, h, **kw)
        assert rc == B.OK, B._lib.bspai_last_error()
        assert st1["stop_reason"] == 1 and st1 == st0
        assert torch.equal(x0, x1)
        h.free()
    # beyond the 64 MiB scratch: the 128^3 operator's basis alone is 1.3 GB
    c = W.config("4a")
    A = c["A"]
    Ad = B.CSRMatrix.from_host(A)
    h = B.build(Ad, B.CSRMatrix.from_host(c["P"]), eps=c["eps"][0], precs=c["precs"])
    b = torch.as_tensor(np.ascontiguousarray(c["b"][:, 0]), device="cuda")
    rc, _, _ = _solve_noalloc(B, Ad, b, h, **kw)
    assert rc == B.EINVAL
    assert b"the limit is" in B._lib.bspai_last_error()
    h.free()

"""The C interface: every function declared in include/bspai.h is exported by
libbspai.so, and argument errors are reported without touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bspai.h")
LIB = os.path.join(ROOT, "paper_2307_03914_amd", "libbspai.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char|double)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("bspai_build", "bspai_apply", "bspai_apply_T", "gmres_ir_solve", "bspai_import", "bspai_free",
                 "bspai_stats", "bspai_last_error", "bspai_export", "bspai_grad_vals"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_lists_the_same_symbols():
    import paper_2307_03914_amd as B

    assert sorted(B.SYMBOLS) == _declared()


def test_argument_errors_without_gpu():
    import paper_2307_03914_amd as B

    lib = B._lib
    out = ctypes.c_void_p()
    # null A
    assert lib.bspai_build(None, None, 1e-3, None, 1, None, ctypes.byref(out), None) == B.EINVAL
    assert b"null A" in lib.bspai_last_error()
    # precision sets: unsorted, duplicate, DROP not last, too many
    a = B._CSR(0, 0, None, None, None)
    for precs in ([B.FP32, B.FP64], [B.FP32, B.FP32], [B.DROP, B.FP32], [B.FP64, B.DROP, B.FP16], [0, 1, 2, 3, 4, 5, 5]):
        arr = (ctypes.c_int * len(precs))(*precs)
        assert lib.bspai_build(ctypes.byref(a), None, 1e-3, arr, len(precs), None, ctypes.byref(out), None) == B.EINVAL
    assert lib.bspai_apply(None, None, None, 1, 1, B.FP32, None) == B.EINVAL
    assert lib.gmres_ir_solve(None, None, None, None, None, 1, None, None) == B.EINVAL
    assert lib.gmres_ir_solve_ab(None, None, None, None, None, None, 1, None, None) == B.EINVAL
    assert b"null A_b" in lib.bspai_last_error()
    assert lib.bspai_stats(None, None) == B.EINVAL

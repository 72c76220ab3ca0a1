"""Differentiable BSPAI-GMRES-IR solve.

``BSPAISolve.apply(a_vals, b, A_pattern, M, opts)`` returns x with A x = b,
A = CSR(A_pattern, a_vals).  The backward pass is the adjoint of the linear
solve: lambda solves A^T lambda = g (GMRES-IR with the transposed bucketed
preconditioner M_b^T on the right, ``gmres_ir_solve`` with trans = 1), then
dL/db = lambda and dL/da_ij = -lambda_i x_j on the pattern
(``bspai_grad_vals``).  The preconditioner only changes how the systems are
solved, not their solutions, so no gradient flows into M.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional

import torch

from . import OK, BSPAIError, CSRMatrix, Handle, _check, _lib, _stream, solve

_lib.bspai_grad_vals.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.bspai_grad_vals.restype = C.c_int


def grad_vals(A: CSRMatrix, lam: torch.Tensor, x: torch.Tensor, stream=None) -> torch.Tensor:
    """out[e] = -lam[i] * x[j] for every entry e = (i, j) of A's pattern."""
    out = torch.empty(A.nnz, dtype=torch.float64, device=lam.device)
    p = A._p()
    _check(_lib.bspai_grad_vals(C.addressof(p), lam.contiguous().data_ptr(), x.contiguous().data_ptr(),
                                out.data_ptr(), _stream(stream)))
    return out


def _require_converged(st, what: str) -> None:
    """A gradient from a solve that met neither tolerance is not the
    gradient of the solution: raise instead of returning it."""
    for q in st if isinstance(st, list) else [st]:
        if q["status"] != OK:
            raise BSPAIError(q["status"], f"{what} ended without meeting a tolerance (stop_reason "
                                          f"{q['stop_reason']}, relres {q['relres'][-1]:.3e}, "
                                          f"eta {q['eta'][-1]:.3e})")


class BSPAISolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a_vals: torch.Tensor, b: torch.Tensor, A_pattern: CSRMatrix, M: Handle,
                opts: Optional[Dict] = None):
        opts = dict(opts or {})
        A = CSRMatrix(A_pattern.row_ptr, A_pattern.col, a_vals.detach(), A_pattern.n)
        x, st = solve(A, b.detach().contiguous(), M, **opts)
        _require_converged(st, "the forward solve")
        ctx.A = A
        ctx.M = M
        ctx.opts = opts
        ctx.stats = st
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (x,) = ctx.saved_tensors
        opts = dict(ctx.opts)
        opts["trans"] = True
        # an output buffer or starting point given for the forward solve is
        # the saved x itself: it must not receive lambda (with x0_mode 3 the
        # adjoint then starts from zero)
        opts.pop("x", None)
        lam, st = solve(ctx.A, g.contiguous().to(torch.float64), ctx.M, **opts)
        _require_converged(st, "the adjoint solve")
        ctx.adjoint_stats = st
        ga = grad_vals(ctx.A, lam, x) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return ga, gb, None, None, None

"""Pins for the oracle's option to apply A bucketed inside GMRES (Section 3,
eqs. (nbe2) and (fe2): A split into buckets with the same precisions and
threshold rule as M).  CPU only.

* One bucket of a single precision stores every entry of A rounded to that
  precision, and the bucketed product then sums those values in FP64 and
  rounds once, which is exactly the u_p product of A: GMRES and the
  refinement loop must reproduce the A_p path bit for bit, for left and for
  transposed right preconditioning.  A bf16 bucket against the u_p = bf16
  path catches an A_b that is ignored (the default u_p is fp32) or applied
  untransposed in the adjoint.
* The first Arnoldi step is recomputed from the pinned products, so A_b is
  checked to sit between the Krylov vector and M_b (left) and after M_b^T
  (transposed).
* With several buckets the refinement residual still uses the exact A, so the
  loop reaches the same backward-error floor; only the inner solves change.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _case(seed, n=300, density=0.02):
    rng = np.random.default_rng(seed)
    A = W.random_sparse(n, density, rng, dominance=0.8)
    P = W.pattern_power(A, 2)
    _, Mv, _ = O.spai(A, P)
    M = W.CSR(n, P.row_ptr, P.col, Mv)
    b = rng.standard_normal(n)
    return A, M, b


def _same_ir(r0, r1):
    assert r0["status"] == r1["status"] == O.OK
    assert r0["steps"] == r1["steps"] and r0["its"] == r1["its"]
    assert np.array_equal(r0["x"], r1["x"])
    assert r0["relres"] == r1["relres"] and r0["eta"] == r1["eta"]


@pytest.mark.parametrize("prec", [O.FP32, O.BF16])
@pytest.mark.parametrize("trans", [False, True])
def test_single_bucket_a_is_the_up_product(orc, prec, trans):
    A, M, b = _case(71)
    Mb = O.Bucketed(M, 1e-4, [O.FP64, O.FP32, O.BF16])
    Ab = O.Bucketed(A, 1e-4, [prec])
    assert np.array_equal(Ab.mt, O.round_to(prec, A.val))
    kw = dict(tol_rr=1e-10, gmres_max=60, trans=trans, dot64=True)
    ref = orc.gmres_ir(A, M, Mb, b, up=prec, **kw)
    got = orc.gmres_ir(A, M, Mb, b, Ab=Ab, **kw)
    _same_ir(ref, got)
    if prec != O.FP32:  # the option is not a no-op
        base = orc.gmres_ir(A, M, Mb, b, **kw)
        assert not np.array_equal(base["x"], got["x"])


@pytest.mark.parametrize("trans", [False, True])
def test_first_arnoldi_step_uses_bucketed_a(orc, trans):
    A, M, _ = _case(72, n=400)
    rng = np.random.default_rng(3)
    Mb = O.Bucketed(M, 1e-3, [O.FP64, O.FP32, O.FP16])
    Ab = O.Bucketed(A, 1e-5, [O.FP32, O.FP16, O.BF16])
    assert min(Ab.counts) > 0  # every bucket holds entries
    r = rng.standard_normal(A.n)
    res = orc.gmres(A, Mb, r, tau=0.5, want_basis=True, dot64=True, trans=trans, Ab=Ab)
    V, H = res["V"], res["H"]
    v1 = V[:, 0]
    if trans:  # z = A_b^T (M_b^T v_1)
        z = orc.apply(Ab.transpose(), orc.apply(Mb.transpose(), v1, O.FP32), O.FP32)
    else:  # z = M_b (A_b v_1)
        z = orc.apply(Mb, orc.apply(Ab, v1, O.FP32), O.FP32)
    h11 = math.fsum(v1 * z)
    assert abs(H[0, 0] - h11) <= 1e-13 * abs(h11)
    z2 = (z - H[0, 0] * v1).astype(np.float32).astype(np.float64)
    assert abs(H[1, 0] - math.sqrt(math.fsum(z2 * z2))) <= 1e-13 * H[1, 0]


def test_bucketed_a_product_error_bound(orc):
    """Entries in bucket k carry a relative error of at most u_k, and the
    thresholds cap |a_ij| u_k by eps ||A||_inf for every bucket but the
    first: each row of A_b x - A x is bounded by eps ||A||_inf times the
    row's count of lower-precision entries times ||x||_inf plus the u_1 term."""
    A, _, _ = _case(73, n=500)
    eps = 1e-3
    precs = [O.FP64, O.FP32, O.FP16, O.BF16]
    Ab = O.Bucketed(A, eps, precs)
    x = np.random.default_rng(4).standard_normal(A.n)
    y = orc.apply(Ab, x)
    exact = A.dense() @ x
    nA = O.norm_inf(A)
    for i in range(A.n):
        lo, hi = A.row_ptr[i], A.row_ptr[i + 1]
        low = int(np.sum(Ab.bucket[lo:hi] > 0))
        s = np.abs(A.val[lo:hi]) @ np.abs(x[A.col[lo:hi]])
        bound = low * eps * nA * np.abs(x).max() * (1 + 1e-12) + 4 * (hi - lo + 4) * 2.0 ** -53 * s
        assert abs(y[i] - exact[i]) <= bound, i


def test_multi_bucket_a_reaches_the_same_floor(orc):
    A, M, b = _case(74, n=400)
    Mb = O.Bucketed(M, 1e-4, [O.FP64, O.FP32, O.BF16])
    kw = dict(tol_rr=1e-12, gmres_max=80, dot64=True, stag_ratio=None, i_max=30)
    ref = orc.gmres_ir(A, M, Mb, b, **kw)
    for eps in (1e-6, 1e-4):
        Ab = O.Bucketed(A, eps, [O.FP32, O.FP16, O.BF16])
        got = orc.gmres_ir(A, M, Mb, b, Ab=Ab, **kw)
        assert got["status"] == O.OK and got["stop_reason"] == 1
        assert got["eta"][-1] <= 1e-14
        assert got["steps"] <= ref["steps"] + 3

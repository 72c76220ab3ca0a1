"""Pins for the oracle's CGS2 option of GMRES (classical Gram-Schmidt run
twice per Arnoldi step instead of the paper's modified Gram-Schmidt).  CPU
only.

* Arnoldi relation M A V_k = V_{k+1} H_k: a pass whose coefficients are not
  added into H breaks it.
* The whole basis stays orthonormal to working accuracy (the "twice is
  enough" property), where MGS keeps only its leading part: a single
  classical pass would lose orthogonality like kappa^2 u.
* Krylov facts that fix the result: termination within n steps, exactness
  after as many steps as A has distinct eigenvalues, the dense solve.
* The first fp32 step recomputed by hand from the pinned products.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _random_spai(seed, n):
    rng = np.random.default_rng(seed)
    A = W.random_sparse(n, 0.06, rng, dominance=0.8)
    P = W.pattern_power(A, 2)
    _, Mv, _ = O.spai(A, P)
    return A, W.CSR(n, P.row_ptr, P.col, Mv), rng


@pytest.mark.parametrize("dot64", [False, True])
def test_cgs2_arnoldi_relation_and_full_orthogonality(orc, dot64):
    A, M, rng = _random_spai(49, 50)
    Mb = O.Bucketed(M, 1e-3, [O.FP64])
    r = rng.standard_normal(50)
    res = orc.gmres(A, Mb, r, tau=1e-10, ug=O.FP64, up=O.FP64, want_basis=True, dot64=dot64, orth="cgs2")
    V, H = res["V"], res["H"]
    k = res["its"]
    MA = M.dense() @ A.dense()
    assert np.linalg.norm(MA @ V[:, :k] - V @ H) <= 1e-13 * np.linalg.norm(MA) * k
    assert np.abs(V.T @ V - np.eye(k + 1)).max() <= 1e-13
    mgs = orc.gmres(A, Mb, r, tau=1e-10, ug=O.FP64, up=O.FP64, want_basis=True, dot64=dot64)
    assert abs(mgs["its"] - k) <= 1


def test_cgs2_keeps_orthogonality_on_an_ill_conditioned_operator(orc):
    """A diagonal operator with eigenvalues spread over 1e-6..1 and M = I:
    the Krylov vectors become nearly parallel, MGS's basis loses
    orthogonality in proportion to the conditioning of the basis, CGS2's
    does not."""
    n = 200
    vals = np.logspace(-6, 0, n)
    A = W.from_dense(np.diag(vals))
    Mb = O.Bucketed(W.from_dense(np.eye(n)), 1e-3, [O.FP64])
    r = np.random.default_rng(3).standard_normal(n)
    kw = dict(tau=1e-14, ug=O.FP64, up=O.FP64, want_basis=True, dot64=True, max_it=150)
    c = orc.gmres(A, Mb, r, orth="cgs2", **kw)
    m = orc.gmres(A, Mb, r, **kw)
    Vc, Vm = c["V"], m["V"]
    loss_c = np.abs(Vc.T @ Vc - np.eye(Vc.shape[1])).max()
    loss_m = np.abs(Vm.T @ Vm - np.eye(Vm.shape[1])).max()
    assert loss_c <= 1e-13
    assert loss_m >= 1e5 * loss_c


@pytest.mark.parametrize("dot64", [False, True])
def test_cgs2_krylov_facts(orc, dot64):
    rng = np.random.default_rng(47)
    n = 12
    A = W.random_sparse(n, 0.3, rng, dominance=0.3)
    Mb = O.Bucketed(W.from_dense(np.eye(n)), 1e-3, [O.FP64])
    r = rng.standard_normal(n)
    res = orc.gmres(A, Mb, r, tau=0.0, ug=O.FP64, up=O.FP64, dot64=dot64, orth="cgs2")
    assert res["its"] <= n
    d_ref = np.linalg.solve(A.dense(), r)
    assert np.allclose(res["d"], d_ref, rtol=1e-9, atol=1e-10 * np.abs(d_ref).max())
    vals = np.array([1.0, 2.0, 5.0] * 10)
    D = W.from_dense(np.diag(vals))
    Mb = O.Bucketed(W.from_dense(np.eye(30)), 1e-3, [O.FP64])
    r = np.random.default_rng(48).standard_normal(30)
    res = orc.gmres(D, Mb, r, tau=1e-12, ug=O.FP64, up=O.FP64, dot64=dot64, orth="cgs2")
    assert res["its"] == 3
    assert np.allclose(res["d"], r / vals, rtol=1e-12)
    A, M, rng = _random_spai(50, 60)
    Mb = O.Bucketed(M, 1e-3, [O.FP64])
    r = rng.standard_normal(60)
    res = orc.gmres(A, Mb, r, tau=1e-13, ug=O.FP64, up=O.FP64, dot64=dot64, orth="cgs2")
    d = np.linalg.solve(A.dense(), r)
    assert np.allclose(res["d"], d, rtol=1e-9, atol=1e-11 * np.abs(d).max())


def test_cgs2_first_fp32_step_by_hand(orc):
    """v_1 = fl32(s / beta); z = fl32(M_b fl32(A_p v_1)); pass 1:
    h = v_1 . z (exact products summed in FP64), z' = fl32(z - h v_1) by one
    FMA; pass 2 on z' gives h'; H_11 = h + h', H_21 = ||fl32(z' - h' v_1)||."""
    rng = np.random.default_rng(54)
    A = W.random_sparse(3000, 8.0 / 3000, rng, dominance=0.8)
    _, Mv, _ = O.spai(A, A.pattern())
    M = W.CSR(A.n, A.row_ptr, A.col, Mv)
    Mb = O.Bucketed(M, 1e-3, [O.FP64, O.FP32, O.FP16])
    r = rng.standard_normal(3000)
    res = orc.gmres(A, Mb, r, tau=0.5, ug=O.FP32, up=O.FP32, want_basis=True, dot64=True, orth="cgs2")
    V, H = res["V"], res["H"]
    v1 = V[:, 0]
    z = orc.apply(Mb, orc.spmv(A, v1, O.FP32, O.FP32), O.FP32)
    h = math.fsum(v1 * z)
    z1 = (z - h * v1).astype(np.float32).astype(np.float64)
    h2 = math.fsum(v1 * z1)
    z2 = (z1 - h2 * v1).astype(np.float32).astype(np.float64)
    assert abs(H[0, 0] - (h + h2)) <= 1e-13 * abs(h)
    assert abs(H[1, 0] - math.sqrt(math.fsum(z2 * z2))) <= 1e-13 * H[1, 0]
    assert abs(h2) <= 1e-6 * abs(h)  # the second pass only removes rounding


def test_cgs2_refinement_reaches_the_same_floor(orc):
    A, M, rng = _random_spai(74, 400)
    Mb = O.Bucketed(M, 1e-4, [O.FP64, O.FP32, O.BF16])
    b = rng.standard_normal(A.n)
    kw = dict(tol_rr=1e-12, gmres_max=80, dot64=True, i_max=30)
    m = orc.gmres_ir(A, M, Mb, b, **kw)
    c = orc.gmres_ir(A, M, Mb, b, orth="cgs2", **kw)
    assert c["status"] == O.OK and c["stop_reason"] == 1
    assert abs(c["steps"] - m["steps"]) <= 1
    assert c["eta"][-1] <= 2 * m["eta"][-1]
    with pytest.raises(ValueError):
        orc.gmres_ir(A, M, Mb, b, orth="cgs")

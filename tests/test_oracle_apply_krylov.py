"""Pins for the oracle's bucketed product (Algorithm 3 and the bound quoted in
Section 2.3), the refinement residual, MGS-GMRES, the refinement loop
(Algorithm 4) and the adjoint gradient.  CPU only; exact references use
``fractions.Fraction`` and NumPy's dense solvers."""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads as W

U64 = 2.0 ** -53


def _exact_matvec(rp, ci, vals, x):
    y = []
    for i in range(len(rp) - 1):
        s = Fraction(0)
        for e in range(rp[i], rp[i + 1]):
            s += Fraction(float(vals[e])) * Fraction(float(x[ci[e]]))
        y.append(s)
    return y


def _random_spai(seed, n=60, power=2):
    rng = np.random.default_rng(seed)
    A = W.random_sparse(n, 0.06, rng, dominance=0.8)
    P = W.pattern_power(A, power)
    _, Mv, _ = O.spai(A, P)
    return A, W.CSR(n, P.row_ptr, P.col, Mv), rng


# ---------------------------------------------------------------- products

def test_device_mode_apply_is_exact_up_to_fp64_summation(orc):
    A, M, rng = _random_spai(40)
    Mb = O.Bucketed(M, 1e-3, [O.FP64, O.FP32, O.FP16, O.BF16, O.FP8])
    x = rng.standard_normal(M.n)
    y = orc.apply(Mb, x)
    ex = _exact_matvec(M.row_ptr, M.col, Mb.mt, x)
    for i in range(M.n):
        p = M.row_ptr[i + 1] - M.row_ptr[i]
        s = sum(abs(float(Fraction(float(Mb.mt[e])) * Fraction(float(x[M.col[e]]))))
                for e in range(M.row_ptr[i], M.row_ptr[i + 1]))
        gamma = (p + 6) * U64 / (1 - (p + 6) * U64)
        assert abs(Fraction(float(y[i])) - ex[i]) <= Fraction(gamma * s + 1e-300), i


def test_single_fp64_bucket_is_plain_spmv(orc):
    A, M, rng = _random_spai(41)
    Mb = O.Bucketed(M, 1e-3, [O.FP64])
    x = rng.standard_normal(M.n)
    ex = _exact_matvec(M.row_ptr, M.col, M.val, x)
    y = orc.apply(Mb, x)
    p = int(np.diff(M.row_ptr).max())
    absprod = np.abs(M.dense()) @ np.abs(x)
    assert all(abs(float(Fraction(float(y[i])) - ex[i])) <= p * U64 * absprod[i] * 1.01 for i in range(M.n))


@pytest.mark.parametrize("eps,precs", [
    (2.0 ** -37, [O.FP64, O.FP32, O.FP16, O.DROP]),
    (2.0 ** -24, [O.FP32, O.FP16, O.DROP]),
    (2.0 ** -18, [O.FP32, O.FP16, O.DROP]),
    (1e-3, [O.FP64, O.FP32, O.FP16, O.BF16, O.FP8]),
    (1e-4, [O.FP64, O.FP32, O.FP16, O.BF16]),
])
def test_normwise_backward_error_bound_of_theorem_31(orc, eps, precs):
    # Section 2.3: eps_nw = ||y_hat - y|| / (||M|| ||x||) <= (q-1) u_1 + c eps,
    # c = (1 + (q-1) u_1) + max_i sum_k p_ik^2 (1 + u_k)^2, with y the exact
    # product with the unrounded M.  Checked for the literal Algorithm 3
    # (partials in u_k) and for the decoupled FP64-accumulating product.
    A, M, rng = _random_spai(42, n=80)
    Mb = O.Bucketed(M, eps, precs)
    x = rng.standard_normal(M.n)
    ex = np.array([float(v) for v in _exact_matvec(M.row_ptr, M.col, M.val, x)])
    q = len(precs)
    u = [orc.unit_roundoff(p) for p in precs]
    u1 = u[0]
    cmax = 0.0
    for i in range(M.n):
        bk = Mb.bucket[M.row_ptr[i]:M.row_ptr[i + 1]]
        cmax = max(cmax, sum((np.count_nonzero(bk == k) ** 2) * (1 + u[k]) ** 2 for k in range(q)))
    c = (1 + (q - 1) * u1) + cmax
    bound = (q - 1) * u1 + c * eps
    denom = Mb.normM * np.abs(x).max()
    for y in (orc.apply_paper(Mb, x), orc.apply(Mb, x)):
        enw = np.abs(y - ex).max() / denom
        assert enw <= bound, (enw, bound)


def _scalar_round(prec):
    """Rounding to a storage format by a library that is not the oracle:
    NumPy's float16/float32 casts and torch's bfloat16 and float8_e4m3fn casts
    (all round to nearest, ties to even); FP64 is the identity."""
    import torch

    if prec == O.FP64:
        return lambda v: float(v)
    if prec == O.FP32:
        return lambda v: float(np.float32(v))
    if prec == O.FP16:
        return lambda v: float(np.float16(v))
    if prec == O.DROP:
        return None
    dt = {O.BF16: torch.bfloat16, O.FP8: torch.float8_e4m3fn}[prec]
    return lambda v: float(torch.tensor(v, dtype=torch.float64).to(dt).to(torch.float64))


@pytest.mark.parametrize("eps,precs", [
    (1e-3, [O.FP64, O.FP32, O.FP16, O.BF16, O.FP8]),
    (2.0 ** -24, [O.FP32, O.FP16, O.DROP]),
    (1e-2, [O.FP32, O.FP16, O.BF16]),
])
def test_literal_algorithm3_matches_scalar_arithmetic(orc, eps, precs):
    """Algorithm 3 as printed, entry by entry: in bucket k every product of
    a stored value and an entry of x (formed in FP64, as the chop emulation of
    Section 4 forms it) and every addition to the bucket's partial sum is
    rounded to u_k; the partials are then added in u_1 from bucket q down to
    bucket 1.  Recomputed here with NumPy / torch scalar roundings, so a
    partial kept in the wrong precision or a product left unrounded changes
    the bits (the order of the final u_1 sum rarely does: those few partials
    add almost exactly)."""
    A, M, rng = _random_spai(47, n=90)
    Mb = O.Bucketed(M, eps, precs)
    # x spans several binades so that the low formats round (and fp8
    # underflows) on a good share of the products
    x = rng.standard_normal(M.n) * 2.0 ** rng.integers(-6, 7, M.n)
    y = orc.apply_paper(Mb, x)
    rnd = [_scalar_round(p) for p in precs]
    nround = 0
    for i in range(M.n):
        part = [0.0] * len(precs)
        for e in range(M.row_ptr[i], M.row_ptr[i + 1]):
            k = int(Mb.bucket[e])
            if precs[k] == O.DROP:
                continue
            exact = float(Mb.mt[e]) * float(x[M.col[e]])
            prod = rnd[k](exact)
            nround += prod != exact
            part[k] = rnd[k](part[k] + prod)
        acc = 0.0
        for k in range(len(precs) - 1, -1, -1):
            acc = rnd[0](acc + part[k])
        assert y[i] == acc, (i, y[i], acc)
    assert nround > M.n  # the roundings are exercised, not vacuous
    # and it is not the decoupled product: that one keeps the low partials
    # in FP32/FP64
    assert not np.array_equal(y, orc.apply(Mb, x))


def test_tight_per_row_error_bound(orc):
    # |y_i - (M x)_i| <= sum_k u_k sum_{B_ik} max(|m_ij|, 2^emin_k s_k) |x_j| + gamma sum |mt_ij x_j|
    A, M, rng = _random_spai(43, n=70)
    precs = [O.FP64, O.FP32, O.FP16, O.BF16, O.FP8]
    Mb = O.Bucketed(M, 1e-2, precs)
    x = rng.standard_normal(M.n)
    ex = _exact_matvec(M.row_ptr, M.col, M.val, x)
    y = orc.apply(Mb, x)
    emin = [-1022, -126, -14, -126, -6]
    for i in range(M.n):
        s = 0.0
        acc = 0.0
        for e in range(M.row_ptr[i], M.row_ptr[i + 1]):
            k = Mb.bucket[e]
            xv = abs(x[M.col[e]])
            s += orc.unit_roundoff(precs[k]) * max(abs(M.val[e]), 2.0 ** emin[k] * Mb.s[k]) * xv
            acc += abs(Mb.mt[e]) * xv
        p = M.row_ptr[i + 1] - M.row_ptr[i]
        bound = s * (1 + 1e-12) + (p + 6) * U64 * acc + 1e-300
        assert abs(float(Fraction(float(y[i])) - ex[i])) <= bound, i


def test_apply_T_is_transpose(orc):
    A, M, rng = _random_spai(44)
    Mb = O.Bucketed(M, 1e-2, [O.FP64, O.FP32, O.FP16, O.BF16])
    x = rng.standard_normal(M.n)
    Mt = W.CSR(M.n, M.row_ptr, M.col, Mb.mt).dense()
    assert np.allclose(orc.apply_T(Mb, x), Mt.T @ x, rtol=1e-14, atol=1e-14 * np.abs(Mt).max())


def test_a32_spmv_rounds_values_then_accumulates(orc):
    rng = np.random.default_rng(45)
    A = W.random_sparse(50, 0.1, rng)
    x = rng.standard_normal(50).astype(np.float32).astype(np.float64)
    y = orc.spmv(A, x, O.FP32, O.FP32)
    a32 = A.val.astype(np.float32).astype(np.float64)
    ex = _exact_matvec(A.row_ptr, A.col, a32, x)
    for i in range(A.n):
        # FP64 sum of exact products (24 x 24 bits) then one rounding to binary32
        assert abs(y[i] - float(ex[i])) <= 2.0 ** -24 * abs(float(ex[i])) + 1e-9 * 2.0 ** -24 * np.abs(a32).max()


# ---------------------------------------------------------------- residual

@pytest.mark.parametrize("dd", [True, False])
def test_residual_against_exact_rationals(orc, dd):
    rng = np.random.default_rng(46)
    A = W.random_sparse(40, 0.15, rng)
    x = rng.standard_normal(40)
    # b close to A x so the residual suffers heavy cancellation
    b = A.dense() @ x + 1e-10 * rng.standard_normal(40)
    r = orc.residual(A, b, x, dd=dd)
    ax = _exact_matvec(A.row_ptr, A.col, A.val, x)
    absax = np.abs(A.dense()) @ np.abs(x)
    for i in range(40):
        ex = Fraction(float(b[i])) - ax[i]
        p = A.row_ptr[i + 1] - A.row_ptr[i]
        if dd:  # Dot2: |r - r_ex| <= u |r_ex| + gamma_p^2 sum|a x|
            g = p * U64 / (1 - p * U64)
            bound = U64 * abs(float(ex)) + 2 * g * g * (absax[i] + abs(b[i]))
        else:
            bound = (p + 1) * U64 * (absax[i] + abs(b[i]))
        assert abs(float(Fraction(float(r[i])) - ex)) <= bound * 1.001 + 1e-320, (i, dd)


# ---------------------------------------------------------------- GMRES

@pytest.mark.parametrize("dot64", [False, True])
def test_gmres_terminates_within_n_steps_in_fp64(orc, dot64):
    rng = np.random.default_rng(47)
    n = 12
    A = W.random_sparse(n, 0.3, rng, dominance=0.3)
    Mb = O.Bucketed(W.from_dense(np.eye(n)), 1e-3, [O.FP64])
    r = rng.standard_normal(n)
    res = orc.gmres(A, Mb, r, tau=0.0, ug=O.FP64, up=O.FP64, dot64=dot64)
    assert res["its"] <= n
    d_ref = np.linalg.solve(A.dense(), r)
    assert np.allclose(res["d"], d_ref, rtol=1e-9, atol=1e-10 * np.abs(d_ref).max())


@pytest.mark.parametrize("dot64", [False, True])
def test_gmres_distinct_eigenvalues_bound(orc, dot64):
    # M = I and A diagonal with 3 distinct values: the Krylov space of any
    # vector has dimension <= 3, so GMRES is exact after 3 steps.
    vals = np.array([1.0, 2.0, 5.0] * 10)
    A = W.from_dense(np.diag(vals))
    Mb = O.Bucketed(W.from_dense(np.eye(30)), 1e-3, [O.FP64])
    r = np.random.default_rng(48).standard_normal(30)
    res = orc.gmres(A, Mb, r, tau=1e-12, ug=O.FP64, up=O.FP64, dot64=dot64)
    assert res["its"] == 3
    assert np.allclose(res["d"], r / vals, rtol=1e-12)


@pytest.mark.parametrize("dot64", [False, True])
def test_arnoldi_relation_and_orthogonality(orc, dot64):
    # M A V_k = V_{k+1} H_k with orthonormal V (MGS, FP64)
    A, M, rng = _random_spai(49, n=50)
    Mb = O.Bucketed(M, 1e-3, [O.FP64])
    r = rng.standard_normal(50)
    res = orc.gmres(A, Mb, r, tau=1e-10, ug=O.FP64, up=O.FP64, want_basis=True, dot64=dot64)
    V, H = res["V"], res["H"]
    k = res["its"]
    MA = M.dense() @ A.dense()
    assert np.linalg.norm(MA @ V[:, :k] - V @ H) <= 1e-13 * np.linalg.norm(MA) * k
    # MGS keeps the early basis orthogonal to working accuracy; orthogonality
    # is lost only as the residual becomes small (the known MGS-GMRES
    # behaviour), so only the leading half of the basis is checked tightly.
    h = (k + 1) // 2
    assert np.abs(V[:, :h].T @ V[:, :h] - np.eye(h)).max() <= 1e-12
    assert np.abs(V.T @ V - np.eye(k + 1)).max() <= 1e-3


@pytest.mark.parametrize("dot64", [False, True])
def test_gmres_matches_dense_preconditioned_solve(orc, dot64):
    A, M, rng = _random_spai(50, n=60)
    Mb = O.Bucketed(M, 1e-3, [O.FP64])
    r = rng.standard_normal(60)
    res = orc.gmres(A, Mb, r, tau=1e-13, ug=O.FP64, up=O.FP64, dot64=dot64)
    d = np.linalg.solve(A.dense(), r)
    assert np.allclose(res["d"], d, rtol=1e-9, atol=1e-11 * np.abs(d).max())


def _ulp32_close(a, b):
    a32, b32 = a.astype(np.float32), b.astype(np.float32)
    assert np.array_equal(a32.astype(np.float64), a) and np.array_equal(b32.astype(np.float64), b)
    return np.abs(a - b).max() <= np.spacing(np.abs(b32)).max()


@pytest.mark.parametrize("dot64", [False, True])
def test_fp32_first_arnoldi_step_by_hand(orc, dot64):
    """First Arnoldi step of fp32 GMRES recomputed with numpy from the pinned
    apply and A_p products: v_1 = fl32(s / beta), z = fl32(M_b fl32(A_p v_1)),
    h_11 = v_1 . z, v_2 = fl32((z - h_11 v_1) / h_21).  With dot64 the dot
    products and norms are exact sums of fp32 products rounded once to FP64;
    the literal mode sums in fp32 and gives h_11 only to about sqrt(n) u_32."""
    import math

    rng = np.random.default_rng(54)
    A = W.random_sparse(3000, 8.0 / 3000, rng, dominance=0.8)
    _, Mv, _ = O.spai(A, A.pattern())
    M = W.CSR(A.n, A.row_ptr, A.col, Mv)
    Mb = O.Bucketed(M, 1e-3, [O.FP64, O.FP32, O.FP16])
    r = rng.standard_normal(3000)
    res = orc.gmres(A, Mb, r, tau=0.5, ug=O.FP32, up=O.FP32, want_basis=True, dot64=dot64)
    V, H = res["V"], res["H"]
    s = orc.apply(Mb, r.astype(np.float32).astype(np.float64), O.FP32)
    beta = math.sqrt(math.fsum(s * s))
    v1 = (s / beta).astype(np.float32).astype(np.float64)
    if dot64:
        assert _ulp32_close(V[:, 0], v1)
    else:  # beta is rounded to fp32 first
        assert np.abs(V[:, 0] - v1).max() <= 4 * 2.0 ** -24 * np.abs(v1).max()
    z = orc.apply(Mb, orc.spmv(A, V[:, 0], O.FP32, O.FP32), O.FP32)
    h11 = math.fsum(V[:, 0] * z)
    if dot64:
        assert abs(H[0, 0] - h11) <= 1e-13 * abs(h11)
        z2 = (z - H[0, 0] * V[:, 0]).astype(np.float32).astype(np.float64)
        h21 = math.sqrt(math.fsum(z2 * z2))
        assert abs(H[1, 0] - h21) <= 1e-13 * h21
        assert _ulp32_close(V[:, 1], (z2 / H[1, 0]).astype(np.float32).astype(np.float64))
    else:
        assert H[0, 0] == float(np.float32(H[0, 0]))  # rounded to fp32
        assert abs(H[0, 0] - h11) <= 3000 * 2.0 ** -24 * np.abs(V[:, 0] * z).sum()


def test_fp32_gmres_with_exact_inverse_takes_one_step(orc):
    rng = np.random.default_rng(51)
    n = 16
    D = rng.standard_normal((n, n)) + 2 * n * np.eye(n)
    A = W.from_dense(D, np.ones((n, n), bool))
    _, Mv, _ = orc.spai(A, W.full_pattern(n))
    M = W.CSR(n, W.full_pattern(n).row_ptr, W.full_pattern(n).col, Mv)
    Mb = O.Bucketed(M, 1e-3, [O.FP64])
    res = orc.gmres(A, Mb, rng.standard_normal(n), tau=1e-4)
    assert res["its"] == 1


@pytest.mark.parametrize("dot64", [False, True])
def test_right_preconditioned_transposed_gmres(orc, dot64):
    A, M, rng = _random_spai(52, n=50)
    Mb = O.Bucketed(M, 1e-3, [O.FP64])
    r = rng.standard_normal(50)
    res = orc.gmres(A, Mb, r, tau=1e-13, ug=O.FP64, up=O.FP64, trans=True, dot64=dot64)
    d = np.linalg.solve(A.dense().T, r)
    assert np.allclose(res["d"], d, rtol=1e-9, atol=1e-11 * np.abs(d).max())


# ---------------------------------------------------------------- refinement

def test_ir_reaches_fp64_backward_error(orc):
    # kappa << 1/u: the refinement drives eta to O(u_64) (Section 1's
    # convergence conditions for GMRES-IR with u_r = u^2).
    A, M, rng = _random_spai(53, n=200, power=1)
    Mb = O.Bucketed(M, 1e-4, [O.FP64, O.FP32, O.FP16, O.BF16])
    xt = rng.standard_normal(200)
    b = W.matvec_extended(A, xt)
    res = orc.gmres_ir(A, M, Mb, b, tol_rr=0.0, tol_be=0.0, i_max=12)
    assert res["stop_reason"] in (3, 4) and res["status"] in (O.ESTAG, O.ENOCONV)
    assert res["eta"][-1] <= 4 * U64
    D = A.dense()
    kappa = np.linalg.cond(D, np.inf)
    assert np.abs(res["x"] - xt).max() / np.abs(xt).max() <= 10 * kappa * U64
    assert res["its_total"] == sum(res["its"])


def test_ir_stagnation_ratio(orc):
    # with no tolerance to meet, the default rule stops on stagnation; a looser
    # ratio cannot stop earlier, and with the test off the loop runs to i_max
    A, M, rng = _random_spai(53, n=200, power=1)
    Mb = O.Bucketed(M, 1e-4, [O.FP64, O.FP32, O.FP16, O.BF16])
    b = W.matvec_extended(A, rng.standard_normal(200))
    runs = {r: orc.gmres_ir(A, M, Mb, b, tol_rr=0.0, tol_be=0.0, i_max=12, stag_ratio=r)
            for r in (0.5, 0.999, None)}
    assert runs[0.5]["stop_reason"] == 3 and runs[0.5]["steps"] < 12
    # no tolerance was met: a stagnation stop is not reported as success
    assert runs[0.5]["status"] == O.ESTAG
    assert runs[0.999]["steps"] >= runs[0.5]["steps"]
    assert runs[None]["stop_reason"] == 4 and runs[None]["steps"] == 12 and runs[None]["status"] == O.ENOCONV
    # the corrections before the stop are the same in every run
    k = runs[0.5]["steps"]
    assert runs[None]["eta"][: k + 1] == runs[0.5]["eta"][: k + 1]


def test_ir_config1_converges_to_relative_residual(orc):
    c = W.config("1", small=True)
    A, P = c["A"], c["P"]
    _, Mv, _ = orc.spai(A, P)
    M = W.CSR(A.n, P.row_ptr, P.col, Mv)
    Mb = O.Bucketed(M, c["eps"][0], c["precs"])
    res = orc.gmres_ir(A, M, Mb, c["b"], tol_rr=1e-10)
    assert res["status"] == O.OK and res["stop_reason"] == 1
    assert res["relres"][-1] <= 1e-10
    assert 2 <= res["steps"] <= 4


def test_ir_caller_starting_vector(orc):
    """x0_mode 3 starts from the caller's x_0: from zero it repeats x0_mode 2
    bit for bit, from the solution it stops before any correction, and from
    elsewhere it still reaches the tolerance."""
    c = W.config("1", small=True)
    A, P = c["A"], c["P"]
    _, Mv, _ = orc.spai(A, P)
    M = W.CSR(A.n, P.row_ptr, P.col, Mv)
    Mb = O.Bucketed(M, c["eps"][0], c["precs"])
    kw = dict(tol_rr=1e-10)
    z = orc.gmres_ir(A, M, Mb, c["b"], x0_mode=2, **kw)
    z3 = orc.gmres_ir(A, M, Mb, c["b"], x0_mode=3, x0=np.zeros(A.n), **kw)
    assert np.array_equal(z["x"], z3["x"]) and z["its"] == z3["its"]
    at = orc.gmres_ir(A, M, Mb, c["b"], x0_mode=3, x0=np.linalg.solve(A.dense(), c["b"]), **kw)
    assert at["steps"] == 0 and at["stop_reason"] == 1
    far = orc.gmres_ir(A, M, Mb, c["b"], x0_mode=3, x0=np.full(A.n, 10.0), **kw)
    assert far["status"] == O.OK and far["relres"][-1] <= 1e-10
    with pytest.raises(ValueError):
        orc.gmres_ir(A, M, Mb, c["b"], x0_mode=3, **kw)


def test_ir_reports_noconvergence(orc):
    c = W.config("1", small=True)
    A, P = c["A"], c["P"]
    _, Mv, _ = orc.spai(A, P)
    M = W.CSR(A.n, P.row_ptr, P.col, Mv)
    Mb = O.Bucketed(M, 2.0 ** -53, [O.FP64])
    res = orc.gmres_ir(A, M, Mb, c["b"], tol_rr=1e-30, i_max=1)
    assert res["status"] == O.ENOCONV and res["steps"] == 1


def test_direct_gradient_matches_dense_and_iterative_adjoint(orc):
    """The sparse-LU gradient equals a dense solve of A^T lambda = g and the
    refinement-based gradient, and dL/da_ij = -lambda_i x_j is checked
    against a finite difference in one entry of A."""
    A, M, rng = _random_spai(55, n=50)
    Mb = O.Bucketed(M, 1e-3, [O.FP64, O.FP32, O.FP16, O.BF16, O.FP8])
    b = rng.standard_normal(50)
    D = A.dense()
    x = np.linalg.solve(D, b)
    g = rng.standard_normal(50)
    out = orc.gradient_direct(A, x, g)
    lam = np.linalg.solve(D.T, g)
    assert np.allclose(out["grad_b"], lam, rtol=1e-12, atol=1e-14 * np.abs(lam).max())
    it = orc.gradient(A, M, Mb, x, g, tol_rr=1e-14, i_max=20)
    assert np.abs(out["grad_vals"] - it["grad_vals"]).max() <= 1e-9 * np.abs(it["grad_vals"]).max()
    # d(g . x)/d a_e for the entry e = (i, j): perturb it alone
    e = int(np.argmax(np.abs(out["grad_vals"])))
    i = int(np.searchsorted(A.row_ptr, e, side="right") - 1)
    j = int(A.col[e])
    h = 1e-6 * abs(D[i, j])
    Dp, Dm = D.copy(), D.copy()
    Dp[i, j] += h
    Dm[i, j] -= h
    fd = (g @ np.linalg.solve(Dp, b) - g @ np.linalg.solve(Dm, b)) / (2 * h)
    assert abs(fd - out["grad_vals"][e]) <= 1e-6 * abs(fd)


def test_gradient_matches_dense_adjoint(orc):
    A, M, rng = _random_spai(54, n=40)
    Mb = O.Bucketed(M, 1e-3, [O.FP64, O.FP32, O.FP16, O.BF16, O.FP8])
    b = rng.standard_normal(40)
    fwd = orc.gmres_ir(A, M, Mb, b, tol_rr=1e-14, i_max=20)
    x = fwd["x"]
    g = rng.standard_normal(40)
    out = orc.gradient(A, M, Mb, x, g, tol_rr=1e-14, i_max=20)
    D = A.dense()
    lam = np.linalg.solve(D.T, g)
    assert np.allclose(out["grad_b"], lam, rtol=1e-10, atol=1e-12 * np.abs(lam).max())
    rows = np.repeat(np.arange(40), np.diff(A.row_ptr))
    gv = -lam[rows] * np.linalg.solve(D, b)[A.col]
    assert np.allclose(out["grad_vals"], gv, rtol=1e-9, atol=1e-12 * np.abs(gv).max())
    # directional finite difference of L(b) = g . x(b) along a random b-direction
    db = rng.standard_normal(40)
    h = 1e-4
    fd = (g @ np.linalg.solve(D, b + h * db) - g @ np.linalg.solve(D, b - h * db)) / (2 * h)
    assert abs(fd - out["grad_b"] @ db) <= 1e-8 * abs(fd) + 1e-12

"""Pins for the oracle's SPAI construction in a lower precision u_f (the
(single, double, quad) and (half, single, double) settings of Section 4, with
its one-sided column scaling).  CPU only.

* Householder least squares is backward stable (Higham, Accuracy and
  Stability of Numerical Algorithms, Thm. 20.3): the normal-equation residual
  of the u_f solution is O(m n u_f) ||A||^2 ||x||, and on a consistent
  problem its forward error is O(m n u_f kappa_2(A)).  Both are checked, and
  so is the converse, that the error is at least a fraction of u_f (the
  arithmetic really is rounded).
* The placement of every rounding is checked against NumPy's IEEE float16 and
  float32 scalar types, whose +, -, *, / and sqrt are correctly rounded.
* A full pattern gives the dense inverse to O(n^2 u_f kappa); every entry of
  M is a u_f number.
* Entries beyond the fp16 range overflow the unscaled half-precision QR, and
  the scaling of Section 4 removes the overflow.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

UF = {O.FP32: 2.0 ** -24, O.FP16: 2.0 ** -11}
NP = {O.FP32: np.float32, O.FP16: np.float16}


def _rand_ls(rng, m, n, prec):
    A = O.round_to(prec, rng.uniform(-1, 1, (m, n)).ravel()).reshape(m, n)
    x = rng.standard_normal(n)
    return A, x


@pytest.mark.parametrize("prec", [O.FP32, O.FP16])
def test_low_precision_ls_is_backward_stable(orc, prec):
    rng = np.random.default_rng(81)
    u = UF[prec]
    for m, n in ((12, 5), (25, 13), (40, 8)):
        A, _ = _rand_ls(rng, m, n, prec)
        b = O.round_to(prec, rng.uniform(-1, 1, m))
        st, x = orc.householder_ls(A, b, prec)
        assert st == O.OK
        st64, x64 = orc.householder_ls(A, b)
        r = b - A @ x
        nA = np.linalg.norm(A, 2)
        assert np.linalg.norm(A.T @ r) <= 10 * m * n * u * nA * (nA * np.linalg.norm(x) + np.linalg.norm(b))
        # the rounding is real: the u_f answer is not the FP64 one
        assert np.abs(x - x64).max() >= 1e-3 * u * np.abs(x64).max()


@pytest.mark.parametrize("prec", [O.FP32, O.FP16])
def test_low_precision_ls_forward_error_on_consistent_systems(orc, prec):
    rng = np.random.default_rng(82)
    u = UF[prec]
    for m, n in ((10, 10), (20, 7), (33, 16)):
        A = O.round_to(prec, (rng.uniform(-1, 1, (m, n)) + 2 * np.eye(m, n)).ravel()).reshape(m, n)
        xt = O.round_to(prec, rng.uniform(-1, 1, n))
        b = A @ xt  # consistent in exact arithmetic; kept in FP64 for the reference
        st64, x64 = orc.householder_ls(A, b)
        bf = O.round_to(prec, b)
        st, x = orc.householder_ls(A, bf, prec)
        assert st == O.OK and st64 == O.OK
        kappa = np.linalg.cond(A)
        err = np.linalg.norm(x - xt) / np.linalg.norm(xt)
        assert err <= 10 * m * n * u * kappa
        assert err >= 1e-3 * u


def _np_householder(A, b, T):
    """The same Householder steps in NumPy scalars of type T (each operation
    correctly rounded in T), sums left to right."""
    m, n = A.shape
    A = [[T(A[i, j]) for j in range(n)] for i in range(m)]
    b = [T(v) for v in b]
    zero = T(0)
    for c in range(n):
        nrm2 = zero
        for i in range(c, m):
            nrm2 = T(nrm2 + T(A[i][c] * A[i][c]))
        nrm = T(np.sqrt(nrm2))
        alpha = A[c][c]
        beta = T(-nrm if alpha >= 0 else nrm)
        v = [A[i][c] for i in range(c, m)]
        v[0] = T(alpha - beta)
        vtv = zero
        for vi in v:
            vtv = T(vtv + T(vi * vi))
        for j in list(range(c + 1, n)) + [None]:
            col = [A[i][j] for i in range(c, m)] if j is not None else b[c:]
            w = zero
            for vi, ci in zip(v, col):
                w = T(w + T(vi * ci))
            f = T(T(T(2) * w) / vtv)
            new = [T(ci - T(f * vi)) for vi, ci in zip(v, col)]
            if j is None:
                b[c:] = new
            else:
                for i in range(c, m):
                    A[i][j] = new[i - c]
        A[c][c] = beta
    x = [zero] * n
    for c in range(n - 1, -1, -1):
        s = b[c]
        for j in range(c + 1, n):
            s = T(s - T(A[c][j] * x[j]))
        x[c] = T(s / A[c][c])
    return np.array([float(v) for v in x])


@pytest.mark.parametrize("prec", [O.FP32, O.FP16])
def test_low_precision_ls_rounding_matches_ieee_scalars(orc, prec):
    rng = np.random.default_rng(83)
    with np.errstate(all="ignore"):
        for m, n in ((6, 3), (11, 6), (9, 9)):
            A, _ = _rand_ls(rng, m, n, prec)
            b = O.round_to(prec, rng.uniform(-1, 1, m))
            st, x = orc.householder_ls(A, b, prec)
            assert st == O.OK
            ref = _np_householder(A, b, NP[prec])
            assert np.array_equal(x, ref), (m, n, x - ref)


@pytest.mark.parametrize("prec", [O.FP32, O.FP16])
def test_low_precision_spai_full_pattern_is_the_inverse(orc, prec):
    rng = np.random.default_rng(84)
    n = 12
    D = rng.uniform(-1, 1, (n, n)) + 4 * np.eye(n)
    A = W.from_dense(D, np.ones((n, n), bool))
    P = W.full_pattern(n)
    for scale in (False, True):
        st, Mv, _ = orc.spai(A, P, scale=scale, uf=prec)
        assert st == O.OK
        assert np.array_equal(O.round_to(prec, Mv), Mv)  # u_f numbers
        M = W.CSR(n, P.row_ptr, P.col, Mv).dense()
        inv = np.linalg.inv(D)
        kappa = np.linalg.cond(D)
        err = np.abs(M - inv).max() / np.abs(inv).max()
        assert 1e-3 * UF[prec] <= err <= 10 * n * n * UF[prec] * kappa


def test_fp64_construction_is_unchanged(orc):
    rng = np.random.default_rng(85)
    A = W.random_sparse(200, 0.03, rng, dominance=0.8)
    P = W.pattern_power(A, 2)
    for scale in (False, True):
        st0, M0, _ = orc.spai(A, P, scale=scale)
        st1, M1, _ = orc.spai(A, P, scale=scale, uf=O.FP64)
        assert st0 == st1 == O.OK and np.array_equal(M0, M1)


def test_half_precision_needs_the_scaling(orc):
    """Rows of size 1e5 exceed fp16's 65,504: unscaled, their entries (and
    the norms of the QR) overflow; scaled to unit column maxima of A^T, the
    half-precision SPAI is finite and close to the FP64 one."""
    rng = np.random.default_rng(86)
    n = 300
    A = W.random_sparse(n, 0.02, rng, dominance=0.8)
    big = np.repeat(np.where(np.arange(n) % 3 == 0, 1e5, 1.0), np.diff(A.row_ptr))
    A = W.CSR(n, A.row_ptr, A.col, A.val * big)
    P = A.pattern()
    st, _, bad = orc.spai(A, P, uf=O.FP16)
    assert st == O.ENAN
    st, Mh, _ = orc.spai(A, P, scale=True, uf=O.FP16)
    assert st == O.OK and np.isfinite(Mh).all()
    st, M64, _ = orc.spai(A, P, scale=True)
    rel = np.abs(Mh - M64).max() / np.abs(M64).max()
    assert rel <= 0.05
    # the residual ||I - M A||_F of the half-precision M is close to the FP64 one
    Ad = A.dense()
    r64 = np.linalg.norm(np.eye(n) - W.CSR(n, P.row_ptr, P.col, M64).dense() @ Ad)
    rh = np.linalg.norm(np.eye(n) - W.CSR(n, P.row_ptr, P.col, Mh).dense() @ Ad)
    assert r64 <= rh <= r64 + 0.05 * math.sqrt(n)

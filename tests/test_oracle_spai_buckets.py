"""Pins for the oracle's SPAI construction (eq. (fronormmin), eq. (redprob),
Algorithm 4 step 1) and bucketing (Algorithm 2, eq. (nint)), plus the storage
column of Tables 3 and 4.  CPU only."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- least squares

@pytest.mark.parametrize("m,n,seed", [(5, 5, 0), (13, 5, 1), (25, 13, 2), (60, 17, 3), (200, 40, 4)])
def test_householder_ls_matches_numpy_lstsq(orc, m, n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    st, x = orc.householder_ls(A, b)
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    assert st == O.OK
    assert np.allclose(x, ref, rtol=1e-12 * np.linalg.cond(A), atol=1e-13)


def test_householder_ls_rank_deficient_reports_erank(orc):
    A = np.ones((6, 3))
    st, _ = orc.householder_ls(A, np.ones(6))
    assert st == O.ERANK


# ---------------------------------------------------------------- SPAI

def test_full_pattern_gives_dense_inverse(orc):
    rng = np.random.default_rng(10)
    n = 14
    D = rng.standard_normal((n, n)) + n * np.eye(n)
    A = W.from_dense(D, np.ones((n, n), bool))
    st, Mv, _ = orc.spai(A, W.full_pattern(n))
    assert st == O.OK
    M = Mv.reshape(n, n)
    Ainv = np.linalg.inv(D)
    assert np.abs(M - Ainv).max() <= 1e-13 * np.abs(Ainv).max() * np.linalg.cond(D)


def test_diagonal_matrix_identity_pattern(orc):
    d = np.array([3.0, -7.0, 0.1, 1e5, 2.0 ** -30])
    A = W.from_dense(np.diag(d))
    st, Mv, _ = orc.spai(A, W.identity_pattern(len(d)))
    assert st == O.OK
    # a 1x1 Householder solve rounds a handful of times: within 2 ulp of 1/d
    assert np.all(np.abs(Mv - 1.0 / d) <= 2 * np.spacing(np.abs(1.0 / d)))


def test_block_diagonal_with_block_pattern_is_exact_inverse(orc):
    rng = np.random.default_rng(11)
    blocks = [rng.standard_normal((k, k)) + 3 * k * np.eye(k) for k in (3, 4, 2, 5)]
    n = sum(b.shape[0] for b in blocks)
    D = np.zeros((n, n))
    mask = np.zeros((n, n), bool)
    o = 0
    for b in blocks:
        k = b.shape[0]
        D[o:o + k, o:o + k] = b
        mask[o:o + k, o:o + k] = True
        o += k
    A = W.from_dense(D, mask)
    st, Mv, _ = orc.spai(A, A.pattern())
    assert st == O.OK
    M = W.CSR(n, A.row_ptr, A.col, Mv).dense()
    assert np.allclose(M, np.linalg.inv(D), rtol=0, atol=1e-14 * 10)


@pytest.mark.parametrize("seed,power", [(20, 1), (21, 2)])
def test_each_row_solves_the_full_least_squares_problem(orc, seed, power):
    # Row k of M must minimise || e_k - A^T m || over m supported on J_k
    # (the k-th term of eq. (fronormmin) for A^T); the shadow reduction of
    # eq. (redprob) may not change the minimiser.  Checked with the full,
    # unreduced columns A^T[:, J_k] and NumPy's lstsq.
    rng = np.random.default_rng(seed)
    n = 40
    A = W.random_sparse(n, 0.08, rng, dominance=0.7)
    P = W.pattern_power(A, power)
    st, Mv, _ = orc.spai(A, P)
    assert st == O.OK
    D = A.dense()
    for k in range(n):
        J = P.col[P.row_ptr[k]:P.row_ptr[k + 1]]
        e = np.zeros(n)
        e[k] = 1
        ref = np.linalg.lstsq(D.T[:, J], e, rcond=None)[0]
        got = Mv[P.row_ptr[k]:P.row_ptr[k + 1]]
        assert np.allclose(got, ref, rtol=1e-10, atol=1e-12), k


def test_frobenius_objective_is_minimal_on_pattern(orc):
    # || I - M A ||_F = || I - A^T M^T ||_F cannot be lowered by any perturbation
    # of M on its pattern (first-order optimality of the row least squares).
    rng = np.random.default_rng(22)
    n = 30
    A = W.random_sparse(n, 0.1, rng, dominance=1.0)
    P = A.pattern()
    st, Mv, _ = orc.spai(A, P)
    D = A.dense()
    f0 = np.linalg.norm(np.eye(n) - W.CSR(n, P.row_ptr, P.col, Mv).dense() @ D)
    for t in range(20):
        dv = 1e-6 * rng.standard_normal(P.nnz)
        f1 = np.linalg.norm(np.eye(n) - W.CSR(n, P.row_ptr, P.col, Mv + dv).dense() @ D)
        assert f1 >= f0 - 1e-15


def test_scaling_matches_unscaled(orc):
    # Section 4's one-sided column scaling of A^T changes nothing in exact
    # arithmetic: the scaled and unscaled M agree to O(kappa u).
    rng = np.random.default_rng(23)
    n = 50
    A = W.random_sparse(n, 0.08, rng)
    A.val *= np.exp(3 * rng.standard_normal(A.nnz))
    P = W.pattern_power(A, 2)
    _, M0, _ = orc.spai(A, P)
    _, M1, _ = orc.spai(A, P, scale=True)
    assert np.allclose(M0, M1, rtol=1e-9, atol=1e-12 * np.abs(M0).max())


def test_zero_diagonal_with_identity_pattern_reports_zero_row(orc):
    # Section 4: with the identity pattern a zero a_kk gives a zero row of M.
    D = np.array([[2.0, 1.0, 0.0], [1.0, 0.0, 1.0], [0.0, 1.0, 3.0]])
    A = W.from_dense(D)
    st, Mv, bad = orc.spai(A, W.identity_pattern(3))
    assert st == O.EZEROROW and bad == 1


def test_row_subset_matches_full_build(orc):
    c = W.config("3", small=True)
    A, P = c["A"], c["P"]
    _, Mfull, _ = orc.spai(A, P)
    rows = np.array([0, 17, 999, 4321, A.n - 1], dtype=np.int32)
    _, Msub, _ = orc.spai(A, P, rows=rows)
    for k in rows:
        s = slice(P.row_ptr[k], P.row_ptr[k + 1])
        assert np.array_equal(Msub[s], Mfull[s])


# ---------------------------------------------------------------- buckets

def _hand_matrix():
    # ||M||_inf = 1 exactly (row 0).  With eps = 2^-30 and (fp64, fp32, fp16):
    # t_2 = 2^-30 / 2^-24 = 2^-6, t_3 = 2^-30 / 2^-11 = 2^-19 (eq. (nint)).
    a = 2.0 ** -6
    b = 2.0 ** -19
    tiny = 2.0 ** -40
    rows = [
        [0.5, 0.5],
        [a, a + tiny, b, b + tiny, 0.0, -a, -(a + tiny), -b],
    ]
    # expected buckets (0-based): bucket 1 strictly above t_2, bucket 3 at or
    # below t_3, bucket 2 in (t_3, t_2].
    expect = [[0, 0], [1, 0, 2, 1, 2, 1, 0, 2]]
    n = 8
    row_ptr = [0]
    col, val = [], []
    for r in rows:
        col += list(range(len(r)))
        val += r
        row_ptr.append(len(col))
    for _ in range(n - len(rows)):
        row_ptr.append(len(col))
    M = W.CSR(n, np.array(row_ptr, np.int32), np.array(col, np.int32), np.array(val))
    return M, sum(expect, [])


def test_bucket_intervals_by_hand(orc):
    M, expect = _hand_matrix()
    Mb = O.Bucketed(M, 2.0 ** -30, [O.FP64, O.FP32, O.FP16])
    assert Mb.normM == 1.0
    assert list(Mb.t) == [2.0 ** 23, 2.0 ** -6, 2.0 ** -19]
    assert list(Mb.bucket) == expect


def test_bucket_with_drop(orc):
    # (fp32, fp16, drop): t_1 = eps/2^-24, t_2 = eps/2^-11, t_3 = eps (u_3 = 1).
    M, _ = _hand_matrix()
    eps = 2.0 ** -20
    Mb = O.Bucketed(M, eps, [O.FP32, O.FP16, O.DROP])
    a = np.abs(M.val)
    exp = np.where(a > 2.0 ** -9, 0, np.where(a <= 2.0 ** -20, 2, 1))
    assert np.array_equal(Mb.bucket, exp)
    assert np.all(Mb.mt[Mb.bucket == 2] == 0.0)


def test_single_bucket_holds_everything(orc):
    M, _ = _hand_matrix()
    Mb = O.Bucketed(M, 1e-3, [O.FP64])
    assert np.all(Mb.bucket == 0) and np.array_equal(Mb.mt, M.val)


def test_bucket_invariants_on_spai(orc):
    c = W.config("2", small=True)
    A, P = c["A"], c["P"]
    _, Mv, _ = orc.spai(A, P)
    M = W.CSR(A.n, P.row_ptr, P.col, Mv)
    prev = None
    for eps in [2.0 ** -60, 1e-12, 1e-8, 1e-6, 1e-4, 1e-2, 1.0, 1e6]:
        Mb = O.Bucketed(M, eps, c["precs"])
        assert Mb.counts.sum() == M.nnz
        if prev is not None:  # entries only move towards lower precision
            assert np.all(Mb.bucket >= prev)
        prev = Mb.bucket.copy()
    lo = O.Bucketed(M, 2.0 ** -60, c["precs"])
    assert np.all(lo.bucket[M.val != 0] == 0)
    hi = O.Bucketed(M, 1e6, c["precs"])
    assert np.all(hi.bucket == len(c["precs"]) - 1)


def test_stored_values_within_unit_roundoff(orc):
    # each stored value is the bucket format's rounding of m (scaled by a power
    # of two): |mt - m| <= u_k |m| wherever the scaled value is normal.
    rng = np.random.default_rng(30)
    n = 200
    A = W.random_sparse(n, 0.05, rng)
    A.val = A.val * np.exp(4 * rng.standard_normal(A.nnz))
    precs = [O.FP64, O.FP32, O.FP16, O.BF16, O.FP8]
    Mb = O.Bucketed(A, 1e-3, precs)
    u = np.array([orc.unit_roundoff(p) for p in precs])
    emin = {O.FP64: -1022, O.FP32: -126, O.FP16: -14, O.BF16: -126, O.FP8: -6}
    for k, p in enumerate(precs):
        sel = Mb.bucket == k
        if not sel.any():
            continue
        bound = u[k] * np.maximum(np.abs(A.val[sel]), 2.0 ** emin[p] * Mb.s[k])
        assert np.all(np.abs(Mb.mt[sel] - A.val[sel]) <= bound)
        assert Mb.s[k] == 2.0 ** np.round(np.log2(Mb.s[k]))


def test_storage_column_of_tables_3_and_4(orc):
    with open(os.path.join(GOLDEN, "storage_tables.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 30
    for table, name, eps, nnz, counts, pct in rows:
        counts = [int(c) for c in counts.split(",")]
        assert sum(counts) == int(nnz), name
        if table == "T3":
            got = orc.storage_pct(counts, [O.FP64, O.FP32, O.FP16, O.DROP], drop_bytes=0)
        else:
            got = orc.storage_pct(counts, [O.FP32, O.FP16, O.DROP], drop_bytes=1)
        assert abs(got - float(pct)) <= 0.1, (table, name, eps, got, pct)
    # the worked example: steam1, eps = 2^-53 -> (556*8 + 537*4 + 12*2) / (1105*8)
    assert abs(orc.storage_pct([556, 537, 12, 0], [O.FP64, O.FP32, O.FP16, O.DROP]) -
               float(Fraction(556 * 8 + 537 * 4 + 12 * 2, 1105 * 8) * 100)) < 1e-12

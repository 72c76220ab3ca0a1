"""Pins of the oracle's adaptive SPAI (Algorithm 1 with its augmentation
loop, run on A^T) against facts that do not depend on its code: the
fixed-pattern SPAI it starts from, a brute-force univariate minimisation
for the index it adds, monotone residuals, and the exact inverse once the
pattern is full."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _row_residuals(A, M):
    """||e_k - A^T m_k||_2 for every row k of M (row k of M times A vs e_k)."""
    R = M.dense() @ A.dense() - np.eye(A.n)
    return np.linalg.norm(R, axis=1)


def _stencil():
    return W.config("2", small=True)["A"]


def test_alpha_zero_is_the_fixed_identity_pattern():
    A = _stencil()
    st, Mv, _ = O.spai(A, W.identity_pattern(A.n))
    for kw in (dict(alpha=0), dict(alpha=5, eps=1e9)):
        r = O.spai_adaptive(A, beta=8, **kw)
        assert r["status"] == O.OK
        assert np.array_equal(r["M"].row_ptr, np.arange(A.n + 1))
        assert np.array_equal(r["M"].col, np.arange(A.n))
        assert np.array_equal(r["M"].val, Mv)
        assert np.all(r["steps"] == 1)


def _brute_force_first_addition(A, k, m0):
    """Index added to J_k = {k} by one augmentation with beta = 1: every
    candidate j's residual min over mu of ||s + mu a_j||_2 by a dense least
    squares solve, rounded to fp32, mean filter, smallest (rho, j)."""
    D = A.dense()
    s = m0 * D[k, :]  # row k of M A with M(k, :) = m0 e_k^T
    s[k] -= 1.0
    support = np.flatnonzero(np.abs(s) > 2.0 ** -40)
    cands = sorted(set(np.flatnonzero(D[:, support].any(axis=1))) - {k})
    if not cands:
        return None, []
    rho = []
    for j in cands:
        a = D[j, :][:, None]
        mu = np.linalg.lstsq(a, -s, rcond=None)[0]
        rho.append(np.float32(np.linalg.norm(s + (a @ mu))))
    rho = np.array(rho, dtype=np.float32)
    mean = rho.astype(np.float64).sum() / len(rho)
    acc = [(float(r), j) for r, j in zip(rho, cands) if float(r) <= mean]
    acc.sort()
    return acc[0][1], acc


def test_first_addition_matches_brute_force_univariate_minimisation():
    rng = np.random.default_rng(61)
    A = W.random_sparse(40, 0.12, rng, dominance=0.6)
    r0 = O.spai_adaptive(A, alpha=0)
    r1 = O.spai_adaptive(A, alpha=1, beta=1, eps=0.0)
    assert r1["status"] == O.OK
    checked = 0
    for k in range(A.n):
        j_bf, acc = _brute_force_first_addition(A, k, r0["M"].val[k])
        s, e = r1["M"].row_ptr[k], r1["M"].row_ptr[k + 1]
        if j_bf is None:  # no candidate: nothing added
            assert list(r1["M"].col[s:e]) == [k]
            continue
        # skip rows whose two best candidates tie within rounding of the fp32 rho
        if len(acc) > 1 and abs(acc[1][0] - acc[0][0]) <= 4 * np.spacing(np.float32(acc[0][0])):
            continue
        assert sorted(r1["M"].col[s:e]) == sorted([k, j_bf]), k
        checked += 1
    assert checked >= 30


def test_residual_never_grows_with_more_rounds():
    A = _stencil()
    prev = None
    for alpha in range(4):
        r = O.spai_adaptive(A, alpha=alpha, beta=4, eps=0.0)
        assert r["status"] == O.OK
        res = _row_residuals(A, r["M"])
        if prev is not None:
            assert np.all(res <= prev * (1 + 1e-12) + 1e-14)
        prev = res


def test_full_pattern_gives_the_inverse():
    rng = np.random.default_rng(62)
    D = rng.standard_normal((8, 8)) + 8 * np.eye(8)
    A = W.from_dense(D, np.ones((8, 8), bool))
    r = O.spai_adaptive(A, alpha=8, beta=8, eps=0.0)
    assert r["status"] == O.OK and r["M"].nnz == 64
    assert np.abs(r["M"].dense() @ D - np.eye(8)).max() <= 1e-12


def test_rows_stopping_early_meet_the_tolerance():
    A = _stencil()
    eps, alpha, beta = 0.3, 5, 8
    r = O.spai_adaptive(A, alpha=alpha, beta=beta, eps=eps)
    res = _row_residuals(A, r["M"])
    lens = np.diff(r["M"].row_ptr)
    early = r["steps"] < alpha + 1
    # a row stops early on the tolerance or when no candidate is acceptable;
    # the second needs the pattern to have stopped growing
    assert np.all((res[early] <= eps * (1 + 1e-12)) | (lens[early] < 1 + beta * (r["steps"][early] - 1) + 1))
    assert np.mean(res[early] <= eps) > 0.9
    assert np.all(lens <= 1 + alpha * beta)


@pytest.mark.parametrize("uf", [O.FP32, O.FP16])
def test_adaptive_in_a_lower_construction_precision(uf):
    """Table 4's setting, the SPAI built in single (or half) precision: every
    row's values are the u_f least squares solution on the pattern the row
    ended with (the fixed-pattern u_f construction, pinned on its own against
    IEEE scalar arithmetic), bit for bit, and are u_f numbers; most rows find
    the FP64 build's pattern (the decisions see only u_f's effect on the
    fit)."""
    A = W.config("2", small=True)["A"]
    ref = O.spai_adaptive(A, alpha=5, beta=8, eps=0.4)
    r = O.spai_adaptive(A, alpha=5, beta=8, eps=0.4, uf=uf, scale=True)
    assert ref["status"] == r["status"] == O.OK
    M = r["M"]
    st, Mv, _ = O.spai(A, M.pattern(), scale=True, uf=uf)
    assert st == O.OK and np.array_equal(Mv, M.val)
    assert np.array_equal(O.round_to(uf, M.val), M.val)
    same = [np.array_equal(M.col[M.row_ptr[k]:M.row_ptr[k + 1]], ref["M"].col[ref["M"].row_ptr[k]:ref["M"].row_ptr[k + 1]])
            for k in range(A.n)]
    assert np.mean(same) >= 0.9, np.mean(same)
    # where the patterns agree the values agree to the construction precision
    u = 2.0 ** -24 if uf == O.FP32 else 2.0 ** -11
    for k in np.flatnonzero(same)[:200]:
        a, b = M.val[M.row_ptr[k]:M.row_ptr[k + 1]], ref["M"].val[ref["M"].row_ptr[k]:ref["M"].row_ptr[k + 1]]
        assert np.abs(a - b).max() <= 200 * u * np.abs(b).max(), k


def test_adaptive_half_precision_overflow_without_scaling():
    """Entries of 1e5 exceed fp16's 65,504: unscaled, the half-precision
    least squares overflow and the build reports ENAN; scaled, it succeeds."""
    rng = np.random.default_rng(91)
    A = W.random_sparse(120, 0.05, rng, dominance=0.8)
    A = W.CSR(A.n, A.row_ptr, A.col, A.val * 1e5)
    assert O.spai_adaptive(A, alpha=2, beta=4, eps=0.1, uf=O.FP16)["status"] == O.ENAN
    assert O.spai_adaptive(A, alpha=2, beta=4, eps=0.1, uf=O.FP16, scale=True)["status"] == O.OK


def test_adaptive_fp64_scaling_changes_little():
    """Column scaling in FP64 only changes the rounding of each solve."""
    A = W.config("2", small=True)["A"]
    a = O.spai_adaptive(A, alpha=3, beta=4, eps=0.2)
    b = O.spai_adaptive(A, alpha=3, beta=4, eps=0.2, scale=True)
    assert np.array_equal(a["M"].col, b["M"].col)
    assert np.abs(a["M"].val - b["M"].val).max() <= 1e-10 * np.abs(a["M"].val).max()

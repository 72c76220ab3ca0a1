"""Seeded synthetic inputs for the BSPAI-GMRES-IR workloads.

This module only constructs inputs: sparse matrices in CSR form, the sparsity
patterns handed to the SPAI construction, right-hand sides and reference
solutions.  It holds none of the method's arithmetic (no SPAI, no bucketing, no
Krylov or refinement step), so both the CPU oracle's tests and the HIP path can
draw the same inputs from it.

The paper evaluates on SuiteSparse matrices (Section 4, Table 1) that are not
available here; the generators below stand in for them with PDE stencils and a
power-law random matrix whose shapes, sizes and value ranges are stated in each
docstring.  Every generator is deterministic in its seed.

CSR convention everywhere: 0-based, int32 ``row_ptr`` (n+1) and ``col`` (nnz)
with column indices sorted ascending inside each row, float64 ``val``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np
import scipy.sparse as sp

# Precision identifiers shared by the C interface and the oracle (interface
# numbering; each side defines its own constants with these values).
FP64, FP32, FP16, BF16, FP8, DROP = 0, 1, 2, 3, 4, 5
PREC_NAMES = {FP64: "fp64", FP32: "fp32", FP16: "fp16", BF16: "bf16", FP8: "fp8_e4m3", DROP: "drop"}


@dataclasses.dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray  # int32 [nnz]
    val: Optional[np.ndarray]  # float64 [nnz] or None for a pattern

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        v = self.val if self.val is not None else np.ones(self.nnz)
        return sp.csr_matrix((v, self.col, self.row_ptr), shape=(self.n, self.n))

    def pattern(self) -> "CSR":
        return CSR(self.n, self.row_ptr.copy(), self.col.copy(), None)

    def dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


def from_scipy(M, keep_values: bool = True) -> CSR:
    M = sp.csr_matrix(M)
    M.sum_duplicates()
    M.sort_indices()
    n = M.shape[0]
    assert M.shape == (n, n)
    return CSR(
        n,
        M.indptr.astype(np.int32),
        M.indices.astype(np.int32),
        M.data.astype(np.float64) if keep_values else None,
    )


def from_dense(D: np.ndarray, pattern: Optional[np.ndarray] = None) -> CSR:
    """CSR of a dense matrix; ``pattern`` (bool) keeps explicit entries."""
    D = np.asarray(D, dtype=np.float64)
    n = D.shape[0]
    mask = (D != 0) if pattern is None else np.asarray(pattern, dtype=bool)
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return CSR(n, row_ptr, cols.astype(np.int32), D[rows, cols].copy())


# ---------------------------------------------------------------- stencils


def poisson2d(m: int) -> CSR:
    """5-point Laplacian on an m x m grid, Dirichlet, lexicographic order.

    Diagonal 4, neighbours -1 (the h^2-scaled operator); nnz = 5 m^2 - 4 m.
    """
    return convdiff2d(m, wx=0.0, wy=0.0)


def convdiff2d(m: int, peclet: float = 50.0, wx: Optional[float] = None,
               wy: Optional[float] = None, cell_peclet: bool = False) -> CSR:
    """First-order upwind convection-diffusion on the unit square.

    -nu Lap(u) + w . grad(u), nu = 1, h = 1/(m+1), wind w = |w| (1,1)/sqrt(2)
    with |w| = ``peclet`` (global Peclet number |w| L / nu with L = 1).  With
    ``cell_peclet`` the wind is scaled so that the cell Peclet |w| h / nu equals
    ``peclet``.  Scaled by h^2: diagonal 4 + h (wx + wy), west -1 - h wx,
    south -1 - h wy, east = north = -1.  Nonsymmetric for w != 0.
    """
    h = 1.0 / (m + 1)
    if wx is None or wy is None:
        mag = peclet / h if cell_peclet else peclet
        wx = wy = mag / math.sqrt(2.0)
    n = m * m
    idx = np.arange(n)
    ix, iy = idx % m, idx // m
    rows, cols, vals = [idx], [idx], [np.full(n, 4.0 + h * (wx + wy))]
    for dx, dy, c in ((-1, 0, -1.0 - h * wx), (1, 0, -1.0), (0, -1, -1.0 - h * wy), (0, 1, -1.0)):
        ok = (ix + dx >= 0) & (ix + dx < m) & (iy + dy >= 0) & (iy + dy < m)
        rows.append(idx[ok])
        cols.append(idx[ok] + dx + dy * m)
        vals.append(np.full(int(ok.sum()), c))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return from_scipy(A)


def aniso3d(m: int, cx: float = 1.0, cy: float = 10.0, cz: float = 100.0) -> CSR:
    """7-point anisotropic diffusion on an m^3 Dirichlet grid (h^2-scaled).

    Diagonal 2 (cx + cy + cz), x/y/z neighbours -cx/-cy/-cz; lexicographic
    index (iz m + iy) m + ix; nnz = 7 m^3 - 6 m^2.
    """
    n = m ** 3
    idx = np.arange(n, dtype=np.int64)
    ix, iy, iz = idx % m, (idx // m) % m, idx // (m * m)
    rows, cols, vals = [idx], [idx], [np.full(n, 2.0 * (cx + cy + cz))]
    for d, stride, c in ((ix, 1, cx), (iy, m, cy), (iz, m * m, cz)):
        for s in (-1, 1):
            ok = (d + s >= 0) & (d + s < m)
            rows.append(idx[ok])
            cols.append(idx[ok] + s * stride)
            vals.append(np.full(int(ok.sum()), -c))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return from_scipy(A)


def grf2d(m: int, ell: float, rng: np.random.Generator) -> np.ndarray:
    """Gaussian random field on an m x m grid with covariance exp(-r^2 / (2 ell^2)).

    White noise convolved (FFT, on a grid padded by 4 ell per side) with a
    Gaussian of standard deviation ell / sqrt(2), cropped, then shifted and
    scaled to zero sample mean and unit sample standard deviation.
    """
    pad = int(math.ceil(4 * ell))
    N = m + 2 * pad
    w = rng.standard_normal((N, N))
    s = ell / math.sqrt(2.0)
    k = np.fft.fftfreq(N)
    kx, ky = np.meshgrid(k, k, indexing="ij")
    # Fourier transform of a unit-mass Gaussian of std s (in cells).
    G = np.exp(-2.0 * (math.pi ** 2) * (s ** 2) * (kx ** 2 + ky ** 2))
    f = np.real(np.fft.ifft2(np.fft.fft2(w) * G))[pad:pad + m, pad:pad + m]
    f = f - f.mean()
    return f / f.std()


def vardiff2d(kcell: np.ndarray) -> CSR:
    """Cell-centred 5-point diffusion -div(k grad u) on an m x m grid (h^2-scaled).

    Interior faces take the harmonic mean 2 k_a k_b / (k_a + k_b); a boundary
    face takes the cell's own k with a zero Dirichlet ghost value.  Diagonal is
    the sum of the four face coefficients, off-diagonals their negatives (SPD).
    """
    m = kcell.shape[0]
    n = m * m
    kc = kcell.reshape(-1)
    idx = np.arange(n)
    ix, iy = idx % m, idx // m
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        ok = (ix + dx >= 0) & (ix + dx < m) & (iy + dy >= 0) & (iy + dy < m)
        nb = idx + dx + dy * m
        kf = np.where(ok, 2.0 * kc * kc[np.where(ok, nb, idx)] / (kc + kc[np.where(ok, nb, idx)]), kc)
        diag += kf
        rows.append(idx[ok])
        cols.append(nb[ok])
        vals.append(-kf[ok])
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return from_scipy(A)


# ---------------------------------------------------------------- random


def _powerlaw_gamma(lmin: int, lmax: int, mean: float) -> float:
    ls = np.arange(lmin, lmax + 1, dtype=np.float64)

    def mean_of(g):
        p = ls ** (-g)
        return float((ls * p).sum() / p.sum())

    lo, hi = 0.0, 10.0  # mean_of is decreasing in g
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mean_of(mid) > mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def powerlaw_random(n: int, rng: np.random.Generator, mean: float = 12.0, lmin: int = 3,
                    lmax: int = 400, sigma: float = 4.0, dominance: float = 1.1) -> CSR:
    """Random nonsymmetric matrix with power-law row lengths and a dominant diagonal.

    Off-diagonal row lengths follow a truncated discrete power law
    P(l) ~ l^-gamma on [lmin, lmax] with gamma solved so the mean is ``mean``.
    Columns are uniform over j != i (duplicates discarded), magnitudes are
    lognormal(0, sigma) with random signs, and a_ii = dominance * sum_j |a_ij|.
    """
    gamma = _powerlaw_gamma(lmin, lmax, mean)
    ls = np.arange(lmin, lmax + 1)
    p = ls.astype(np.float64) ** (-gamma)
    p /= p.sum()
    lens = rng.choice(ls, size=n, p=p).astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    cols = rng.integers(0, n - 1, size=rows.size, dtype=np.int64)
    cols = cols + (cols >= rows)  # uniform over j != i
    key = np.unique(rows * n + cols)
    rows, cols = key // n, key % n
    mag = np.exp(sigma * rng.standard_normal(rows.size))
    sign = np.where(rng.random(rows.size) < 0.5, -1.0, 1.0)
    vals = mag * sign
    rowsum = np.bincount(rows, weights=np.abs(vals), minlength=n)
    diag = dominance * rowsum
    diag[diag == 0] = 1.0
    A = sp.coo_matrix((np.concatenate([vals, diag]),
                       (np.concatenate([rows, np.arange(n)]), np.concatenate([cols, np.arange(n)]))),
                      shape=(n, n))
    return from_scipy(A)


def random_sparse(n: int, density: float, rng: np.random.Generator, dominance: float = 2.0,
                  symmetric_pattern: bool = False) -> CSR:
    """Small random sparse test matrix with a nonzero diagonal (tests only)."""
    mask = rng.random((n, n)) < density
    if symmetric_pattern:
        mask = mask | mask.T
    np.fill_diagonal(mask, True)
    D = np.where(mask, rng.standard_normal((n, n)), 0.0)
    np.fill_diagonal(D, 0.0)
    d = dominance * np.abs(D).sum(axis=1)
    d[d == 0] = 1.0
    np.fill_diagonal(D, d * np.where(rng.random(n) < 0.5, -1.0, 1.0))
    return from_dense(D, mask)


# ---------------------------------------------------------------- patterns, RHS


def pattern_power(A: CSR, k: int) -> CSR:
    """Sparsity pattern of A^k (structural)."""
    S = sp.csr_matrix((np.ones(A.nnz), A.col, A.row_ptr), shape=(A.n, A.n))
    P = S
    for _ in range(k - 1):
        P = P @ S
        P.data[:] = 1.0
    return from_scipy(P, keep_values=False)


def identity_pattern(n: int) -> CSR:
    return CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), None)


def full_pattern(n: int) -> CSR:
    return CSR(n, (np.arange(n + 1) * n).astype(np.int32), np.tile(np.arange(n, dtype=np.int32), n), None)


def matvec_extended(A: CSR, x: np.ndarray) -> np.ndarray:
    """y = A x accumulated in extended (x87 long double) precision, rounded to fp64."""
    prod = A.val.astype(np.longdouble) * x[A.col].astype(np.longdouble)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    acc = np.zeros(A.n, dtype=np.longdouble)
    np.add.at(acc, rows, prod)
    return acc.astype(np.float64)


# ---------------------------------------------------------------- named workloads


def _sorted_precs(ps: List[int]) -> List[int]:
    order = [FP64, FP32, FP16, BF16, FP8, DROP]
    return sorted(ps, key=order.index)


def config(k: str, small: bool = False, seed: Optional[int] = None) -> Dict:
    """Named workload.  ``k`` in {"1", "2", "3", "4a", "4b", "5"}.

    ``small`` selects a scaled-down instance of the same family (used where the
    oracle must finish in seconds).  Returned dict keys: A (CSR), P (pattern
    CSR), b (float64 [n] or [n, nrhs]), x_true (or None), precs (sorted ints),
    eps (list of bucketing targets), name, plus family-specific extras.
    """
    if k == "1":
        s = 1 if seed is None else seed
        m = 32 if not small else 12
        A = poisson2d(m)
        rng = np.random.default_rng(s)
        x = rng.standard_normal(A.n)
        return dict(name=f"poisson2d_{m}x{m}", A=A, P=A.pattern(), b=matvec_extended(A, x), x_true=x,
                    precs=[FP64], eps=[2.0 ** -53], grid=m)
    if k == "2":
        s = 2 if seed is None else seed
        m = 256 if not small else 40
        A = convdiff2d(m, peclet=50.0)
        rng = np.random.default_rng(s)
        x = rng.standard_normal(A.n)
        return dict(name=f"convdiff2d_{m}x{m}_pe50", A=A, P=pattern_power(A, 2), b=matvec_extended(A, x),
                    x_true=x, precs=_sorted_precs([FP64, FP32, BF16, FP16]), eps=[1e-6, 1e-4, 1e-2], grid=m)
    if k == "3":
        s = 3 if seed is None else seed
        n = 1 << 20 if not small else 6000
        rng = np.random.default_rng(s)
        A = powerlaw_random(n, rng, lmax=400 if not small else 120)
        b = rng.uniform(-1.0, 1.0, size=n)
        return dict(name=f"powerlaw_n{n}", A=A, P=A.pattern(), b=b, x_true=None,
                    precs=_sorted_precs([FP64, FP32, FP16, FP8]), eps=[1e-3])
    if k == "4a":
        s = 41 if seed is None else seed
        m = 128 if not small else 16
        nrhs = 64 if not small else 8
        A = aniso3d(m)
        rng = np.random.default_rng(s)
        B = rng.standard_normal((A.n, nrhs))
        return dict(name=f"aniso3d_{m}^3_rhs{nrhs}", A=A, P=A.pattern(), b=B, x_true=None,
                    precs=_sorted_precs([FP32, FP16, BF16]), eps=[1e-2], grid=m, nrhs=nrhs)
    if k == "4b":
        s = 42 if seed is None else seed
        rng = np.random.default_rng(s)
        nsys = 32 if not small else 4
        lo, hi = (32, 448) if not small else (12, 40)
        sides = rng.integers(lo, hi + 1, size=nsys)
        systems = []
        for i, m in enumerate(sides):
            r = np.random.default_rng([s, i])
            theta = grf2d(int(m), 16.0 if not small else 4.0, r)
            A = vardiff2d(np.exp(theta))
            systems.append(dict(A=A, P=A.pattern(), b=r.standard_normal(A.n), grid=int(m)))
        return dict(name=f"multisys_{nsys}", systems=systems, precs=_sorted_precs([FP32, FP16, BF16]), eps=[1e-2])
    if k == "5":
        s = 5 if seed is None else seed
        m = 512 if not small else 32
        ell = 16.0 if not small else 4.0
        rng = np.random.default_rng(s)
        theta = grf2d(m, ell, rng)
        theta_p = grf2d(m, ell, rng)
        h = 1.0 / (m + 1)
        A = vardiff2d(np.exp(theta))
        return dict(name=f"vardiff2d_{m}x{m}", A=A, P=A.pattern(), b=np.full(A.n, h * h), x_true=None,
                    theta=theta, theta_obs=theta + 0.1 * theta_p, precs=_sorted_precs([FP64, FP32, FP16, BF16, FP8]),
                    eps=[1e-3], grid=m)
    raise ValueError(f"unknown workload {k!r}")

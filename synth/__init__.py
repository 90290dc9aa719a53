"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module builds matrices and right-hand sides only.  It holds none of the
method's arithmetic (no factorization, no solve, no level scheduling): every
function returns plain CSR arrays ``(row_ptr int32, col_idx int32, val float64)``
with sorted, unique columns per row, plus the sizes, so that the CPU oracle and
the HIP path both read identical bytes.

Workloads (natural ordering, x fastest: r = i + nx*j + nx*ny*k):

* ``laplace2d(nx, ny)``          5-point Laplacian, diagonal 4, -1 per in-grid neighbour.
* ``laplace3d(nx, ny, nz)``      7-point Laplacian, diagonal 6, -1 per in-grid neighbour.
* ``convdiff3d(m, pe)``          first-order upwind convection-diffusion on an m^3 grid,
                                 scaled by h^2/nu; cell Peclet numbers pe = (pe_x, pe_y, pe_z).
* ``random_banded(n, ...)``      random unsymmetric rows: ``band`` columns uniform within
                                 +-``halfwidth`` of the diagonal plus ``rnd`` uniform columns,
                                 N(0,1) off-diagonals, diagonal = 1.1 * sum |off-diagonals|.
* ``diffusion2d_varcoef(...)``   5-point finite-volume diffusion with log-normal cell
                                 coefficients, harmonic face means, Dirichlet boundary faces.
* ``batch_diffusion2d(...)``     a batch of the above with log-uniform grid sides.

Small families for tests: ``tridiag``, ``dense_pattern``, ``banded``, ``random_sparse``,
``integer_unit_lower``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "CSR", "laplace2d", "laplace3d", "convdiff3d", "random_banded", "diffusion2d_varcoef",
    "batch_diffusion2d", "tridiag", "dense_pattern", "banded", "random_sparse",
    "integer_unit_lower", "rhs", "workload", "WORKLOADS", "csr_to_dense", "csr_from_coo",
]


class CSR:
    """Plain CSR triple with its dimension."""

    __slots__ = ("n", "row_ptr", "col_idx", "val")

    def __init__(self, n, row_ptr, col_idx, val):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def __repr__(self):
        return f"CSR(n={self.n}, nnz={self.nnz})"


def csr_from_coo(n, rows, cols, vals) -> CSR:
    """Sorts (row, col) pairs and builds CSR; duplicate pairs are not allowed."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if rows.size > 1:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if dup.any():
            raise ValueError("duplicate entries in COO input")
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    return CSR(n, row_ptr, cols, vals)


def csr_to_dense(A: CSR) -> np.ndarray:
    D = np.zeros((A.n, A.n))
    for i in range(A.n):
        s, e = A.row_ptr[i], A.row_ptr[i + 1]
        D[i, A.col_idx[s:e]] = A.val[s:e]
    return D


# --------------------------------------------------------------------------------------
# Structured stencils
# --------------------------------------------------------------------------------------

def _stencil(dims, diag, offsets):
    """Generic constant-coefficient stencil on a box grid in natural ordering.

    ``offsets`` is a list of (axis, step, value); a neighbour outside the box is dropped
    (Dirichlet boundary eliminated).  ``diag`` is a scalar or a per-row array.
    """
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for d in dims:
        coords.append(rem % d)
        rem //= d
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    rows_l, cols_l, vals_l = [idx], [idx], [np.broadcast_to(np.asarray(diag, dtype=np.float64), (n,))]
    for axis, step, value in offsets:
        c = coords[axis] + step
        ok = (c >= 0) & (c < dims[axis])
        r = idx[ok]
        rows_l.append(r)
        cols_l.append(r + step * strides[axis])
        vals_l.append(np.full(r.size, value, dtype=np.float64))
    rows = np.concatenate(rows_l)
    cols = np.concatenate(cols_l)
    vals = np.concatenate(vals_l)
    return csr_from_coo(n, rows, cols, vals)


def laplace2d(nx: int, ny: int | None = None) -> CSR:
    ny = nx if ny is None else ny
    offs = [(0, -1, -1.0), (0, 1, -1.0), (1, -1, -1.0), (1, 1, -1.0)]
    return _stencil((nx, ny), 4.0, offs)


def laplace3d(nx: int, ny: int | None = None, nz: int | None = None) -> CSR:
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    offs = [(a, s, -1.0) for a in range(3) for s in (-1, 1)]
    return _stencil((nx, ny, nz), 6.0, offs)


def convdiff3d(m: int, pe=(10.0, 5.0, 2.5)) -> CSR:
    """Upwind convection-diffusion with positive velocity, scaled by h^2/nu.

    Diffusion gives 6 on the diagonal and -1 per neighbour; first-order upwind
    convection with cell Peclet number pe_d adds pe_d to the diagonal and -pe_d to
    the upstream (lower-index) neighbour along axis d.
    """
    px, py, pz = (float(p) for p in pe)
    diag = 6.0 + px + py + pz
    offs = [
        (0, -1, -1.0 - px), (0, 1, -1.0),
        (1, -1, -1.0 - py), (1, 1, -1.0),
        (2, -1, -1.0 - pz), (2, 1, -1.0),
    ]
    return _stencil((m, m, m), diag, offs)


# --------------------------------------------------------------------------------------
# Random unsymmetric banded + scattered
# --------------------------------------------------------------------------------------

def random_banded(n: int, band: int = 8, rnd: int = 8, halfwidth: int = 64,
                  rng: np.random.Generator | None = None, chunk: int = 131072) -> CSR:
    """Random unsymmetric matrix with a strictly diagonally dominant diagonal.

    Row i gets ``band`` distinct columns drawn uniformly from
    [i-halfwidth, i+halfwidth] intersect [0, n) minus {i}, then ``rnd`` distinct columns
    drawn uniformly from [0, n) avoiding the band columns and i (collisions are
    redrawn).  Off-diagonal values are N(0,1); the diagonal is 1.1 * sum |off|.
    """
    rng = np.random.default_rng(0) if rng is None else rng
    if 2 * halfwidth < band:
        raise ValueError("band wider than the window")
    offsets = np.concatenate([np.arange(-halfwidth, 0), np.arange(1, halfwidth + 1)])
    per_row = band + rnd
    cols_all = np.empty((n, per_row), dtype=np.int64)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        rows = np.arange(s, e, dtype=np.int64)
        cand = rows[:, None] + offsets[None, :]
        keys = rng.random(cand.shape, dtype=np.float32)
        keys[(cand < 0) | (cand >= n)] = np.inf
        pick = np.argpartition(keys, band - 1, axis=1)[:, :band]
        bcols = np.take_along_axis(cand, pick, axis=1)
        if np.isinf(np.take_along_axis(keys, pick, axis=1)).any():
            raise ValueError("window too small for the band count near the boundary")
        rcols = rng.integers(0, n, size=(e - s, rnd), dtype=np.int64)
        while True:
            bad = (rcols == rows[:, None])
            bad |= (rcols[:, :, None] == bcols[:, None, :]).any(axis=2)
            # duplicates among the random columns: keep the first occurrence
            for j in range(1, rnd):
                bad[:, j] |= (rcols[:, :j] == rcols[:, j:j + 1]).any(axis=1)
            if not bad.any():
                break
            nb = int(bad.sum())
            rcols[bad] = rng.integers(0, n, size=nb, dtype=np.int64)
        cols_all[s:e, :band] = bcols
        cols_all[s:e, band:] = rcols
    off = rng.standard_normal((n, per_row))
    diag = 1.1 * np.abs(off).sum(axis=1)
    cols = np.concatenate([cols_all, np.arange(n, dtype=np.int64)[:, None]], axis=1)
    vals = np.concatenate([off, diag[:, None]], axis=1)
    # every row holds exactly per_row + 1 distinct columns: sort within rows
    order = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    row_ptr = np.arange(n + 1, dtype=np.int64) * (per_row + 1)
    return CSR(n, row_ptr, cols.ravel(), vals.ravel())


def heavy_rows(n: int, light: int = 4, halfwidth: int = 16, heavy_frac: float = 0.01,
               heavy_len: tuple = (256, 2048), rng: np.random.Generator | None = None) -> CSR:
    """Irregular rows: every row couples to ``light`` distinct columns drawn uniformly
    from [i-halfwidth, i+halfwidth] minus {i}; a fraction ``heavy_frac`` of the rows
    (each row independently) also gets L ~ U[heavy_len] columns uniform over [0, n)
    (repeats merged), the long rows of circuit-like matrices.  Off-diagonal values
    N(0,1); diagonal 1.2 * sum |off| + 1 (strict row dominance)."""
    rng = np.random.default_rng(0) if rng is None else rng
    offsets = np.concatenate([np.arange(-halfwidth, 0), np.arange(1, halfwidth + 1)])
    rows_i = np.arange(n, dtype=np.int64)
    cand = rows_i[:, None] + offsets[None, :]
    keys = rng.random(cand.shape, dtype=np.float32)
    keys[(cand < 0) | (cand >= n)] = np.inf
    k = min(light, 2 * halfwidth)
    pick = np.argpartition(keys, k - 1, axis=1)[:, :k]
    lc = np.take_along_axis(cand, pick, axis=1)
    ok = np.isfinite(np.take_along_axis(keys, pick, axis=1))
    r_parts = [np.repeat(rows_i, k)[ok.ravel()]]
    c_parts = [lc.ravel()[ok.ravel()]]
    heavy = np.flatnonzero(rng.random(n) < heavy_frac)
    lens = rng.integers(heavy_len[0], heavy_len[1] + 1, size=heavy.size)
    lens = np.minimum(lens, n - 1)
    r_parts.append(np.repeat(heavy, lens))
    c_parts.append(rng.integers(0, n, size=int(lens.sum()), dtype=np.int64))
    r = np.concatenate(r_parts)
    c = np.concatenate(c_parts)
    off = r != c
    key = np.unique(r[off] * n + c[off])
    r, c = key // n, key % n
    v = rng.standard_normal(r.size)
    dsum = np.bincount(r, weights=np.abs(v), minlength=n)
    r = np.concatenate([r, rows_i])
    c = np.concatenate([c, rows_i])
    v = np.concatenate([v, 1.2 * dsum + 1.0])
    return csr_from_coo(n, r, c, v)


# --------------------------------------------------------------------------------------
# Variable-coefficient diffusion (finite volume) and its batch
# --------------------------------------------------------------------------------------

def diffusion2d_varcoef(nx: int, ny: int, kappa: np.ndarray) -> CSR:
    """5-point finite-volume diffusion, cell coefficients kappa[j, i] (shape (ny, nx)).

    Interior face coefficient: harmonic mean 2 ka kb / (ka + kb).  Each boundary face of
    a cell adds 2 kappa_c to its diagonal (Dirichlet value at the face).  The matrix is
    a symmetric M-matrix.
    """
    kappa = np.asarray(kappa, dtype=np.float64).reshape(ny, nx)
    n = nx * ny
    idx = np.arange(n, dtype=np.int64).reshape(ny, nx)
    diag = np.zeros((ny, nx))
    rows_l, cols_l, vals_l = [], [], []
    # x faces
    kf = 2.0 * kappa[:, :-1] * kappa[:, 1:] / (kappa[:, :-1] + kappa[:, 1:])
    diag[:, :-1] += kf
    diag[:, 1:] += kf
    rows_l += [idx[:, :-1].ravel(), idx[:, 1:].ravel()]
    cols_l += [idx[:, 1:].ravel(), idx[:, :-1].ravel()]
    vals_l += [-kf.ravel(), -kf.ravel()]
    # y faces
    kf = 2.0 * kappa[:-1, :] * kappa[1:, :] / (kappa[:-1, :] + kappa[1:, :])
    diag[:-1, :] += kf
    diag[1:, :] += kf
    rows_l += [idx[:-1, :].ravel(), idx[1:, :].ravel()]
    cols_l += [idx[1:, :].ravel(), idx[:-1, :].ravel()]
    vals_l += [-kf.ravel(), -kf.ravel()]
    # boundary faces
    diag[:, 0] += 2.0 * kappa[:, 0]
    diag[:, -1] += 2.0 * kappa[:, -1]
    diag[0, :] += 2.0 * kappa[0, :]
    diag[-1, :] += 2.0 * kappa[-1, :]
    rows_l.append(idx.ravel())
    cols_l.append(idx.ravel())
    vals_l.append(diag.ravel())
    return csr_from_coo(n, np.concatenate(rows_l), np.concatenate(cols_l), np.concatenate(vals_l))


def batch_diffusion2d(count: int = 512, side_lo: int = 32, side_hi: int = 256,
                      rng: np.random.Generator | None = None):
    """``count`` variable-coefficient diffusion matrices with log-uniform grid sides.

    nx and ny are drawn independently as round(exp(U[ln lo, ln hi])); cell
    coefficients are exp(N(0,1)).  Returns a list of CSR.
    """
    rng = np.random.default_rng(0) if rng is None else rng
    mats = []
    lo, hi = np.log(side_lo), np.log(side_hi)
    for _ in range(count):
        nx = int(np.rint(np.exp(rng.uniform(lo, hi))))
        ny = int(np.rint(np.exp(rng.uniform(lo, hi))))
        kappa = np.exp(rng.standard_normal((ny, nx)))
        mats.append(diffusion2d_varcoef(nx, ny, kappa))
    return mats


# --------------------------------------------------------------------------------------
# Small families for tests
# --------------------------------------------------------------------------------------

def tridiag(n: int, lo=-1.0, d=2.0, up=-1.0) -> CSR:
    rows = np.concatenate([np.arange(1, n), np.arange(n), np.arange(n - 1)])
    cols = np.concatenate([np.arange(0, n - 1), np.arange(n), np.arange(1, n)])
    vals = np.concatenate([np.full(n - 1, lo), np.full(n, d), np.full(n - 1, up)])
    return csr_from_coo(n, rows, cols, vals)


def dense_pattern(n: int, rng: np.random.Generator) -> CSR:
    """Full pattern, column diagonally dominant (partial pivoting would not swap)."""
    M = rng.uniform(-1.0, 1.0, size=(n, n))
    np.fill_diagonal(M, 0.0)
    colsum = np.abs(M).sum(axis=0)
    M[np.arange(n), np.arange(n)] = colsum + 1.0 + rng.uniform(0, 1, size=n)
    r, c = np.nonzero(np.ones((n, n)))
    return csr_from_coo(n, r, c, M[r, c])


def banded(n: int, p: int, rng: np.random.Generator) -> CSR:
    """Full band |i-j| <= p, diagonally dominant by rows and columns."""
    r, c = np.nonzero(np.abs(np.subtract.outer(np.arange(n), np.arange(n))) <= p)
    v = rng.uniform(-1.0, 1.0, size=r.size)
    v[r == c] = 0.0
    D = np.zeros((n, n))
    D[r, c] = v
    dom = np.maximum(np.abs(D).sum(axis=0), np.abs(D).sum(axis=1)) + 1.0
    v[r == c] = dom[r[r == c]]
    return csr_from_coo(n, r, c, v)


def random_sparse(n: int, density: float, rng: np.random.Generator, symmetric_pattern=False,
                  diag_dominant=True, drop_diag_frac: float = 0.0) -> CSR:
    """Random pattern with N(0,1) values; optional symmetric pattern; strong diagonal."""
    mask = rng.random((n, n)) < density
    if symmetric_pattern:
        mask = mask | mask.T
    np.fill_diagonal(mask, True)
    if drop_diag_frac > 0:
        drop = rng.random(n) < drop_diag_frac
        mask[np.arange(n)[drop], np.arange(n)[drop]] = False
    r, c = np.nonzero(mask)
    v = rng.standard_normal(r.size)
    if diag_dominant:
        D = np.zeros((n, n))
        D[r, c] = v
        off = np.abs(D).sum(axis=1) - np.abs(np.diag(D))
        on = r == c
        v[on] = np.sign(v[on] + 1e-300) * (off[r[on]] + 1.0)
    return csr_from_coo(n, r, c, v)


def integer_unit_lower(n: int, density: float, rng: np.random.Generator, amax: int = 2) -> CSR:
    """Unit lower-triangular matrix with small integer off-diagonals."""
    r, c = np.nonzero(np.tril(rng.random((n, n)) < density, -1))
    v = rng.integers(-amax, amax + 1, size=r.size).astype(np.float64)
    keep = v != 0
    r, c, v = r[keep], c[keep], v[keep]
    rr = np.concatenate([r, np.arange(n)])
    cc = np.concatenate([c, np.arange(n)])
    vv = np.concatenate([v, np.ones(n)])
    return csr_from_coo(n, rr, cc, vv)


# --------------------------------------------------------------------------------------
# The five named workloads
# --------------------------------------------------------------------------------------

def rhs(n: int, nrhs: int, rng: np.random.Generator) -> np.ndarray:
    """Right-hand sides ~ U[-1, 1], row-major [n][nrhs] (squeezed to [n] when nrhs == 1)."""
    b = rng.uniform(-1.0, 1.0, size=(n, nrhs))
    return b[:, 0].copy() if nrhs == 1 else b


WORKLOADS = {
    # id: (name, description)
    1: ("laplace2d_64", "2D 5-point Laplacian 64x64, ILU(0), PCG"),
    2: ("laplace3d_128", "3D 7-point Laplacian 128^3, ILU(0), PCG FP64 vs FP32 factors"),
    3: ("convdiff3d_96", "3D upwind convection-diffusion 96^3, ILU(1, 1e-3), FGMRES(30)"),
    4: ("random_1m", "random unsymmetric n=1e6, 16 off-diagonals/row, ILU(0), 16 RHS"),
    5: ("batch512_diffusion2d", "512 variable-coefficient 2D diffusion matrices, 4 RHS each"),
}


def workload(wid: int, scale: float = 1.0):
    """Matrix (or list of matrices) and RHS for workload ``wid``.

    ``scale`` < 1 shrinks the grid / size for quick tests while keeping the recipe.
    Seeds: default_rng([wid, 0]) for the matrix and default_rng([wid, 1]) for the RHS.
    """
    mrng = np.random.default_rng([wid, 0])
    brng = np.random.default_rng([wid, 1])
    if wid == 1:
        m = max(2, int(round(64 * scale)))
        A = laplace2d(m, m)
        return A, rhs(A.n, 1, brng)
    if wid == 2:
        m = max(2, int(round(128 * scale)))
        A = laplace3d(m, m, m)
        return A, rhs(A.n, 1, brng)
    if wid == 3:
        m = max(2, int(round(96 * scale)))
        A = convdiff3d(m)
        return A, rhs(A.n, 1, brng)
    if wid == 4:
        n = max(200, int(round(1_000_000 * scale)))
        A = random_banded(n, band=8, rnd=8, halfwidth=64, rng=mrng)
        return A, rhs(A.n, 16, brng)
    if wid == 5:
        count = max(1, int(round(512 * min(1.0, scale))))
        lo = max(4, int(round(32 * scale)))
        hi = max(lo, int(round(256 * scale)))
        mats = batch_diffusion2d(count, lo, hi, rng=mrng)
        return mats, [rhs(M.n, 4, brng) for M in mats]
    raise KeyError(wid)

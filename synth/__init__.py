"""Seeded synthetic inputs for the triangular-solve path.

This module builds problem matrices, right-hand sides, subdomain cuts and batch
size draws.  It holds none of the method's arithmetic (no factorization, no
level analysis, no solve): it only produces the inputs that both the oracle and
the GPU path consume.  Every generator is deterministic in its seed.

Workload shapes follow the paper's experiments: Example 1 of the numerical
results section uses a three-dimensional Poisson matrix with n = 1,000,000 and
6,940,000 non-zeros, which is exactly the unscaled 7-point Laplacian on a 100^3
grid with homogeneous Dirichlet boundaries (``poisson3d(100)``).  The other
inputs (heterogeneous coefficients, subdomain cuts, system-size draws) are
synthetic stand-ins with the structure stated in each docstring.

All matrices are returned as :class:`CSR` with int32 row pointers and column
indices, float64 values, rows sorted by ascending column index, natural grid
ordering ``idx = x + nx*(y + ny*z)``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR",
    "poisson2d",
    "poisson3d",
    "diffusion2d",
    "diffusion3d",
    "rhs",
    "subdomain_cuts",
    "grid_bisection",
    "batch_systems",
    "random_lower",
]


@dataclass
class CSR:
    """Compressed sparse row matrix (square, n x n)."""

    n: int
    rowptr: np.ndarray  # int32 [n+1]
    col: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        np.add.at(d, (rows, self.col), self.val)
        return d

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


def _from_coo(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CSR(n, rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


def _grid_faces(shape):
    """Yield (axis, lo_index, hi_index) arrays of interior faces of a grid."""
    idx = np.arange(int(np.prod(shape)), dtype=np.int64).reshape(shape[::-1])  # [z][y][x]
    ndim = len(shape)
    for axis in range(ndim):
        ax = ndim - 1 - axis  # numpy axis of grid direction `axis` (x is last)
        lo = np.take(idx, np.arange(0, idx.shape[ax] - 1), axis=ax).ravel()
        hi = np.take(idx, np.arange(1, idx.shape[ax]), axis=ax).ravel()
        yield axis, lo, hi


def _stencil_matrix(shape, kappa=None) -> CSR:
    """Finite-volume diffusion matrix on a 2D/3D grid with Dirichlet walls.

    With ``kappa is None`` this is the unscaled Laplacian: diagonal 2*dim, each
    neighbour -1.  With a cell field ``kappa`` (flattened, natural order) each
    interior face carries the harmonic mean 2*ka*kb/(ka+kb); a boundary face
    adds the cell's own kappa to the diagonal, so kappa == 1 reduces to the
    unscaled Laplacian.
    """
    n = int(np.prod(shape))
    ndim = len(shape)
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    if kappa is None:
        diag[:] = 2.0 * ndim
    else:
        # every cell has 2*ndim faces; boundary faces contribute kappa_c
        nfaces_int = np.zeros(n)
    for axis, lo, hi in _grid_faces(shape):
        if kappa is None:
            c = np.ones(lo.shape[0])
        else:
            ka, kb = kappa[lo], kappa[hi]
            c = 2.0 * ka * kb / (ka + kb)
            diag += np.bincount(lo, weights=c, minlength=n) + np.bincount(hi, weights=c, minlength=n)
            nfaces_int += np.bincount(lo, minlength=n) + np.bincount(hi, minlength=n)
        rows += [lo, hi]
        cols += [hi, lo]
        vals += [-c, -c]
    if kappa is not None:
        diag += (2.0 * ndim - nfaces_int) * kappa
    ar = np.arange(n, dtype=np.int64)
    rows.append(ar)
    cols.append(ar)
    vals.append(diag)
    return _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def poisson2d(nx: int, ny: int | None = None) -> CSR:
    """2D 5-point Laplacian (diag 4, neighbours -1), natural order."""
    ny = nx if ny is None else ny
    return _stencil_matrix((nx, ny))


def poisson3d(nx: int, ny: int | None = None, nz: int | None = None) -> CSR:
    """3D 7-point Laplacian (diag 6, neighbours -1), natural order.

    ``poisson3d(100)`` has n = 1,000,000 and nnz = 6,940,000, the matrix of the
    paper's first example.
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return _stencil_matrix((nx, ny, nz))


def _lognormal_field(n: int, sigma: float, seed: int) -> np.ndarray:
    z = np.random.default_rng(seed).standard_normal(n)
    return np.exp(sigma * z)


def diffusion2d(nx: int, ny: int | None, sigma: float, seed: int) -> CSR:
    """2D 5-point heterogeneous diffusion; cell kappa = exp(sigma * N(0,1))."""
    ny = nx if ny is None else ny
    return _stencil_matrix((nx, ny), _lognormal_field(nx * ny, sigma, seed))


def diffusion3d(nx: int, ny: int | None, nz: int | None, sigma: float, seed: int) -> CSR:
    """3D 7-point heterogeneous diffusion; cell kappa = exp(sigma * N(0,1))."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return _stencil_matrix((nx, ny, nz), _lognormal_field(nx * ny * nz, sigma, seed))


def rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Right-hand sides U[-1, 1], shape [n][nrhs] (RHS index fastest), float64."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (n, nrhs))


def subdomain_cuts(n: int, nsub: int, lo: int, hi: int, seed: int, max_draws: int = 100000):
    """Contiguous natural-order subdomains of uneven, seeded sizes.

    Sizes are ``lo + floor(Dirichlet(2,...,2) * (n - nsub*lo))`` with the last
    subdomain absorbing the rounding remainder; draws are rejected until every
    size is at most ``hi``.  Returns the owner array (int32 [n]) and the sizes.
    """
    if nsub * lo > n or nsub * hi < n:
        raise ValueError("infeasible subdomain size bounds")
    rng = np.random.default_rng(seed)
    spare = n - nsub * lo
    for _ in range(max_draws):
        w = rng.dirichlet(np.full(nsub, 2.0))
        sizes = lo + np.floor(w * spare).astype(np.int64)
        sizes[-1] += n - int(sizes.sum())
        if sizes.max() <= hi and sizes.min() >= lo:
            owner = np.repeat(np.arange(nsub, dtype=np.int32), sizes)
            return owner, sizes
    raise RuntimeError("no admissible subdomain cut found")


def grid_bisection(nx: int, ny: int, nz: int, nparts: int) -> np.ndarray:
    """Geometric partition of an nx x ny x nz grid (natural order
    idx = x + nx*(y + ny*z)) into ``nparts`` boxes by recursive coordinate
    bisection: the longest side of the current box (z, then y, then x on
    ties) is cut so that the two halves get cell counts in the ratio of the
    parts they receive (floor(parts/2) : the rest).  A stand-in for a graph
    partitioner's subdomains.  Returns the owner array (int32 [n])."""
    if nparts < 1 or nparts > nx * ny * nz:
        raise ValueError("bad number of parts")
    owner = np.empty((nz, ny, nx), dtype=np.int32)

    def rec(box, first, parts):
        if parts == 1:
            (z0, z1), (y0, y1), (x0, x1) = box
            owner[z0:z1, y0:y1, x0:x1] = first
            return
        ext = [hi - lo for lo, hi in box]
        ax = int(np.argmax(ext))
        if ext[ax] < 2:
            raise ValueError("more parts than the grid can be cut into")
        left = parts // 2
        lo, hi = box[ax]
        cut = lo + min(max(1, int(round(ext[ax] * left / parts))), ext[ax] - 1)
        a, b = list(box), list(box)
        a[ax], b[ax] = (lo, cut), (cut, hi)
        rec(a, first, left)
        rec(b, first + left, parts - left)

    rec([(0, nz), (0, ny), (0, nx)], 0, nparts)
    return owner.ravel()


def batch_systems(nsys: int, seed: int, nmin: float = 1e3, nmax: float = 2e5):
    """Draw independent system shapes: log-uniform target size, 2D or 3D grid.

    Returns a list of (dim, side): n* = exp(U[ln nmin, ln nmax]); dim is a
    seeded coin flip between 2 and 3; side = round(n*^(1/dim)).
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nsys):
        nstar = float(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))
        dim = 2 if rng.uniform() < 0.5 else 3
        side = max(2, int(round(nstar ** (1.0 / dim))))
        out.append((dim, side))
    return out


def random_lower(n: int, density: float, seed: int, unit: bool = False,
                 long_range: bool = True, dense_row: int | None = None,
                 dtype=np.float64) -> CSR:
    """Random sparse lower-triangular matrix with a dominant diagonal.

    Off-diagonal entries are U[-1, 1] / (row length) so the solve stays well
    conditioned; the diagonal is U[1, 2] (or 1.0 when ``unit``).  ``long_range``
    adds a few dependencies that skip many rows; ``dense_row`` (index) makes one
    row depend on every earlier row.
    """
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(1, n):
        k = rng.binomial(i, min(1.0, density))
        js = rng.choice(i, size=k, replace=False) if k else np.empty(0, np.int64)
        if long_range and i > 8 and rng.uniform() < 0.1:
            js = np.union1d(js, rng.integers(0, max(1, i // 4), size=1))
        if dense_row is not None and i == dense_row:
            js = np.arange(i)
        rows.append(np.full(len(js), i))
        cols.append(np.asarray(js, dtype=np.int64))
    r = np.concatenate(rows) if rows else np.empty(0, np.int64)
    c = np.concatenate(cols) if cols else np.empty(0, np.int64)
    rowlen = np.bincount(r, minlength=n).astype(np.float64)
    v = rng.uniform(-1.0, 1.0, r.shape[0]) / np.maximum(1.0, rowlen[r])
    d = np.ones(n) if unit else rng.uniform(1.0, 2.0, n)
    ar = np.arange(n)
    m = _from_coo(n, np.concatenate([r, ar]), np.concatenate([c, ar]), np.concatenate([v, d]))
    m.val = m.val.astype(dtype)
    return m

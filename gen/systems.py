"""Synthetic SPD systems (CSR, both triangles, sorted columns, explicit diagonal).

Every generator is deterministic given its seed.  Random draws use NumPy's
PCG64 ``default_rng``; the matrix of a seeded system draws from
``default_rng([seed, 0])`` and right-hand sides from ``default_rng([seed, 1])``
so that either can be regenerated without the other.

Vertex numbering on grids is row-major with x fastest:
``v = (z * ny + y) * nx + x``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class CSR:
    """Symmetric sparse matrix in CSR form (int64 rowptr, int32 col, f64 val)."""

    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    coords: np.ndarray | None = None  # (n, d) float64 vertex coordinates, optional
    dims: tuple | None = None  # grid dimensions (nx, ny, nz) when the graph is a grid
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        for i in range(self.n):
            s, e = self.rowptr[i], self.rowptr[i + 1]
            a[i, self.col[s:e]] = self.val[s:e]
        return a

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


def _from_coo(n, rows, cols, vals, **kw) -> CSR:
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order].astype(np.int32)
    vals = vals[order].astype(np.float64)
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CSR(n=n, rowptr=rowptr, col=cols, val=vals, **kw)


def _grid_coords(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float64)


def _stencil_edges(nx, ny, nz):
    """Undirected grid edges (u < v) along x, then y, then z, each in vertex order."""
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    ex = (idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel())
    ey = (idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel())
    ez = (idx[:-1, :, :].ravel(), idx[1:, :, :].ravel())
    return [ex, ey, ez]


def _assemble_weighted(n, edge_u, edge_v, w, diag, **kw) -> CSR:
    rows = np.concatenate([edge_u, edge_v, np.arange(n)])
    cols = np.concatenate([edge_v, edge_u, np.arange(n)])
    vals = np.concatenate([-w, -w, diag])
    return _from_coo(n, rows, cols, vals, **kw)


def laplace2d_dirichlet(nx: int, ny: int | None = None) -> CSR:
    """5-point Laplacian (4 on the diagonal, -1 to each grid neighbour), Dirichlet."""
    ny = nx if ny is None else ny
    n = nx * ny
    es = _stencil_edges(nx, ny, 1)[:2]
    u = np.concatenate([e[0] for e in es])
    v = np.concatenate([e[1] for e in es])
    w = np.ones(u.shape[0])
    return _assemble_weighted(n, u, v, w, np.full(n, 4.0), coords=_grid_coords(nx, ny, 1)[:, :2],
                              dims=(nx, ny, 1), meta=dict(kind="laplace2d", nx=nx, ny=ny))


def poisson3d_dirichlet(nx: int, ny: int | None = None, nz: int | None = None) -> CSR:
    """7-point Poisson matrix (6 on the diagonal, -1 to each neighbour), Dirichlet."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz
    es = _stencil_edges(nx, ny, nz)
    u = np.concatenate([e[0] for e in es])
    v = np.concatenate([e[1] for e in es])
    w = np.ones(u.shape[0])
    return _assemble_weighted(n, u, v, w, np.full(n, 6.0), coords=_grid_coords(nx, ny, nz),
                              dims=(nx, ny, nz), meta=dict(kind="poisson3d", nx=nx, ny=ny, nz=nz))


def lognormal_conductance_2d(nx: int, ny: int | None = None, seed: int = 2, shift: float = 1e-3,
                             mu: float = 0.0, sigma: float = 1.0) -> CSR:
    """Graph Laplacian of a 2D grid with lognormal(mu, sigma) edge conductances, plus shift*I.

    Neumann (no boundary terms).  Weights are drawn for the x-edges first, then
    the y-edges, each in vertex order.
    """
    ny = nx if ny is None else ny
    n = nx * ny
    rng = np.random.default_rng([seed, 0])
    es = _stencil_edges(nx, ny, 1)[:2]
    u = np.concatenate([e[0] for e in es])
    v = np.concatenate([e[1] for e in es])
    w = np.exp(mu + sigma * rng.standard_normal(u.shape[0]))
    diag = np.full(n, shift)
    np.add.at(diag, u, w)
    np.add.at(diag, v, w)
    return _assemble_weighted(n, u, v, w, diag, coords=_grid_coords(nx, ny, 1)[:, :2], dims=(nx, ny, 1),
                              meta=dict(kind="lognormal2d", nx=nx, ny=ny, seed=seed, shift=shift))


def grf_field(nx: int, ny: int, sigma: float, ell: float, seed: int) -> np.ndarray:
    """Gaussian random field with squared-exponential covariance exp(-d^2 / (2 ell^2)).

    White noise on a 2x-padded periodic grid is filtered in Fourier space by the
    square root of the covariance spectrum, cropped to (ny, nx) and standardised
    to sample mean 0 and standard deviation ``sigma``.
    """
    rng = np.random.default_rng([seed, 0])
    py, px = 2 * ny, 2 * nx
    noise = rng.standard_normal((py, px))
    dy = np.minimum(np.arange(py), py - np.arange(py))
    dx = np.minimum(np.arange(px), px - np.arange(px))
    d2 = dy[:, None] ** 2 + dx[None, :] ** 2
    cov = np.exp(-d2 / (2.0 * ell * ell))
    spec = np.maximum(np.fft.fft2(cov).real, 0.0)
    g = np.fft.ifft2(np.fft.fft2(noise) * np.sqrt(spec)).real[:ny, :nx]
    g = (g - g.mean()) / g.std() * sigma
    return g


def diffusion_tpfa(kcell: np.ndarray, seed: int | None = None) -> CSR:
    """Cell-centred two-point-flux diffusion matrix on a grid of cells.

    Face transmissibility between cells i and j is the harmonic mean
    ``2 k_i k_j / (k_i + k_j)``; the domain boundary is zero Dirichlet with a
    boundary-face transmissibility ``2 k_i``.
    """
    ny, nx = kcell.shape
    n = nx * ny
    k = kcell.ravel()
    es = _stencil_edges(nx, ny, 1)[:2]
    u = np.concatenate([e[0] for e in es])
    v = np.concatenate([e[1] for e in es])
    w = 2.0 * k[u] * k[v] / (k[u] + k[v])
    diag = np.zeros(n)
    np.add.at(diag, u, w)
    np.add.at(diag, v, w)
    idx = np.arange(n).reshape(ny, nx)
    for bnd in (idx[0, :], idx[-1, :], idx[:, 0], idx[:, -1]):
        np.add.at(diag, bnd, 2.0 * k[bnd])
    return _assemble_weighted(n, u, v, w, diag, coords=_grid_coords(nx, ny, 1)[:, :2], dims=(nx, ny, 1),
                              meta=dict(kind="tpfa2d", nx=nx, ny=ny, seed=seed))


def random_geometric_graph(n: int, seed: int, mean_degree: float = 8.0, wlo: float = 0.1,
                           whi: float = 1.0, shift: float = 1e-2) -> CSR:
    """Random geometric graph Laplacian in the unit square plus shift*I.

    n uniform points; radius r with pi r^2 n = mean_degree; edge weights
    uniform[wlo, whi].  Vertices are renumbered by (cell row, cell column, x)
    on a grid of r-sized cells so that nearby vertices get nearby numbers.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng([seed, 0])
    pts = rng.random((n, 2))
    r = float(np.sqrt(mean_degree / (np.pi * n)))
    ncell = max(1, int(1.0 / r))
    cx = np.minimum((pts[:, 0] * ncell).astype(np.int64), ncell - 1)
    cy = np.minimum((pts[:, 1] * ncell).astype(np.int64), ncell - 1)
    order = np.lexsort((pts[:, 0], cx, cy))
    pts = pts[order]
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    pairs = np.sort(pairs, axis=1)
    pairs = pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))]
    u = pairs[:, 0].astype(np.int64)
    v = pairs[:, 1].astype(np.int64)
    w = rng.uniform(wlo, whi, size=u.shape[0])
    diag = np.full(n, shift)
    np.add.at(diag, u, w)
    np.add.at(diag, v, w)
    return _assemble_weighted(n, u, v, w, diag, coords=pts, dims=None,
                              meta=dict(kind="rgg", n=n, seed=seed, radius=r))


def random_rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Right-hand sides, i.i.d. uniform[-1, 1]; shape (nrhs, n), each row one RHS."""
    rng = np.random.default_rng([seed, 1])
    return rng.uniform(-1.0, 1.0, size=(nrhs, n))


def block_diag(systems: list[CSR]) -> CSR:
    """Concatenate independent systems into one block-diagonal CSR (coords offset per block)."""
    n = sum(s.n for s in systems)
    rowptr = [np.zeros(1, dtype=np.int64)]
    cols, vals = [], []
    off_n, off_nnz = 0, 0
    for s in systems:
        rowptr.append(s.rowptr[1:] + off_nnz)
        cols.append(s.col.astype(np.int64) + off_n)
        vals.append(s.val)
        off_n += s.n
        off_nnz += s.nnz
    return CSR(n=n, rowptr=np.concatenate(rowptr), col=np.concatenate(cols).astype(np.int32),
               val=np.concatenate(vals), meta=dict(kind="block_diag", sizes=[s.n for s in systems]))


def paper_example_32() -> tuple[CSR, np.ndarray]:
    """The 6-unknown system (3.2) of Example 3.1 and its right-hand side."""
    a = np.array([[6, -1, -2, 0, 0, 0],
                  [-1, 7, 0, -1, 0, 0],
                  [-2, 0, 8, -2, -1, 0],
                  [0, -1, -2, 9, 0, -3],
                  [0, 0, -1, 0, 10, -5],
                  [0, 0, 0, -3, -5, 11]], dtype=np.float64)
    b = np.array([1, 2, 3, 4, 5, 6], dtype=np.float64)
    r, c = np.nonzero(a)
    return _from_coo(6, r, c, a[r, c]), b

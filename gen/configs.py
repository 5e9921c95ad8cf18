"""The five workloads (and small versions of each for tests).

A config is a plain dict:
  A        CSR system (block-diagonal concatenation for batches)
  spec     partition specification (dict, see below)
  b        right-hand sides, shape (nrhs, n)
  tol      relative-residual target
  nsys     number of independent systems (1 except for batches)
  sys_ptr  vertex ranges of the systems (nsys + 1)
  name     workload name

Partition specification dicts:
  {"kind": "grid",  "dims": (nx, ny, nz), "parts": (px, py, pz)}
  {"kind": "rcb",   "dims": (nx, ny, nz), "levels": L, "seed": s, "min_size": a, "max_size": b}
  {"kind": "graph", "coords": (n, d) array, "blocks": [(start, count, nparts), ...]}
  {"kind": "user",  "s_ptr": int64 (n + 1), "s_idx": int32}
"""
from __future__ import annotations

import numpy as np

from . import systems as S

CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5")


def _single(A, spec, nrhs, seed, tol, name, **extra):
    b = S.random_rhs(A.n, nrhs, seed)
    cfg = dict(A=A, spec=spec, b=b, tol=tol, nsys=1, sys_ptr=np.array([0, A.n], dtype=np.int64), name=name)
    cfg.update(extra)
    return cfg


def c1(small: bool = False):
    """2D 5-point Dirichlet Laplacian on 64x64, 4x4 tiles, tol 1e-10, seed 1."""
    A = S.laplace2d_dirichlet(64)
    spec = dict(kind="grid", dims=(64, 64, 1), parts=(4, 4, 1))
    return _single(A, spec, 1, 1, 1e-10, "c1_laplace2d_64x64_4x4")


def c2(small: bool = False):
    """Lognormal(0,1) conductance Laplacian + 1e-3 I on 1024^2, 32x32 tiles, seed 2."""
    nx, p = (128, 4) if small else (1024, 32)
    A = S.lognormal_conductance_2d(nx, seed=2, shift=1e-3)
    spec = dict(kind="grid", dims=(nx, nx, 1), parts=(p, p, 1))
    return _single(A, spec, 1, 2, 1e-8, f"c2_lognormal2d_{nx}x{nx}_{p}x{p}")


def c3(small: bool = False):
    """3D 7-point Poisson on 128^3, seeded RCB into 4096 boxes, 8 RHS, seed 3."""
    nx, levels = (32, 6) if small else (128, 12)
    A = S.poisson3d_dirichlet(nx)
    spec = dict(kind="rcb", dims=(nx, nx, nx), levels=levels, seed=3, min_size=300.0, max_size=700.0)
    return _single(A, spec, 8, 3, 1e-8, f"c3_poisson3d_{nx}^3_rcb{2 ** levels}")


def c4_system(seed: int, small: bool = False):
    """TPFA diffusion with k = exp(g), g a GRF (sigma 1.5, correlation length 16 cells)."""
    nx = 128 if small else 512
    g = S.grf_field(nx, nx, 1.5, 16.0, seed)
    return S.diffusion_tpfa(np.exp(g), seed=seed)


def c4(small: bool = False, seed: int = 4200):
    """Learned-Z workload: 512^2 TPFA GRF diffusion, 16x16 tiles; eval seeds 4200-4209."""
    nx, p = (128, 4) if small else (512, 16)
    A = c4_system(seed, small)
    spec = dict(kind="grid", dims=(nx, nx, 1), parts=(p, p, 1))
    return _single(A, spec, 1, seed, 1e-8, f"c4_tpfa_grf_{nx}x{nx}_{p}x{p}_seed{seed}")


C4_TRAIN_SEEDS = tuple(range(4000, 4200))
C4_EVAL_SEEDS = tuple(range(4200, 4210))


def c5(small: bool = False, nsys: int | None = None):
    """Batch of random geometric graph Laplacians + 1e-2 I, n ~ U{20k..200k}, 4 RHS each; graph EVS
    with tree VTLs."""
    if nsys is None:
        nsys = 4 if small else 64
    lo, hi = (2000, 8000) if small else (20000, 200000)
    sizes = [int(np.random.default_rng([5000 + i, 2]).integers(lo, hi + 1)) for i in range(nsys)]
    syss = [S.random_geometric_graph(nk, 5000 + i) for i, nk in enumerate(sizes)]
    A = S.block_diag(syss)
    coords = np.concatenate([s.coords for s in syss], axis=0)
    blocks, start = [], 0
    for s in syss:
        blocks.append((start, s.n, max(1, (s.n + 256) // 512)))
        start += s.n
    # graph partitions split vertices three ways around triangles of subgraphs: tree VTLs
    spec = dict(kind="graph", coords=coords, blocks=blocks, topology="tree")
    b = np.concatenate([S.random_rhs(s.n, 4, 5000 + i) for i, s in enumerate(syss)], axis=1)
    sys_ptr = np.array([0] + list(np.cumsum(sizes)), dtype=np.int64)
    return dict(A=A, spec=spec, b=b, tol=1e-8, nsys=nsys, sys_ptr=sys_ptr,
                name=f"c5_rgg_batch{nsys}", sizes=sizes)


def make_config(name: str, small: bool = False):
    return {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}[name](small=small)

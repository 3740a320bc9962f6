"""Seeded synthetic inputs for the two-grid matching-AMG solver.

This package only builds problems (matrices, right-hand sides, targets); it
holds none of the solver's arithmetic, so both the HIP library's tests and the
CPU oracle may use it.

Named workloads (draw order within one numpy Generator: kappa blocks, then the
right-hand sides as an (nrhs, N) array, then x_target):

* ``fv2d_64``   : 64x64 cells, kappa on 8x8 blocks, log10 kappa ~ U(-3, 3),
                  a = (1, 0.5), one RHS ~ U(-1, 1).
* ``fv2d_1024`` : 1024x1024 cells, kappa on 64x64 blocks, log10 kappa ~ U(-4, 4),
                  rotating a = 10 (sin pi x cos pi y, -cos pi x sin pi y).
* ``fv3d_128``  : 128^3 cells, kappa on 16^3 blocks, log10 kappa ~ U(-6, 6),
                  a = (1, 1, 1).
* ``rgg_500k``  : random geometric graph, 500k nodes, directed kNN with
                  k in {6..14} (see ``rgg.py``).
* ``fv2d_512_grad``: 512x512 cells, per-cell kappa from the fv2d_64 block law
                  (8 blocks per direction), 16 RHS and x_target ~ U(-1, 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .fv import block_kappa, dc1_kappa, fv_matrix, velocity_const, velocity_rotating
from .grid7 import grid7_matrix
from .rgg import rgg_matrix


@dataclass
class Problem:
    name: str
    n_rows: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    b: np.ndarray                      # (N, nrhs) row-major
    kappa: np.ndarray | None = None    # per-cell, grids only
    grid: tuple | None = None          # (n, dim)
    velocity: object = None
    x_target: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def _rhs(rng, N, nrhs):
    return np.ascontiguousarray(rng.uniform(-1.0, 1.0, size=(nrhs, N)).T)


def fv_problem(n, dim, nblocks, lo, hi, velocity, seed=0, nrhs=1, target=False, name=None):
    rng = np.random.default_rng(seed)
    kap = block_kappa(n, dim, nblocks, lo, hi, rng)
    rp, ci, va = fv_matrix(n, dim, kap, velocity)
    N = n ** dim
    b = _rhs(rng, N, nrhs)
    xt = _rhs(rng, N, nrhs) if target else None
    return Problem(name or f"fv{dim}d_{n}", N, rp, ci, va, b, kappa=kap, grid=(n, dim),
                   velocity=velocity, x_target=xt,
                   meta=dict(n=n, dim=dim, nblocks=nblocks, log10_kappa=(lo, hi), seed=seed))


def rgg_problem(N=500_000, seed=0, nrhs=1, name=None):
    rng = np.random.default_rng(seed)
    rp, ci, va = rgg_matrix(N, rng)
    b = _rhs(rng, N, nrhs)
    return Problem(name or f"rgg_{N}", N, rp, ci, va, b, meta=dict(seed=seed))


def paper_problem(case: str, n: int, seed: int = 0, nrhs: int = 1) -> Problem:
    """The paper's analytic test problems (Section 3.1) on an n^dim cell grid:
    ``dc1_2d`` / ``dc1_3d`` (discontinuous kappa of dc1_kappa, zero velocity),
    ``dcc1_2d`` (velocity (1000, 1000)) and ``dcc2_3d`` (velocity
    (1000, 1000, 1000)); right-hand side U(-1, 1) from the seed."""
    dims = {"dc1_2d": 2, "dc1_3d": 3, "dcc1_2d": 2, "dcc2_3d": 3}
    if case not in dims:
        raise KeyError(case)
    dim = dims[case]
    kap = dc1_kappa(n, dim)
    vel = velocity_const((1000.0,) * dim) if case.startswith("dcc") else None
    rp, ci, va = fv_matrix(n, dim, kap, vel)
    N = n ** dim
    b = _rhs(np.random.default_rng(seed), N, nrhs)
    return Problem(f"{case}_{n}", N, rp, ci, va, b, kappa=kap, grid=(n, dim), velocity=vel,
                   meta=dict(n=n, dim=dim, case=case, seed=seed))


def make(name: str, seed: int = 0, **kw) -> Problem:
    """Build one of the named workloads (see module docstring)."""
    if name == "fv2d_64":
        return fv_problem(64, 2, 8, -3, 3, velocity_const((1.0, 0.5)), seed, name=name, **kw)
    if name == "fv2d_1024":
        return fv_problem(1024, 2, 64, -4, 4, velocity_rotating(10.0), seed, name=name, **kw)
    if name == "fv3d_128":
        return fv_problem(128, 3, 16, -6, 6, velocity_const((1.0, 1.0, 1.0)), seed, name=name, **kw)
    if name == "rgg_500k":
        return rgg_problem(500_000, seed, name=name, **kw)
    if name == "fv2d_512_grad":
        return fv_problem(512, 2, 8, -3, 3, velocity_const((1.0, 0.5)), seed, nrhs=16,
                          target=True, name=name, **kw)
    if name == "fv2d_32_grad":
        return fv_problem(32, 2, 8, -3, 3, velocity_const((1.0, 0.5)), seed, nrhs=16,
                          target=True, name=name, **kw)
    raise KeyError(name)


def scaled(kind: str, n: int, seed: int = 0, nrhs: int = 1) -> Problem:
    """Smaller members of the same families, for tests: ``fv2d``/``fv3d``
    (n cells per direction, kappa blocks of the fv2d_64 / fv3d_128 law) and
    ``rgg`` (n nodes)."""
    if kind == "fv2d":
        nb = 8 if n % 8 == 0 else 1
        return fv_problem(n, 2, nb, -3, 3, velocity_const((1.0, 0.5)), seed, nrhs=nrhs,
                          name=f"fv2d_{n}")
    if kind == "fv2d_rot":
        nb = 8 if n % 8 == 0 else 1
        return fv_problem(n, 2, nb, -4, 4, velocity_rotating(10.0), seed, nrhs=nrhs,
                          name=f"fv2d_rot_{n}")
    if kind == "fv3d":
        nb = 4 if n % 4 == 0 else 1
        return fv_problem(n, 3, nb, -6, 6, velocity_const((1.0, 1.0, 1.0)), seed, nrhs=nrhs,
                          name=f"fv3d_{n}")
    if kind == "rgg":
        return rgg_problem(n, seed, nrhs=nrhs, name=f"rgg_{n}")
    raise KeyError(kind)


__all__ = ["Problem", "make", "scaled", "fv_matrix", "fv_problem", "rgg_problem",
           "paper_problem", "block_kappa", "dc1_kappa", "velocity_const", "velocity_rotating", "rgg_matrix",
           "grid7_matrix"]

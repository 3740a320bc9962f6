"""Seven-point matrices on nx x ny x nz grids in natural order (cell
(z * ny + y) * nx + x), for the 3D wavefront sweeps' tests and timings."""
from __future__ import annotations

import numpy as np


def grid7_matrix(nx, ny, nz, seed):
    """Nonsymmetric seven-point matrix: off-diagonal entries
    -U(0.1, 1) * (1 + 0.3 U(-1, 1)), diagonal 1.05 * (sum of their magnitudes)
    + 0.01 (strictly diagonally dominant).  CSR arrays (rowptr, col, val)."""
    rng = np.random.default_rng(seed)
    n = nx * ny * nz
    c = np.arange(n)
    x, y, z = c % nx, (c // nx) % ny, c // (nx * ny)
    offs = [(-nx * ny, z > 0), (-nx, y > 0), (-1, x > 0), (1, x < nx - 1), (nx, y < ny - 1), (nx * ny, z < nz - 1)]
    cols = [np.where(m, c + d, -1) for d, m in offs]
    vals = [np.where(m, -rng.uniform(0.1, 1.0, n) * (1 + 0.3 * rng.uniform(-1, 1, n)), 0.0) for d, m in offs]
    diag = 1.05 * np.sum(np.abs(vals), axis=0) + 0.01
    allc = np.stack(cols[:3] + [c] + cols[3:], axis=1)
    allv = np.stack(vals[:3] + [diag] + vals[3:], axis=1)
    keep = allc >= 0
    rowptr = np.concatenate([[0], np.cumsum(keep.sum(axis=1))]).astype(np.int32)
    return rowptr, allc[keep].astype(np.int32), allv[keep]

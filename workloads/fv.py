"""Cell-centred finite-volume convection-diffusion matrices on the unit square/cube.

Problem statement: div(a u) - div(kappa grad u) = f on [0,1]^d, u = 0 on the
faces y = 0 and y = 1 (Dirichlet), du/dn = 0 on the other faces (Neumann)
(paper, Section 1, Eq. (pde) and the boundary description after it).

The paper names the discretisation ("cell centered finite volume") but gives no
stencil.  The reading implemented here:

* uniform grid, h = 1/n, cell (i, j[, k]) is unknown ``i + n*j (+ n*n*k)``
  (x fastest);
* every row is the cell's flux balance divided by the cell volume h^d;
* diffusion: an interior face between cells c and m carries the harmonic
  transmissibility T = 2 kc km / ((kc + km) h^2); a Dirichlet face adds
  2 kc / h^2 to the diagonal; a Neumann face adds nothing;
* convection: first-order upwind on the face-averaged outward normal velocity
  F of each face: the diagonal gets max(F, 0)/h, the neighbour column gets
  min(F, 0)/h; on a boundary face outflow adds max(F, 0)/h to the diagonal and
  inflow adds nothing (boundary value 0);
* face-averaged velocities of a divergence-free field are taken from its stream
  function, so they are discretely divergence free.

With div a = 0 the result is an irreducibly diagonally dominant M-matrix.
Columns are sorted within each row and the diagonal is always stored.
"""
from __future__ import annotations

import numpy as np


def _csr_from_bands(n_rows: int, offsets, bands, present):
    """Assemble CSR from per-row diagonals.

    ``offsets`` ascending column offsets, ``bands[d][r]`` the value of row r at
    column r + offsets[d], ``present[d][r]`` whether that entry is stored.
    """
    mask = np.stack(present, axis=1)            # (n, nd)
    vals = np.stack(bands, axis=1)
    cols = np.arange(n_rows, dtype=np.int64)[:, None] + np.asarray(offsets, dtype=np.int64)[None, :]
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = cols[mask].astype(np.int32)
    val = vals[mask].astype(np.float64)
    return rowptr.astype(np.int32), col, val


def velocity_const(a):
    """Face-averaged normal velocities for a constant field ``a``."""
    a = tuple(float(t) for t in a)

    def faces(n, dim):
        out = []
        for d in range(dim):
            shape = [n] * dim
            shape[dim - 1 - d] = n + 1            # axis order (z, y, x)
            out.append(np.full(shape, a[d]))
        return out
    return faces


def velocity_rotating(scale=10.0):
    """a = scale * (sin(pi x) cos(pi y), -cos(pi x) sin(pi y)) in 2D.

    Stream function psi = (scale/pi) sin(pi x) sin(pi y), a = (d psi/dy,
    -d psi/dx).  The average normal velocity over a face is the difference of
    psi at the face's end points divided by h, which makes the discrete
    divergence of every cell exactly a telescoping sum of zero.
    """
    def faces(n, dim):
        assert dim == 2
        h = 1.0 / n
        nodes = np.arange(n + 1) * h
        psi = (scale / np.pi) * np.sin(np.pi * nodes)[None, :] * np.sin(np.pi * nodes)[:, None]  # [y, x]
        # x-faces at x = i h, spanning y in [j h, (j+1) h]: flux +x = psi(top) - psi(bottom)
        fx = (psi[1:, :] - psi[:-1, :]) / h                    # shape (n, n+1) [j, i]
        # y-faces at y = j h, spanning x in [i h, (i+1) h]: flux +y = -(psi(right) - psi(left))
        fy = -(psi[:, 1:] - psi[:, :-1]) / h                   # shape (n+1, n) [j, i]
        return [fx, fy]
    return faces


def fv_matrix(n: int, dim: int, kappa: np.ndarray, velocity=None):
    """Assemble the FV matrix on an n^dim grid.

    ``kappa``: per-cell diffusion coefficient, flat in row order (length n^dim).
    ``velocity``: callable (n, dim) -> list of face-velocity arrays (x, y[, z]),
    face array d has n+1 entries along axis d; None means a = 0.
    Returns (rowptr int32, col int32, val float64).
    """
    assert dim in (2, 3)
    N = n ** dim
    h = 1.0 / n
    h2 = h * h
    shape = (n,) * dim                     # axis order (z,) y, x
    kap = np.asarray(kappa, dtype=np.float64).reshape(shape)
    if velocity is None:
        vel = velocity_const((0.0,) * dim)(n, dim)
    else:
        vel = velocity(n, dim)

    diag = np.zeros(shape)
    bands = {}
    stride = {0: 1, 1: n, 2: n * n}
    for d in range(dim):                   # physical direction d: 0=x, 1=y, 2=z
        ax = dim - 1 - d                   # numpy axis of direction d
        F = vel[d]                         # face velocities, length n+1 along ax
        sl_lo = [slice(None)] * dim
        sl_hi = [slice(None)] * dim
        sl_lo[ax] = slice(0, n)
        sl_hi[ax] = slice(1, n + 1)
        F_lo = F[tuple(sl_lo)]              # face on the low side of each cell (flux +d)
        F_hi = F[tuple(sl_hi)]              # face on the high side
        # interior faces: between cell c and c+e_d
        a_sl = [slice(None)] * dim
        b_sl = [slice(None)] * dim
        a_sl[ax] = slice(0, n - 1)
        b_sl[ax] = slice(1, n)
        ka = kap[tuple(a_sl)]
        kb = kap[tuple(b_sl)]
        T = 2.0 * ka * kb / ((ka + kb) * h2)
        up = np.zeros(shape)                # coefficient of column c + e_d in row c
        dn = np.zeros(shape)                # coefficient of column c - e_d in row c
        has_up = np.zeros(shape, dtype=bool)
        has_dn = np.zeros(shape, dtype=bool)
        has_up[tuple(a_sl)] = True
        has_dn[tuple(b_sl)] = True
        # high face of cell c (outward flux +F_hi), low face (outward flux -F_lo)
        out_hi = F_hi
        out_lo = -F_lo
        # diffusion
        d_int = np.zeros(shape)
        d_int[tuple(a_sl)] += T
        d_int[tuple(b_sl)] += T
        up[tuple(a_sl)] -= T
        dn[tuple(b_sl)] -= T
        # convection, interior and boundary faces
        conv = np.maximum(out_hi, 0.0) / h + np.maximum(out_lo, 0.0) / h
        up[tuple(a_sl)] += np.minimum(out_hi[tuple(a_sl)], 0.0) / h
        dn[tuple(b_sl)] += np.minimum(out_lo[tuple(b_sl)], 0.0) / h
        diag += d_int
        diag += conv
        if d == 1:                          # Dirichlet faces y = 0 and y = 1
            lo = [slice(None)] * dim
            hi = [slice(None)] * dim
            lo[ax] = slice(0, 1)
            hi[ax] = slice(n - 1, n)
            diag[tuple(lo)] += 2.0 * kap[tuple(lo)] / h2
            diag[tuple(hi)] += 2.0 * kap[tuple(hi)] / h2
        bands[+stride[d]] = (up.reshape(N), has_up.reshape(N))
        bands[-stride[d]] = (dn.reshape(N), has_dn.reshape(N))
    offsets = sorted(list(bands.keys()) + [0])
    bl, pl = [], []
    for off in offsets:
        if off == 0:
            bl.append(diag.reshape(N))
            pl.append(np.ones(N, dtype=bool))
        else:
            bl.append(bands[off][0])
            pl.append(bands[off][1])
    return _csr_from_bands(N, offsets, bl, pl)


def block_kappa(n: int, dim: int, nblocks: int, lo: float, hi: float, rng) -> np.ndarray:
    """Piecewise-constant kappa on nblocks^dim equal blocks, log10 kappa ~ U(lo, hi),
    one draw per block in block-lexicographic order (x block index fastest).
    Returns a flat per-cell array in row order."""
    assert n % nblocks == 0
    bs = n // nblocks
    logk = rng.uniform(lo, hi, size=nblocks ** dim)
    kb = 10.0 ** logk
    idx = np.arange(n) // bs
    if dim == 2:
        blk = idx[None, :] + nblocks * idx[:, None]                      # [y, x]
    else:
        blk = (idx[None, None, :] + nblocks * idx[None, :, None]
               + nblocks * nblocks * idx[:, None, None])                # [z, y, x]
    return kb[blk].reshape(-1)


def dc1_kappa(n: int, dim: int) -> np.ndarray:
    """The DC1 coefficient of the paper's test cases (Section 3.1): 1e3*([10 y]+1)
    where [10 x_i] is even in every direction, 1 elsewhere; evaluated at cell
    centres."""
    c = (np.arange(n) + 0.5) / n
    f = np.floor(10.0 * c).astype(np.int64)
    even = (f % 2) == 0
    if dim == 2:
        m = even[None, :] & even[:, None]
        val = 1e3 * (f[:, None] + 1.0) * np.ones((n, n))
    else:
        m = even[None, None, :] & even[None, :, None] & even[:, None, None]
        val = 1e3 * (f[None, :, None] + 1.0) * np.ones((n, n, n))
    k = np.where(m, val, 1.0)
    return k.reshape(-1)

"""Synthetic unstructured nonsymmetric matrices from a random geometric graph.

Stand-in for the unstructured sparse matrices the paper takes from a public
collection (Section 3.1, Table Tab:FMM), which are not available here.

Recipe (all draws from one numpy Generator, in this order):
1. N points uniform in [0,1)^2;
2. per row i a neighbour count k_i uniform in {kmin..kmax};
3. row i stores its k_i nearest other points (directed kNN, so the pattern is
   not symmetric);
4. one base magnitude m ~ U(0.1, 1) per unordered pair {i, j} that appears in
   either direction, pairs sorted by (min, max);
5. one asymmetry draw eps ~ U(-1, 1) per stored off-diagonal entry in CSR
   order; a_ij = -m_{ij} (1 + 0.1 eps_ij);
6. a_ii = 1.05 * sum_j |a_ij|  (strictly diagonally dominant M-matrix).
"""
from __future__ import annotations

import numpy as np


def rgg_matrix(N: int, rng, kmin: int = 6, kmax: int = 14):
    from scipy.spatial import cKDTree

    pts = rng.random((N, 2))
    k = rng.integers(kmin, kmax + 1, size=N)
    tree = cKDTree(pts)
    _, nb = tree.query(pts, k=kmax + 1)
    nb = np.asarray(nb, dtype=np.int64)
    # drop self (first hit for distinct points); fall back to filtering if a tie moved it
    rows, cols = [], []
    sel = np.arange(kmax + 1)[None, :] < (k[:, None] + 1)
    cand = np.where(sel, nb, -1)
    r_idx = np.repeat(np.arange(N), kmax + 1)
    c_idx = cand.reshape(-1)
    keep = (c_idx >= 0) & (c_idx != r_idx)
    rows = r_idx[keep]
    cols = c_idx[keep]
    # a self hit that was not first leaves k_i+1 candidates: trim to k_i per row
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    # enforce exactly k_i per row by distance rank (cand already distance ordered);
    # the lexsort above only orders by column for CSR, counts are unaffected unless
    # self was absent from the first k_i+1 (never for distinct random points)
    counts = np.bincount(rows, minlength=N)
    assert np.all(counts >= k), "kNN query returned too few neighbours"
    if np.any(counts != k):
        raise RuntimeError("duplicate points in the random geometric graph")
    # unordered pairs
    lo = np.minimum(rows, cols)
    hi = np.maximum(rows, cols)
    pair_key = lo * N + hi
    uniq, inv = np.unique(pair_key, return_inverse=True)
    m = rng.uniform(0.1, 1.0, size=uniq.shape[0])
    eps = rng.uniform(-1.0, 1.0, size=rows.shape[0])
    off = -m[inv] * (1.0 + 0.1 * eps)
    dsum = np.zeros(N)
    np.add.at(dsum, rows, np.abs(off))
    diag = 1.05 * dsum
    # merge diagonal into CSR (columns ascending)
    all_r = np.concatenate([rows, np.arange(N)])
    all_c = np.concatenate([cols, np.arange(N)])
    all_v = np.concatenate([off, diag])
    o = np.lexsort((all_c, all_r))
    all_r, all_c, all_v = all_r[o], all_c[o], all_v[o]
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(all_r, minlength=N), out=rowptr[1:])
    return rowptr.astype(np.int32), all_c.astype(np.int32), all_v.astype(np.float64)

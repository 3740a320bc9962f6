"""Brute-force references used to pin the oracle (tests only).

Everything here is written from the definitions, in plain Python / dense
numpy, and shares nothing with ``oracle/`` beyond the published definitions of
the edge order and of the aggregation it pins.
"""
from __future__ import annotations

import math
import struct

import numpy as np
import scipy.sparse as sp

M64 = (1 << 64) - 1


def splitmix64_out(z: int) -> int:
    # output function of SplitMix64 (Steele, Lea, Flood, OOPSLA 2014)
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def edge_key(w: float, a: int, b: int, qbits: int, seed: int):
    lo, hi = min(a, b), max(a, b)
    bits = struct.unpack("<Q", struct.pack("<d", w))[0]
    return (bits >> (52 - qbits), splitmix64_out(((lo << 32) | hi) ^ seed), lo, hi)


def dict_graph(rowptr, col, w):
    """{(i, j): w} for a CSR graph."""
    g = {}
    for i in range(len(rowptr) - 1):
        for p in range(rowptr[i], rowptr[i + 1]):
            g[(i, int(col[p]))] = float(w[p])
    return g


def greedy_matching(nv: int, edges: dict, qbits: int, seed: int):
    """Sequential greedy maximal matching taking edges by descending key."""
    und = {}
    for (i, j), w in edges.items():
        if i < j:
            und[(i, j)] = w
    order = sorted(und.items(), key=lambda kv: edge_key(kv[1], kv[0][0], kv[0][1], qbits, seed),
                   reverse=True)
    mate = [-1] * nv
    for (i, j), _ in order:
        if mate[i] < 0 and mate[j] < 0:
            mate[i], mate[j] = j, i
    return mate


def is_maximal(nv, edges, mate):
    for (i, j) in edges:
        if i != j and mate[i] < 0 and mate[j] < 0:
            return False
    return True


def sym_graph(rowptr, col, val):
    """Fine graph: {i,j}, i != j, stored in either direction; w = |a_ij| + |a_ji|."""
    n = len(rowptr) - 1
    a = {}
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            a[(i, int(col[p]))] = float(val[p])
    g = {}
    for (i, j) in a:
        if i == j:
            continue
        wij = abs(a.get((i, j), 0.0)) + abs(a.get((j, i), 0.0))
        g[(i, j)] = wij
        g[(j, i)] = abs(a.get((j, i), 0.0)) + abs(a.get((i, j), 0.0))
    return g


def multipass_aggregation(rowptr, col, val, cf, max_passes, qbits, seed):
    """Iterated greedy matching on aggregate graphs (reference of the oracle's
    handshake passes, using greedy == handshake for locally dominant edges)."""
    n = len(rowptr) - 1
    g0 = sym_graph(rowptr, col, val)
    rows = {}
    for (i, j), w in g0.items():
        rows.setdefault(i, []).append((j, w))
    for i in rows:
        rows[i].sort()
    agg = list(range(n))
    nv = n
    target = math.floor(n / cf)
    passes = 0
    while nv > target and passes < max_passes:
        # aggregate graph weights, summed in fine CSR order from the smaller id
        w = {}
        for k in range(n):
            for (l, wkl) in rows.get(k, []):
                I, J = agg[k], agg[l]
                if I < J:
                    w[(I, J)] = w[(I, J)] + wkl if (I, J) in w else wkl
        edges = dict(w)
        for (I, J), x in w.items():
            edges[(J, I)] = x
        mate = greedy_matching(nv, edges, qbits, seed)
        if all(m < 0 for m in mate):
            break
        new = [0] * nv
        c = 0
        for v in range(nv):
            if mate[v] < 0 or v < mate[v]:
                new[v] = c
                c += 1
            else:
                new[v] = new[mate[v]]
        agg = [new[a] for a in agg]
        nv = c
        passes += 1
    return np.array(agg, dtype=np.int32), passes


def dense(rowptr, col, val, n=None):
    n = n or len(rowptr) - 1
    return sp.csr_matrix((val, col, rowptr), shape=(len(rowptr) - 1, n)).toarray()


def prolongation(agg, nc):
    n = len(agg)
    P = np.zeros((n, nc))
    P[np.arange(n), agg] = 1.0
    return P


def lu_nopivot(A):
    """Dense Doolittle LU without pivoting (textbook)."""
    n = A.shape[0]
    U = A.astype(np.float64).copy()
    L = np.eye(n)
    for k in range(n):
        for i in range(k + 1, n):
            L[i, k] = U[i, k] / U[k, k]
            U[i, k:] -= L[i, k] * U[k, k:]
    return L, U


def random_mmatrix(n, rng, density=0.1, sym=False, integer=False):
    """Random strictly diagonally dominant M-matrix with a random pattern."""
    M = (rng.random((n, n)) < density).astype(float)
    np.fill_diagonal(M, 0)
    if sym:
        M = np.maximum(M, M.T)
    if integer:
        V = -rng.integers(1, 9, size=(n, n)).astype(float)
    else:
        V = -rng.uniform(0.1, 1.0, size=(n, n))
    if sym:
        V = np.triu(V) + np.triu(V, 1).T
    A = M * V
    d = np.abs(A).sum(axis=1) + (1.0 if integer else 0.05) + (rng.integers(0, 3, n) if integer else 0)
    A[np.arange(n), np.arange(n)] = d
    S = sp.csr_matrix(A)
    S.sort_indices()
    return S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64), A


def nd_order_ref(n, adj, nodes=None):
    """Nested-dissection numbering, recursive, from the definition: returns
    the list of vertices in their new order.  adj: list of neighbour sets.
    nodes (a list) receives (first position, |part 1|, |part 2|, |separator|)
    of every split: a bisection (separator > 0) or a split into the component
    of the smallest vertex and the rest (separator 0)."""
    import sys
    sys.setrecursionlimit(max(10000, 4 * n))

    def bfs(S, src):
        d = {src: 0}
        q = [src]
        for u in q:
            for v in adj[u]:
                if v in S and v not in d:
                    d[v] = d[u] + 1
                    q.append(v)
        return d

    def nd(S, start):
        S = sorted(S)
        if len(S) <= 64:
            return S
        Sset = set(S)
        d = bfs(Sset, S[0])
        if len(d) < len(S):
            comp = sorted(d)
            rest = [v for v in S if v not in d]
            if nodes is not None:
                nodes.append((start, len(comp), len(rest), 0))
            return nd(comp, start) + nd(rest, start + len(comp))
        far = max(d.values())
        r = min(v for v in S if d[v] == far)
        d = bfs(Sset, r)
        L = max(d.values())
        if L < 2:
            return S
        m, cum = 0, 0
        counts = [0] * (L + 1)
        for v in S:
            counts[d[v]] += 1
        cum = counts[0]
        while cum < len(S) / 2:
            m += 1
            cum += counts[m]
        m = min(max(m, 1), L - 1)
        A = [v for v in S if d[v] < m]
        Bp = [v for v in S if d[v] > m]
        sep = [v for v in S if d[v] == m]
        if nodes is not None:
            nodes.append((start, len(A), len(Bp), len(sep)))
        return nd(A, start) + nd(Bp, start + len(A)) + sep

    return nd(list(range(n)), 0)


def coarse_pattern_adj(rowptr, col, agg, nc):
    """Neighbour sets of the aggregate graph of A's stored pattern."""
    adj = [set() for _ in range(nc)]
    n = len(rowptr) - 1
    for k in range(n):
        for p in range(rowptr[k], rowptr[k + 1]):
            I, J = int(agg[k]), int(agg[col[p]])
            if I != J:
                adj[I].add(J)
                adj[J].add(I)
    return adj

"""Per-entry error scales for comparing one application of the two-grid
preconditioner computed two ways (GPU kernels against the oracle).

Every entry of q = B~^{-1} z is produced by a chain of sums: the smoother's
triangular sweeps, the residual, the restriction, the coarse solve and the
prolongation.  Two correct implementations may add the same terms in another
order or contract them into fused multiply-adds, so q_i can differ by a small
multiple of the unit roundoff times the MAGNITUDES that flow into q_i, not
times |q_i| (which can be tiny through cancellation).  ``apply_scale`` bounds
those magnitudes entry by entry by running the application on absolute values
with the comparison matrices of the triangular factors,

    M(T)_ii = |t_ii|,  M(T)_ij = -|t_ij|  (i != j),  |T^{-1}| <= M(T)^{-1},

so that, for the forward application,

    m_t  = M(U0)^{-1} M(L0)^{-1} |z|          (bounds |t| and its partial sums)
    m_rc = P^T (|z| + |A| m_t)                (bounds r = z - A t, then P^T r)
    m_ec = M(U~)^{-1} M(L~)^{-1} m_rc         (coarse factors; |M| m_rc for a
                                               sparse approximate inverse,
                                               |A_c^{-1}| m_rc for the dense one)
    scale = m_t + P m_ec,

and the adjoint application transposes each step.  For the M-matrices of the
test problems M(T) = T and this is exactly |S^{-1}| |z| + ... with no
overestimation from the comparison matrices.  Parity is then
|q_i - ref_i| <= tol * scale_i for every i.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _cmp(T):
    """Comparison matrix of a sparse triangular factor (CSR)."""
    T = sp.csr_matrix(T, copy=True)
    d = T.diagonal()
    T.data = -np.abs(T.data)
    T = T + sp.diags(np.abs(d) + np.abs(d))      # -|t_ii| + 2|t_ii| = |t_ii|
    return sp.csr_matrix(T)


def _tri(T, b, lower):
    return spla.spsolve_triangular(sp.csr_matrix(T), b, lower=lower)


def _parts(O, A):
    """Fine smoother factors (in the smoother's numbering) and coarse operator
    pieces of an oracle setup."""
    n = O.n
    perm, (frp, fci, fv) = O.fine()
    ilu = O.ilu0()
    F = sp.csr_matrix((ilu, fci, frp), shape=(n, n))
    L0 = sp.tril(F, -1) + sp.identity(n)
    U0 = sp.triu(F)
    agg = O.aggregates()
    P = sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, O.nc))
    return perm, L0, U0, P


def apply_scale(O, A, z, adjoint=False, coarse=None):
    """Per-entry magnitude bound of one preconditioner application on z.
    O: oracle.Oracle of the same setup; A: scipy CSR of A.  coarse: None for
    the ILUT factors (or their Jacobi sweeps, which the same bound covers),
    ("spai", M) with M the sparse approximate inverse, ("dense", Ainv) with
    the dense A_c^{-1}."""
    perm, L0, U0, P = _parts(O, A)
    absA = abs(sp.csr_matrix(A))
    az = np.abs(np.asarray(z, dtype=np.float64))
    if coarse is None:
        (lrp, lci, lv), (urp, uci, uv) = O.ilut()
        nc = O.nc
        Lc = sp.csr_matrix((lv, lci, lrp), shape=(nc, nc)) + sp.identity(nc)
        Uc = sp.csr_matrix((uv, uci, urp), shape=(nc, nc))

    def coarse_abs(v, transpose):
        if coarse is None:
            if not transpose:
                return _tri(_cmp(Uc), _tri(_cmp(Lc), v, True), False)
            return _tri(_cmp(Lc).T, _tri(_cmp(Uc).T, v, True), False)
        kind, M = coarse
        M = abs(sp.csr_matrix(M)) if kind == "spai" else np.abs(M)
        return (M.T if transpose else M) @ v

    def smooth_abs(v, transpose):
        vp = v[perm]                     # into the smoother's numbering
        if not transpose:
            tp = _tri(_cmp(U0), _tri(_cmp(L0), vp, True), False)
        else:
            tp = _tri(_cmp(L0).T, _tri(_cmp(U0).T, vp, True), False)
        out = np.empty_like(tp)
        out[perm] = tp
        return out

    if not adjoint:
        mt = smooth_abs(az, False)
        mrc = P.T @ (az + absA @ mt)
        mec = coarse_abs(mrc, False)
        return mt + P @ mec
    mec = coarse_abs(P.T @ az, True)
    ms = az + absA.T @ (P @ mec)
    mt = smooth_abs(ms, True)
    return P @ mec + mt


def check_elementwise(q, ref, scale, tol, what=""):
    """|q - ref| <= tol * scale entry by entry; returns the largest ratio
    |q - ref| / scale (printed by the callers so the margin is visible)."""
    q = np.asarray(q)
    ref = np.asarray(ref)
    d = np.abs(q - ref)
    ratio = np.max(d / np.maximum(scale, 1e-300)) if d.size else 0.0
    bad = np.flatnonzero(d > tol * scale)
    assert bad.size == 0, (f"{what}: {bad.size} entries beyond {tol:g} x scale; first {bad[:5].tolist()}, "
                           f"max ratio {ratio:.3e}")
    return float(ratio)

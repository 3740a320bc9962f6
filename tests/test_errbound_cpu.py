"""The per-entry error scale used by the GPU parity tests, checked on the CPU:
an application of the two-grid operator computed independently here (scipy
triangular solves: another summation order than the oracle's) agrees with the
oracle's entry by entry within 1e-13 of the scale, and a single entry
perturbed by 1e-9 of its own size is caught at the GPU tests' 1e-12."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from tests import _errbound as E


def _independent_apply(O, A, z, adjoint):
    n = O.n
    perm, L0, U0, P = E._parts(O, A)
    (lrp, lci, lv), (urp, uci, uv) = O.ilut()
    nc = O.nc
    Lc = sp.csr_matrix((lv, lci, lrp), shape=(nc, nc)) + sp.identity(nc)
    Uc = sp.csr_matrix((uv, uci, urp), shape=(nc, nc))
    tri = lambda T, b, lo: spla.spsolve_triangular(sp.csr_matrix(T), b, lower=lo)

    def smooth(v, tr):
        vp = v[perm]
        tp = tri(L0.T, tri(U0.T, vp, True), False) if tr else tri(U0, tri(L0, vp, True), False)
        out = np.empty(n)
        out[perm] = tp
        return out

    if not adjoint:
        t = smooth(z, False)
        rc = P.T @ (z - A @ t)
        ec = tri(Uc, tri(Lc, rc, True), False)
        return t + P @ ec
    ec = tri(Lc.T, tri(Uc.T, P.T @ z, True), False)
    s = z - A.T @ (P @ ec)
    return P @ ec + smooth(s, True)


CASES = {
    "fv2d_rot_48": (lambda: W.scaled("fv2d_rot", 48), {}),
    "rgg_800": (lambda: W.scaled("rgg", 800), {}),
    "fv3d_10_nd": (lambda: W.scaled("fv3d", 10), {"fine_order": 1}),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("adjoint", [False, True])
def test_scale_covers_reordered_rounding(oracle_mod, name, adjoint):
    mk, kw = CASES[name]
    p = mk()
    if adjoint and kw.get("fine_order"):
        pytest.skip("the adjoint runs with fine_order 0 only")
    O = oracle_mod.Oracle(p.rowptr, p.col, p.val, **kw)
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    z = np.random.default_rng(7).uniform(-1, 1, p.n_rows)
    ref = O.apply_adjoint(z) if adjoint else O.apply(z, 0)
    mine = _independent_apply(O, A, z, adjoint)
    scale = E.apply_scale(O, A, z, adjoint=adjoint)
    assert np.all(scale >= np.abs(ref) * (1 - 1e-12))       # a bound of the result itself
    r = E.check_elementwise(mine, ref, scale, 1e-13, name)
    print(f"{name} adjoint={adjoint}: max |diff|/scale = {r:.2e}")
    # one wrong entry, 1e-9 of its own size, is caught
    bad = ref.copy()
    i = int(np.argmax(np.abs(ref)))
    bad[i] *= 1 + 1e-9
    with pytest.raises(AssertionError):
        E.check_elementwise(bad, ref, scale, 1e-12, name)


def test_scale_bounds_fp32_cycle(oracle_mod):
    """The FP32 cycle differs from the FP64 one by FP32 rounding: within a few
    hundred FP32 ulps of the scale, entry by entry."""
    p = W.scaled("fv2d_rot", 48)
    O = oracle_mod.Oracle(p.rowptr, p.col, p.val)
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    z = np.random.default_rng(8).uniform(-1, 1, p.n_rows)
    scale = E.apply_scale(O, A, z)
    r = E.check_elementwise(O.apply(z, 1), O.apply(z, 0), scale, 2e-5, "fp32")
    print(f"fp32 vs fp64: max |diff|/scale = {r:.2e}")

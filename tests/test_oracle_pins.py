"""Pins of the CPU oracle against brute force, dense linear algebra, closed
forms and the paper's worked example (no GPU needed)."""
from __future__ import annotations

import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from tests import _brute as B

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    out = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            out[k] = [float(t) for t in v]
    return out


def _mk(O_mod, A, **kw):
    S = sp.csr_matrix(A)
    S.sort_indices()
    return O_mod.Oracle(S.indptr, S.indices, S.data, **kw)


# ---------------------------------------------------------------- aggregation
def test_counter_example_restriction(oracle_mod):
    """Section 2.1 worked example: G1={1,3}, G2={2,4}; printed P^T; P^T x = 0."""
    g = _read_golden("counter_example_n4.txt")
    n = int(g["N"][0])
    agg = np.array(g["agg"], dtype=np.int32)
    A = 4 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)          # SPD
    O = _mk(oracle_mod, A, agg=agg)
    aptr, amem = O.members()
    PT = np.zeros((O.nc, n))
    for I in range(O.nc):
        PT[I, amem[aptr[I]:aptr[I + 1]]] = 1.0
    assert np.array_equal(PT, np.array([g["PT_row0"], g["PT_row1"]]))
    x = np.array(g["x"])
    assert np.array_equal(PT @ x, np.array(g["PTx"]))
    # A_c = P^T A P stays SPD (Theorem: A > 0 implies A_c > 0) ...
    rp, ci, cv = O.coarse()
    Ac = B.dense(rp, ci, cv, O.nc)
    np.linalg.cholesky(Ac)
    # ... while M = P A_c P^T is singular on x (the theorem's point)
    P = PT.T
    assert abs(x @ (P @ Ac @ P.T) @ x) == 0.0


@pytest.mark.parametrize("seed", range(12))
def test_handshake_equals_greedy_and_is_maximal(oracle_mod, seed):
    """One handshake pass == sequential greedy matching by descending key
    (locally dominant edges), and it is a valid maximal matching."""
    rng = np.random.default_rng(seed)
    nv = int(rng.integers(2, 200))
    dens = float(rng.uniform(0.01, 0.2))
    M = rng.random((nv, nv)) < dens
    M = np.triu(M, 1)
    kind = seed % 4
    if kind == 0:
        W_ = rng.uniform(0.1, 10.0, size=(nv, nv))
    elif kind == 1:      # many exact ties: hash decides
        W_ = rng.integers(1, 3, size=(nv, nv)).astype(float)
    elif kind == 2:      # a path with increasing weights: long chains
        M = np.eye(nv, k=1, dtype=bool)
        W_ = np.tile(np.arange(nv, dtype=float) + 1.0, (nv, 1))
    else:                # weights within one quantisation bin: hash decides
        W_ = 1.0 + 1e-3 * rng.random((nv, nv))
    Wm = np.where(M, W_, 0.0)
    Wm = Wm + Wm.T
    S = sp.csr_matrix(Wm)
    S.sort_indices()
    for qbits in (4, 52):
        mate, rounds = oracle_mod.match_once(S.indptr, S.indices, S.data, qbits=qbits)
        edges = B.dict_graph(S.indptr, S.indices, S.data)
        seedv = oracle_mod.default_options()["seed"]
        ref = B.greedy_matching(nv, edges, qbits, seedv)
        assert list(mate) == ref
        for v in range(nv):
            if mate[v] >= 0:
                assert mate[mate[v]] == v and (v, int(mate[v])) in edges
        assert B.is_maximal(nv, edges, list(mate))


@pytest.mark.parametrize("case", ["fv2d_16", "fv3d_6", "rand_mm", "rand_int"])
def test_multipass_aggregation_matches_reference(oracle_mod, case):
    """The full multi-pass aggregation equals iterated greedy matching on
    aggregate graphs built from the fine graph (brute force)."""
    rng = np.random.default_rng(7)
    if case == "fv2d_16":
        p = W.scaled("fv2d", 16)
        rp, ci, v = p.rowptr, p.col, p.val
    elif case == "fv3d_6":
        p = W.fv_problem(6, 3, 1, -6, 6, W.velocity_const((1, 1, 1)), 3)
        rp, ci, v = p.rowptr, p.col, p.val
    elif case == "rand_mm":
        rp, ci, v, _ = B.random_mmatrix(150, rng, 0.05)
    else:
        rp, ci, v, _ = B.random_mmatrix(120, rng, 0.06, integer=True)
    opts = oracle_mod.default_options()
    for cf in (2.0, 4.0, 8.0):
        ref, passes = B.multipass_aggregation(rp, ci, v, cf, opts["max_passes"], opts["qbits"],
                                              opts["seed"])
        # numbering by smallest fine index
        O = oracle_mod.Oracle(rp, ci, v, cf=cf, coarse_order=0)
        agg = O.aggregates()
        assert np.array_equal(agg, ref)
        assert O.passes == passes
        # nested-dissection numbering of the same aggregates
        nc = int(ref.max()) + 1
        perm = B.nd_order_ref(nc, B.coarse_pattern_adj(rp, ci, ref, nc))
        rank = np.empty(nc, dtype=np.int64)
        rank[np.array(perm)] = np.arange(nc)
        Ond = oracle_mod.Oracle(rp, ci, v, cf=cf, coarse_order=1)
        assert np.array_equal(Ond.aggregates(), rank[ref])
        agg = O.aggregates()
        # P: one 1 per row (P 1 = 1), columns non-empty, ids ordered by first member
        assert agg.min() == 0 and agg.max() == O.nc - 1
        firsts = [np.flatnonzero(agg == I)[0] for I in range(O.nc)]
        assert np.all(np.diff(firsts) > 0)
        aptr, amem = O.members()
        assert np.array_equal(np.diff(aptr), np.bincount(agg, minlength=O.nc))


# ------------------------------------------------------------------ galerkin
@pytest.mark.parametrize("integer", [True, False])
def test_galerkin_equals_dense_PtAP(oracle_mod, integer):
    rng = np.random.default_rng(3 + integer)
    rp, ci, v, A = B.random_mmatrix(160, rng, 0.05, integer=integer)
    O = oracle_mod.Oracle(rp, ci, v, cf=3.0)
    P = B.prolongation(O.aggregates(), O.nc)
    Ac_dense = P.T @ A @ P
    crp, cci, cv = O.coarse()
    Ac = B.dense(crp, cci, cv, O.nc)
    if integer:
        assert np.array_equal(Ac, Ac_dense)          # exact sums of integers
    else:
        assert np.max(np.abs(Ac - Ac_dense)) <= 1e-15 * np.max(np.abs(Ac_dense)) * 8
    # pattern: (I,J) stored iff some a_kl with k in G_I, l in G_J is stored
    Pat = (P.T @ (A != 0).astype(float) @ P) != 0
    assert np.array_equal(Pat, Ac != 0 if integer else Pat)
    S = sp.csr_matrix((np.ones_like(cv), cci, crp), shape=(O.nc, O.nc)).toarray() != 0
    assert np.array_equal(S, Pat)
    # M-matrix preserved (Theorem Th:Mprop): positive diagonal, non-positive off-diagonal,
    # diagonally dominant rows
    d = np.diag(Ac)
    off = Ac - np.diag(d)
    assert np.all(d > 0) and np.all(off <= 0)
    assert np.all(d >= np.abs(off).sum(axis=1) * (1 - 1e-14))


def test_galerkin_spd(oracle_mod):
    """A SPD implies A_c SPD (Section 2.1)."""
    rng = np.random.default_rng(11)
    rp, ci, v, A = B.random_mmatrix(140, rng, 0.05, sym=True)
    np.linalg.cholesky(A)
    O = oracle_mod.Oracle(rp, ci, v, cf=4.0)
    crp, cci, cv = O.coarse()
    Ac = B.dense(crp, cci, cv, O.nc)
    # symmetric up to the summation order of the two mirrored double sums
    assert np.abs(Ac - Ac.T).max() <= 1e-14 * np.abs(Ac).max()
    np.linalg.cholesky(0.5 * (Ac + Ac.T))


# ------------------------------------------------------------------ ILU(0)
@pytest.mark.parametrize("case", ["fv2d", "rand"])
def test_ilu0_reproduces_A_on_pattern(oracle_mod, case):
    if case == "fv2d":
        p = W.scaled("fv2d", 24)
        rp, ci, v = p.rowptr, p.col, p.val
        A = B.dense(rp, ci, v)
    else:
        rp, ci, v, A = B.random_mmatrix(120, np.random.default_rng(5), 0.08)
    O = oracle_mod.Oracle(rp, ci, v)
    F = B.dense(rp, ci, O.ilu0())
    n = A.shape[0]
    L = np.tril(F, -1) + np.eye(n)
    U = np.triu(F)
    mask = A != 0
    # pattern of the factors is pattern(A)
    assert np.all((F != 0) <= mask)
    err = np.abs((L @ U - A)[mask]).max() / np.abs(A).max()
    assert err < 1e-14


def test_ilu0_tridiagonal_is_exact_lu(oracle_mod):
    n = 50
    rng = np.random.default_rng(2)
    A = np.diag(rng.uniform(3, 4, n)) - np.diag(rng.uniform(0.1, 1, n - 1), 1) \
        - np.diag(rng.uniform(0.1, 1, n - 1), -1)
    O = _mk(oracle_mod, A)
    S = sp.csr_matrix(A)
    F = B.dense(S.indptr, S.indices, O.ilu0())
    L, U = B.lu_nopivot(A)
    assert np.allclose(np.tril(F, -1) + np.eye(n), L, rtol=1e-14, atol=1e-15)
    assert np.allclose(np.triu(F), U, rtol=1e-14, atol=1e-15)


# ------------------------------------------------------------------ ILUT
def _ilut_dense(O):
    (lrp, lci, lv), (urp, uci, uv) = O.ilut()
    nc = O.nc
    L = B.dense(lrp, lci, lv, nc) + np.eye(nc)
    U = B.dense(urp, uci, uv, nc)
    return L, U


def test_ilut_tau0_is_dense_lu(oracle_mod):
    p = W.scaled("fv2d", 16)
    O = oracle_mod.Oracle(p.rowptr, p.col, p.val, ilut_tau=0.0)
    crp, cci, cv = O.coarse()
    Ac = B.dense(crp, cci, cv, O.nc)
    L, U = _ilut_dense(O)
    Lr, Ur = B.lu_nopivot(Ac)
    assert np.allclose(L, Lr, rtol=1e-12, atol=1e-14)
    assert np.allclose(U, Ur, rtol=1e-12, atol=1e-12 * np.abs(Ur).max())


def test_ilut_huge_tau_is_diagonal(oracle_mod):
    p = W.scaled("fv2d", 16)
    O = oracle_mod.Oracle(p.rowptr, p.col, p.val, ilut_tau=1e300)
    crp, cci, cv = O.coarse()
    Ac = B.dense(crp, cci, cv, O.nc)
    L, U = _ilut_dense(O)
    assert np.array_equal(L, np.eye(O.nc))
    assert np.array_equal(U, np.diag(np.diag(Ac)))


def _read_fractions(name):
    """tests/golden file of 'key i j value' lines with rational values."""
    from fractions import Fraction
    out = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, *v = line.split()
            if k == "tau":
                out["tau"] = Fraction(v[0])
            else:
                out.setdefault(k, {})[(int(v[0]), int(v[1]))] = Fraction(v[2])
    return out


def check_ilut_hand_fixture(oracle_mod):
    """The oracle's ILUT(tau) on the hand-worked 5 x 5 example: every kept and
    dropped entry of L~ and U~ as derived in tests/golden/ilut_hand_5x5.txt
    (drop test before the pivot division, 2-norm of the original row, final
    drop of small U entries)."""
    g = _read_fractions("ilut_hand_5x5.txt")
    n = 5
    A = np.zeros((n, n))
    for (i, j), v in g["A"].items():
        A[i, j] = float(v)
    # P = I (aggregates given as the identity, numbered by smallest index), so
    # A_c = A and the coarse ILUT is the ILUT of the example itself
    O = _mk(oracle_mod, A, agg=np.arange(n, dtype=np.int32), coarse_order=0,
            ilut_tau=float(g["tau"]))
    (lrp, lci, lv), (urp, uci, uv) = O.ilut()
    got_l = {(i, int(lci[p])): lv[p] for i in range(n) for p in range(lrp[i], lrp[i + 1])}
    got_u = {(i, int(uci[p])): uv[p] for i in range(n) for p in range(urp[i], urp[i + 1])}
    assert set(got_l) == set(g["L"]), sorted(got_l)
    assert set(got_u) == set(g["U"]), sorted(got_u)
    for key, v in g["L"].items():
        assert abs(got_l[key] - float(v)) <= 4e-16 * abs(float(v)), (key, got_l[key], v)
    for key, v in g["U"].items():
        assert abs(got_u[key] - float(v)) <= 4e-16 * abs(float(v)), (key, got_u[key], v)
    # U rows store the diagonal first
    assert all(uci[urp[i]] == i for i in range(n))


def test_ilut_hand_worked_example(oracle_mod):
    check_ilut_hand_fixture(oracle_mod)


def test_ilut_nnz_monotone(oracle_mod):
    """Fill shrinks as tau grows (ILUT(0) is the complete LU)."""
    p = W.scaled("fv3d", 12)
    prev = None
    for tau in (0.0, 1e-6, 1e-4, 1e-2, 1.0):
        O = oracle_mod.Oracle(p.rowptr, p.col, p.val, ilut_tau=tau, cf=4.0)
        nz = O.nnz_lc + O.nnz_uc
        if prev is not None:
            assert nz <= prev
        prev = nz


def check_ilut_error_table(oracle_mod, sizes=(30, 40)):
    """Table T:norm: on JUMP3D (DC1 3D) the ILUT(1e-4) factor error
    ||A_c - L~U~||_2 / ||A_c||_2 lies within a factor 3 of the paper's value
    for the numbering used (NO column: coarse_order 0; ND column: 1)."""
    g = _read_golden("ilut_factor_error_jump3d.txt")
    for n in sizes:
        col = g["h_inv"].index(float(n))
        kap = W.dc1_kappa(n, 3)
        rp, ci, v = W.fv_matrix(n, 3, kap, None)
        for order, key in ((0, "rel_err_NO"), (1, "rel_err_ND")):
            O = oracle_mod.Oracle(rp, ci, v, ilut_tau=1e-4, cf=4.0, coarse_order=order)
            crp, cci, cv = O.coarse()
            Ac = sp.csr_matrix((cv, cci, crp), shape=(O.nc, O.nc))
            (lrp, lci, lv), (urp, uci, uv) = O.ilut()
            L = sp.csr_matrix((lv, lci, lrp), shape=(O.nc, O.nc)) + sp.identity(O.nc)
            U = sp.csr_matrix((uv, uci, urp), shape=(O.nc, O.nc))
            E = (L @ U - Ac).tocsr()
            two = lambda M: sp.linalg.svds(M, k=1, return_singular_vectors=False, random_state=0)[0]
            err = two(E) / two(Ac)
            paper = g[key][col]
            assert paper / 3 < err < paper * 3, (n, key, err, paper)


def test_ilut_error_matches_table_tnorm(oracle_mod):
    check_ilut_error_table(oracle_mod)


# ------------------------------------------------------------ preconditioner
def _dense_parts(O, rp, ci, v):
    n = O.n
    A = B.dense(rp, ci, v)
    F = B.dense(rp, ci, O.ilu0())
    S = (np.tril(F, -1) + np.eye(n)) @ np.triu(F)
    L, U = _ilut_dense(O)
    P = B.prolongation(O.aggregates(), O.nc)
    Mi = P @ np.linalg.inv(L @ U) @ P.T
    Si = np.linalg.inv(S)
    return A, S, Si, Mi, P


@pytest.mark.parametrize("case", ["fv2d", "rgg"])
def test_preconditioner_matches_dense_twogrid(oracle_mod, case):
    """Apply == dense B~^{-1} = S^{-1} + M~^{-1} - M~^{-1} A S^{-1} (Eq. (twogrid),
    Algorithm 1); the two-solve form agrees; the error propagator factors as
    (I - M~^{-1} A)(I - S^{-1} A); the adjoint apply is the exact transpose."""
    if case == "fv2d":
        p = W.scaled("fv2d", 20)
    else:
        p = W.scaled("rgg", 400)
    rp, ci, v = p.rowptr, p.col, p.val
    O = oracle_mod.Oracle(rp, ci, v)
    A, S, Si, Mi, P = _dense_parts(O, rp, ci, v)
    Binv = Si + Mi - Mi @ A @ Si
    rng = np.random.default_rng(0)
    Z = rng.standard_normal((O.n, 4))
    for z in Z.T:
        ref = Binv @ z
        sc = np.abs(ref).max()
        assert np.abs(O.apply(z) - ref).max() <= 1e-11 * sc
        assert np.abs(O.apply_twosolve(z) - ref).max() <= 1e-11 * sc
        reft = Binv.T @ z
        assert np.abs(O.apply_adjoint(z) - reft).max() <= 1e-11 * np.abs(reft).max()
    I = np.eye(O.n)
    E = I - Binv @ A
    E2 = (I - Mi @ A) @ (I - Si @ A)
    assert np.abs(E - E2).max() <= 1e-9 * max(1.0, np.abs(E).max())
    # coarse correction annihilates the coarse space when exact: (I - P Ac^-1 P^T A) P = 0
    crp, cci, cv = O.coarse()
    Ac = B.dense(crp, cci, cv, O.nc)
    assert np.abs((I - P @ np.linalg.inv(Ac) @ P.T @ A) @ P).max() < 1e-9


@pytest.mark.parametrize("case", ["fv2d", "rgg"])
def test_exact_coarse_solve_is_twogrid_with_inverse(oracle_mod, case):
    """ILUT with tau = 0 (the exact coarse solve of the paper's EGMG) makes the
    preconditioner the two-grid operator with M~^{-1} = P A_c^{-1} P^T itself,
    A_c^{-1} taken by numpy's pivoted dense inverse; tau > 0 does not."""
    p = W.scaled("fv2d", 20) if case == "fv2d" else W.scaled("rgg", 400)
    rp, ci, v = p.rowptr, p.col, p.val
    O = oracle_mod.Oracle(rp, ci, v, ilut_tau=0.0)
    A, S, Si, _, P = _dense_parts(O, rp, ci, v)
    crp, cci, cv = O.coarse()
    Mi = P @ np.linalg.inv(B.dense(crp, cci, cv, O.nc)) @ P.T
    Binv = Si + Mi - Mi @ A @ Si
    z = np.random.default_rng(7).standard_normal(O.n)
    ref = Binv @ z
    assert np.abs(O.apply(z) - ref).max() <= 1e-11 * np.abs(ref).max()
    inexact = oracle_mod.Oracle(rp, ci, v, ilut_tau=1e-2).apply(z)
    assert np.abs(inexact - ref).max() > 1e-6 * np.abs(ref).max()


def test_preconditioner_fp32_close_to_fp64(oracle_mod):
    p = W.scaled("fv2d", 32)
    O = oracle_mod.Oracle(p.rowptr, p.col, p.val)
    z = np.random.default_rng(1).uniform(-1, 1, O.n)
    q64 = O.apply(z, 0)
    q32 = O.apply(z, 1)
    rel = np.linalg.norm(q32 - q64) / np.linalg.norm(q64)
    assert 0 < rel < 1e-3


def test_coarse_jacobi_mode_converges_to_exact(oracle_mod):
    """Jacobi sweeps on a triangular factor are exact after (levels) sweeps."""
    p = W.scaled("fv2d", 12)
    O0 = oracle_mod.Oracle(p.rowptr, p.col, p.val)
    O1 = oracle_mod.Oracle(p.rowptr, p.col, p.val, coarse_mode=1, coarse_sweeps=O0.nc)
    z = np.random.default_rng(4).standard_normal(O0.n)
    a, b = O0.apply(z), O1.apply(z)
    assert np.abs(a - b).max() <= 1e-10 * np.abs(a).max()


def check_jacobi_closed_form(oracle_mod, sweeps=(1, 2, 3)):
    """coarse_mode 1 with k sweeps (the parallel inexact coarse solve of
    Section 2's outlook): y_k = sum_{i<=k} (I - L~)^i r_c from y_0 = r_c, then
    e_k = sum_{i<=k} (-D^{-1} N)^i D^{-1} y_k with U~ = D + N, written out
    densely; the rest of the two-grid application as Algorithm 1."""
    p = W.scaled("fv2d", 12)
    A = B.dense(p.rowptr, p.col, p.val)
    n = A.shape[0]
    z = np.random.default_rng(4).standard_normal(n)
    for k in sweeps:
        O = oracle_mod.Oracle(p.rowptr, p.col, p.val, coarse_mode=1, coarse_sweeps=k)
        F = B.dense(p.rowptr, p.col, O.ilu0())
        L0 = np.tril(F, -1) + np.eye(n)
        U0 = np.triu(F)
        t = np.linalg.solve(U0, np.linalg.solve(L0, z))
        P = B.prolongation(O.aggregates(), O.nc)
        rc = P.T @ (z - A @ t)
        Lc, Uc = _ilut_dense(O)
        NL = Lc - np.eye(O.nc)
        D = np.diag(np.diag(Uc))
        Dinv = np.diag(1.0 / np.diag(Uc))
        NU = Uc - D
        y = np.zeros(O.nc)
        term = rc.copy()
        for _ in range(k + 1):
            y += term
            term = -NL @ term
        e = np.zeros(O.nc)
        term = Dinv @ y
        for _ in range(k + 1):
            e += term
            term = -Dinv @ (NU @ term)
        q = t + P @ e
        got = O.apply(z)
        assert np.abs(got - q).max() <= 1e-12 * np.abs(q).max(), (k, np.abs(got - q).max())
        # and it is not the exact coarse solve (k is below the factors' depth)
        ex = t + P @ np.linalg.solve(Uc, np.linalg.solve(Lc, rc))
        assert np.abs(ex - q).max() > 1e-6 * np.abs(q).max()


def test_coarse_jacobi_closed_form(oracle_mod):
    check_jacobi_closed_form(oracle_mod)


# -------------------------------------------------------------------- FGMRES
@pytest.mark.parametrize("case", ["fv2d_64", "rgg_1500", "fv3d_10"])
def test_solve_matches_dense_solution(oracle_mod, case):
    if case == "fv2d_64":
        p = W.make("fv2d_64")
    elif case == "rgg_1500":
        p = W.scaled("rgg", 1500)
    else:
        p = W.scaled("fv3d", 12)
    A = sp.csr_matrix((p.val, p.col, p.rowptr))
    b = p.b[:, 0]
    O = oracle_mod.Oracle(p.rowptr, p.col, p.val)
    tol = 1e-8
    x, info = O.solve(b, tol=tol)
    assert info.status == oracle_mod.OK
    r = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert r < tol and abs(r - info.relres) <= 1e-12
    xd = sp.linalg.spsolve(A.tocsc(), b)
    assert np.linalg.norm(A @ (x - xd)) / np.linalg.norm(b) <= tol * 1.01
    lam, info2 = O.solve(b, tol=tol, adjoint=True)
    assert info2.status == oracle_mod.OK
    assert np.linalg.norm(b - A.T @ lam) / np.linalg.norm(b) < tol


def test_fgmres_iterate_is_least_squares_minimiser(oracle_mod):
    """x_j minimises ||b - A x|| over x0 + span(Z_j) (one cycle, tiny N);
    residual estimates are non-increasing and equal the true residual."""
    p = W.scaled("fv2d", 10)
    A = B.dense(p.rowptr, p.col, p.val)
    b = p.b[:, 0]
    O = oracle_mod.Oracle(p.rowptr, p.col, p.val)
    for j in (1, 3, 7):
        x, info, ex = O.solve(b, tol=0.0, maxit=j, restart=30, zdump=True, history=True)
        Z = ex["Z"][:j].T
        y, *_ = np.linalg.lstsq(A @ Z, b, rcond=None)
        xls = Z @ y
        assert np.linalg.norm(A @ (x - xls)) <= 1e-10 * np.linalg.norm(b)
        h = ex["history"]
        assert np.all(np.diff(h) <= 1e-15)
        assert abs(h[-1] - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) < 1e-10


def test_fgmres_exact_preconditioner_one_step(oracle_mod):
    """B~^{-1} = A^{-1} in two special cases, so one step converges:
    (i) tridiagonal A (ILU(0) is exact LU); (ii) P = I with ILUT(0)."""
    n = 60
    rng = np.random.default_rng(8)
    A = np.diag(rng.uniform(3, 4, n)) - np.diag(rng.uniform(0.1, 1, n - 1), 1) \
        - np.diag(rng.uniform(0.1, 1, n - 1), -1)
    b = rng.uniform(-1, 1, n)
    O = _mk(oracle_mod, A)
    x, info = O.solve(b, tol=1e-12)
    assert info.steps == 1 and info.status == 0
    p = W.scaled("rgg", 300)
    O2 = oracle_mod.Oracle(p.rowptr, p.col, p.val, agg=np.arange(300, dtype=np.int32), ilut_tau=0.0)
    x, info = O2.solve(p.b[:, 0], tol=1e-12)
    assert info.steps == 1 and info.status == 0


def test_fgmres_full_space_converges(oracle_mod):
    """With restart >= N, GMRES reaches the exact solution in <= N steps."""
    rp, ci, v, A = B.random_mmatrix(40, np.random.default_rng(9), 0.1)
    O = oracle_mod.Oracle(rp, ci, v, ilut_tau=1e30)     # weak coarse solve
    b = np.random.default_rng(10).uniform(-1, 1, 40)
    x, info = O.solve(b, tol=1e-13, restart=40, maxit=40)
    assert info.steps <= 40 and info.status == 0


def test_fgmres_fp32_preconditioner_converges(oracle_mod):
    p = W.make("fv2d_64")
    A = sp.csr_matrix((p.val, p.col, p.rowptr))
    b = p.b[:, 0]
    O = oracle_mod.Oracle(p.rowptr, p.col, p.val)
    x64, _ = O.solve(b)
    x32, info = O.solve(b, precision=1)
    assert info.status == 0
    assert np.linalg.norm(b - A @ x32) / np.linalg.norm(b) < 1e-8
    assert np.linalg.norm(x32 - x64) / np.linalg.norm(x64) < 1e-5


def test_error_codes(oracle_mod):
    # zero pivot: a 2x2 matrix with a zero leading entry (pivoting would be needed)
    A = np.array([[0.0, 1.0], [1.0, 1.0]])
    with pytest.raises(oracle_mod.OracleError) as e:
        _mk(oracle_mod, A, agg=np.array([0, 1], dtype=np.int32))
    assert e.value.code in (oracle_mod.ERR_ZERO_PIVOT, oracle_mod.ERR_INVALID)
    # missing diagonal
    rp = np.array([0, 1, 2], dtype=np.int32)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.Oracle(rp, np.array([1, 0], dtype=np.int32), np.array([1.0, 1.0]))
    # non-finite entry
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.Oracle(np.array([0, 1], dtype=np.int32), np.array([0], dtype=np.int32),
                          np.array([np.nan]))
    assert e.value.code == oracle_mod.ERR_NONFINITE
    # not converged within maxit
    p = W.scaled("fv2d", 16)
    O = oracle_mod.Oracle(p.rowptr, p.col, p.val)
    _, info = O.solve(p.b[:, 0], tol=1e-12, maxit=2)
    assert info.status == oracle_mod.NOT_CONVERGED and info.steps == 2


def test_zero_coarse_pivot_is_an_error(oracle_mod):
    """Two chains of four unknowns, weakly coupled: matching aggregates each
    chain (brute-force aggregation agrees), the first chain's entries sum to
    zero, so A_c = [[0, -0.1], [-0.1, 4]]: ILU(0) of A succeeds, the coarse
    factorisation without pivoting meets a zero pivot and says so."""
    A = np.zeros((8, 8))
    for o, d in ((0, (3.0, 3.0, 2.5, 0.5)), (4, (3.5, 3.0, 3.0, 3.5))):
        A[o, o + 1] = A[o + 1, o] = -2.0
        A[o + 1, o + 2] = A[o + 2, o + 1] = -0.5
        A[o + 2, o + 3] = A[o + 3, o + 2] = -2.0
        for k in range(4):
            A[o + k, o + k] = d[k]
    A[3, 4] = A[4, 3] = -0.1
    M = sp.csr_matrix(A)
    M.sort_indices()
    o = oracle_mod.default_options()
    agg, _ = B.multipass_aggregation(M.indptr, M.indices, M.data, 4.0, 8, o["qbits"], o["seed"])
    assert np.array_equal(agg, [0, 0, 0, 0, 1, 1, 1, 1])
    P = B.prolongation(agg, 2)
    assert np.array_equal(P.T @ A @ P, np.array([[0.0, -0.1], [-0.1, 4.0]]))
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.Oracle(M.indptr, M.indices, M.data, coarse_order=0, ilut_tau=0.0)
    assert e.value.code == oracle_mod.ERR_ZERO_PIVOT
    A[3, 3] = 1.5
    M = sp.csr_matrix(A)
    M.sort_indices()
    assert oracle_mod.Oracle(M.indptr, M.indices, M.data, coarse_order=0, ilut_tau=0.0).nc == 2


def test_nested_dissection_numbering(oracle_mod):
    """ND numbering of a grid-like coarse graph: equals the recursive definition;
    at every dissection step the separator (numbered last) disconnects the two
    parts numbered before it (checked on A_c itself); ILUT depth drops versus
    the smallest-fine-index numbering."""
    p = W.scaled("fv2d", 96)
    O0 = oracle_mod.Oracle(p.rowptr, p.col, p.val, coarse_order=0)
    O1 = oracle_mod.Oracle(p.rowptr, p.col, p.val, coarse_order=1)
    a0, a1 = O0.aggregates(), O1.aggregates()
    nc = O0.nc
    perm = B.nd_order_ref(nc, B.coarse_pattern_adj(p.rowptr, p.col, a0, nc))
    rank = np.empty(nc, dtype=np.int64)
    rank[np.array(perm)] = np.arange(nc)
    assert np.array_equal(a1, rank[a0])
    # same aggregates, same A_c up to the permutation
    r0, c0, v0 = O0.coarse()
    r1, c1, v1 = O1.coarse()
    A0 = sp.csr_matrix((v0, c0, r0), shape=(nc, nc)).toarray()
    A1 = sp.csr_matrix((v1, c1, r1), shape=(nc, nc)).toarray()
    assert np.array_equal(A1, A0[np.ix_(perm, perm)])
    # every dissection step of the definition: the two parts numbered before
    # a separator are not coupled in A_c (numbered as the oracle numbers them)
    nodes = []
    B.nd_order_ref(nc, B.coarse_pattern_adj(p.rowptr, p.col, a0, nc), nodes=nodes)
    dissected = [t for t in nodes if t[3] > 0]
    assert dissected and dissected[0][0] == 0 and dissected[0][1] + dissected[0][2] + dissected[0][3] == nc
    for start, na, nb, ns in nodes:
        blk = A1[start:start + na, start + na:start + na + nb]
        assert not blk.any() and not A1[start + na:start + na + nb, start:start + na].any(), (start, na, nb, ns)
        if ns > 0:
            assert na > 0 and nb > 0 and ns < na + nb

    def depth(rp, ci):
        lev = np.zeros(len(rp) - 1, dtype=int)
        for i in range(len(rp) - 1):
            c = ci[rp[i]:rp[i + 1]]
            c = c[c < i]
            lev[i] = lev[c].max() + 1 if len(c) else 0
        return lev.max() + 1
    (l0, *_), _u0 = O0.ilut()
    (l1, *_), _u1 = O1.ilut()
    d0 = depth(l0, O0.ilut()[0][1])
    d1 = depth(l1, O1.ilut()[0][1])
    assert d1 < d0


# ------------------------------------------------------ GMG-ND fine smoother
def _nd_case(name):
    if name == "fv2d_24":
        p = W.scaled("fv2d", 24)
    elif name == "fv3d_8":
        p = W.scaled("fv3d", 8)
    else:
        p = W.scaled("rgg", 500)
    return p.rowptr, p.col, p.val, p.n_rows


@pytest.mark.parametrize("case", ["fv2d_24", "fv3d_8", "rgg_500"])
def test_color_order(oracle_mod, case):
    """Multicolour smoother numbering (fine_order 2): on 5- and 7-point grids
    the greedy colouring is red-black, so the numbering is the cells with
    even coordinate sum, ascending, then the odd ones; on any graph the
    colouring is proper and each vertex has the smallest colour its earlier
    neighbours leave free (brute force), and the numbering sorts by colour."""
    rp, ci, v, n = _nd_case(case)
    O = oracle_mod.Oracle(rp, ci, v, fine_order=2)
    perm, _ = O.fine()
    if case != "rgg_500":
        g = round(n ** 0.5) if case == "fv2d_24" else round(n ** (1 / 3))
        idx = np.arange(n)
        par = (idx % g + (idx // g) % g + (idx // (g * g))) % 2
        assert np.array_equal(perm, np.concatenate([idx[par == 0], idx[par == 1]]))
    adj = B.coarse_pattern_adj(rp, ci, np.arange(n), n)
    color = [0] * n
    for i in range(n):
        used = {color[j] for j in adj[i] if j < i}
        c = 0
        while c in used:
            c += 1
        color[i] = c
    assert all(color[i] != color[j] for i in range(n) for j in adj[i])
    assert np.array_equal(perm, np.array(sorted(range(n), key=lambda i: (color[i], i))))


@pytest.mark.parametrize("fine_order", [1, 2])
@pytest.mark.parametrize("case", ["fv2d_24", "fv3d_8", "rgg_500"])
def test_fine_nd_smoother(oracle_mod, case, fine_order):
    """GMG-ND (Section 3.1 variants) and the multicolour smoother: the smoother
    is ILU(0) of A renumbered by nested dissection (fine_order 1; the
    numbering equals the recursive definition on A's graph) or by colour
    classes (fine_order 2; numbering pinned above); F = A[perm][:, perm]; its factors satisfy the ILU(0) definition
    (L U = F on F's pattern); the preconditioner and its adjoint equal the
    dense Eq. (twogrid) operator built with S = Q^T L U Q."""
    rp, ci, v, n = _nd_case(case)
    O = oracle_mod.Oracle(rp, ci, v, fine_order=fine_order)
    perm, (frp, fci, fv) = O.fine()
    if fine_order == 1:
        ref = B.nd_order_ref(n, B.coarse_pattern_adj(rp, ci, np.arange(n), n))
        assert np.array_equal(perm, np.array(ref))
    assert not np.array_equal(perm, np.arange(n))
    A = B.dense(rp, ci, v)
    F = B.dense(frp, fci, fv)
    assert np.array_equal(F, A[np.ix_(perm, perm)])
    Fi = B.dense(frp, fci, O.ilu0())
    L = np.tril(Fi, -1) + np.eye(n)
    U = np.triu(Fi)
    pat = F != 0
    assert np.allclose((L @ U)[pat], F[pat], rtol=1e-12, atol=1e-12 * np.abs(F).max())
    # dense two-grid operator
    LU = L @ U
    Q = np.zeros((n, n))
    Q[np.arange(n), perm] = 1.0                        # (Q x)_k = x[perm[k]]
    Sinv = Q.T @ np.linalg.inv(LU) @ Q
    (lrp, lci, lv), (urp, uci, uv) = O.ilut()
    Lc = B.dense(lrp, lci, lv, O.nc) + np.eye(O.nc)
    Uc = B.dense(urp, uci, uv, O.nc)
    P = B.prolongation(O.aggregates(), O.nc)
    Minv = P @ np.linalg.inv(Lc @ Uc) @ P.T
    Binv = Sinv + Minv @ (np.eye(n) - A @ Sinv)
    z = np.random.default_rng(5).uniform(-1, 1, n)
    q = O.apply(z)
    assert np.allclose(q, Binv @ z, rtol=1e-9, atol=1e-9 * np.abs(Binv @ z).max())
    qa = O.apply_adjoint(z)
    assert np.allclose(qa, Binv.T @ z, rtol=1e-9, atol=1e-9 * np.abs(Binv.T @ z).max())
    # the natural numbering is the same operator with Q = I
    O0 = oracle_mod.Oracle(rp, ci, v, fine_order=0)
    p0, (r0, c0, v0) = O0.fine()
    assert np.array_equal(p0, np.arange(n)) and np.array_equal(r0, rp) and np.array_equal(v0, v)


def test_fine_nd_exact_on_dense_blocks(oracle_mod):
    """Block-diagonal A with dense, diagonally dominant blocks of at most 40
    rows under a shuffled numbering: ILU(0) keeps every entry of each block, so
    the smoother is exact in either numbering and the preconditioner is A^{-1}
    (any mix-up of the permutation's two directions breaks this)."""
    rng = np.random.default_rng(11)
    sizes = [int(s) for s in rng.integers(5, 41, size=12)]
    n = sum(sizes)
    A = np.zeros((n, n))
    o = 0
    for s in sizes:
        Bk = rng.uniform(-1, 1, (s, s))
        Bk[np.arange(s), np.arange(s)] = np.abs(Bk).sum(axis=1) + 1.0
        A[o:o + s, o:o + s] = Bk
        o += s
    sh = rng.permutation(n)
    A = A[np.ix_(sh, sh)]
    z = rng.uniform(-1, 1, n)
    x = np.linalg.solve(A, z)
    for fo in (0, 1):
        O = _mk(oracle_mod, A, fine_order=fo)
        q = O.apply(z)
        assert np.allclose(q, x, rtol=1e-10, atol=1e-10 * np.abs(x).max()), fo
    perm, _ = _mk(oracle_mod, A, fine_order=1).fine()
    assert not np.array_equal(perm, np.arange(n))


# ------------------------------------------------- SPAI coarse solve (mode 2)
@pytest.mark.parametrize("case", ["fv2d_24", "rgg_500"])
def test_spai_columns_minimise_the_residual(oracle_mod, case):
    """Each column of the sparse approximate inverse is the least-squares
    minimiser of ||A_c m - e_j|| over A_c's column pattern: equal to an SVD
    least-squares solve of the same problem, and its residual is orthogonal
    to the columns it may use (normal equations)."""
    rp, ci, v, n = _nd_case(case)
    O = oracle_mod.Oracle(rp, ci, v, coarse_mode=2)
    crp, cci, cv = O.coarse()
    Ac = B.dense(crp, cci, cv, O.nc)
    mrp, mci, mv = O.spai()
    assert np.array_equal(mrp, crp) and np.array_equal(mci, cci)   # A_c's pattern
    M = B.dense(mrp, mci, mv, O.nc)
    pat = B.dense(crp, cci, np.ones_like(cv), O.nc) != 0          # stored entries, zeros included
    for j in range(O.nc):
        J = np.flatnonzero(pat[:, j])
        e = np.zeros(O.nc)
        e[j] = 1.0
        ref = np.linalg.lstsq(Ac[:, J], e, rcond=None)[0]
        m = M[J, j]
        assert np.allclose(m, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max()), j
        res = Ac[:, J] @ m - e
        assert np.abs(Ac[:, J].T @ res).max() <= 1e-10 * np.abs(Ac[:, J]).max()
        assert np.count_nonzero(M[:, j][np.setdiff1d(np.arange(O.nc), J)]) == 0


def test_spai_special_cases(oracle_mod):
    """A diagonal A_c gives M = D^{-1}; a dense A_c gives M = A_c^{-1}, so the
    SPAI preconditioner equals the exact-coarse-solve one (ILUT tau = 0)."""
    rng = np.random.default_rng(7)
    d = rng.uniform(0.5, 3.0, 40)
    O = _mk(oracle_mod, np.diag(d), coarse_mode=2)
    mrp, mci, mv = O.spai()
    assert np.array_equal(mci, np.arange(40)) and np.allclose(mv, 1.0 / d, rtol=1e-15, atol=0)
    n = 12
    A = rng.uniform(-1, 1, (n, n))
    A[np.arange(n), np.arange(n)] = np.abs(A).sum(axis=1) + 1.0
    agg = np.repeat(np.arange(n // 2), 2).astype(np.int32)
    O2 = _mk(oracle_mod, A, agg=agg, coarse_mode=2)
    crp, cci, cv = O2.coarse()
    Ac = B.dense(crp, cci, cv, O2.nc)
    assert np.all(Ac != 0)
    M = B.dense(*O2.spai(), O2.nc)
    assert np.allclose(M, np.linalg.inv(Ac), rtol=1e-12, atol=1e-13)
    O0 = _mk(oracle_mod, A, agg=agg, coarse_mode=0, ilut_tau=0.0)
    z = rng.uniform(-1, 1, n)
    assert np.allclose(O2.apply(z), O0.apply(z), rtol=1e-12, atol=1e-13)


ADJOINT_VARIANTS = {
    "jacobi1": dict(coarse_mode=1, coarse_sweeps=1),
    "jacobi3": dict(coarse_mode=1, coarse_sweeps=3),
    "spai": dict(coarse_mode=2),
    "nd": dict(fine_order=1),
    "color": dict(fine_order=2),
    "nd_jacobi": dict(fine_order=1, coarse_mode=1, coarse_sweeps=2),
}


def check_adjoint_transpose(oracle_mod, variant="jacobi3", case="fv2d"):
    """The adjoint application of a variant is the transpose of its forward
    application (column by column on the identity), and the adjoint FGMRES
    solves A^T lambda = g."""
    p = W.scaled("fv2d", 12) if case == "fv2d" else W.scaled("rgg", 300)
    rp, ci, v = p.rowptr, p.col, p.val
    O = oracle_mod.Oracle(rp, ci, v, **ADJOINT_VARIANTS[variant])
    n = O.n
    I = np.eye(n)
    Bf = np.column_stack([O.apply(I[:, j]) for j in range(n)])
    Ba = np.column_stack([O.apply_adjoint(I[:, j]) for j in range(n)])
    err = np.abs(Ba - Bf.T).max() / np.abs(Bf).max()
    assert err <= 1e-12, (variant, err)
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    g = np.random.default_rng(1).uniform(-1, 1, n)
    lam, info = O.solve(g, tol=1e-10, restart=n, maxit=n, adjoint=True)
    assert info.status == 0 and np.linalg.norm(g - A.T @ lam) / np.linalg.norm(g) < 1e-10


def check_adjoint_spai(oracle_mod):
    check_adjoint_transpose(oracle_mod, "spai", "fv2d")


@pytest.mark.parametrize("variant", list(ADJOINT_VARIANTS))
@pytest.mark.parametrize("case", ["fv2d", "rgg"])
def test_adjoint_apply_is_transpose_of_variants(oracle_mod, variant, case):
    """For the inexact coarse solves (Jacobi sweeps, sparse approximate
    inverse) and the reordered smoothers (the transposes of Eq. (twogrid)'s
    parts, taken in reverse order)."""
    check_adjoint_transpose(oracle_mod, variant, case)

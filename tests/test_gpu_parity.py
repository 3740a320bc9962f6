"""Parity of the HIP path (through the C ABI) against the CPU oracle.

Bars: integer results (aggregates, patterns) bit-exact; setup values that the
definition fixes in FP64 without multiplications (A_c sums) bit-exact; ILU(0)
and ILUT values bit-exact (same operation order, no contraction); one
preconditioner application in FP64 entry by entry within 1e-13 of the
magnitudes that flow into that entry (tests/_errbound.py; FMA contraction,
reciprocal-multiply and another summation order move each entry by a few ulps
of those magnitudes); iterates at equal step counts within ||A (x - x_oracle)|| /
||b|| <= 1e-10; converged solves at true relative residual < tol.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg  # noqa: F401  (sp.linalg)

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_1105_3468_amd import GmgError, Solver  # noqa: E402
from paper_1105_3468_amd import gmg as G  # noqa: E402
from tests import _errbound as EB  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _elementwise(O, A, z, q, ref, tol, what, adjoint=False, coarse=None):
    """|q - ref| <= tol * scale entry by entry, scale = the magnitudes that
    flow into each entry of the application (tests/_errbound.py)."""
    scale = EB.apply_scale(O, A, z, adjoint=adjoint, coarse=coarse)
    r = EB.check_elementwise(q, ref, scale, tol, what)
    _say(f"  {what}: max |diff|/scale = {r:.2e} (bar {tol:g})")


CASES = {
    "fv2d_64": lambda: W.make("fv2d_64"),
    "fv2d_rot_96": lambda: W.scaled("fv2d_rot", 96),
    "fv3d_20": lambda: W.scaled("fv3d", 20),
    "rgg_3001": lambda: W.scaled("rgg", 3001),
    "fv2d_37": lambda: W.fv_problem(37, 2, 1, -2, 2, W.velocity_const((1.0, 0.5)), 5),
}
# 150 grid rows: three bands of the wavefront sweep, the last one partly
# outside the grid
BAND_CASES = {"fv2d_150": lambda: W.fv_problem(150, 2, 1, -2, 2, W.velocity_const((1.0, 0.5)), 6)}


# coarse numbering: nested dissection (default) and smallest fine index
ORDERS = {"nd": dict(coarse_order=1), "natural": dict(coarse_order=0)}


@pytest.fixture(scope="module", params=[(c, m) for c in CASES for m in ORDERS],
                ids=lambda cm: f"{cm[0]}-{cm[1]}")
def case(request):
    name, mode = request.param
    _say(f"[case] {name} coarse_order={mode}")
    p = CASES[name]()
    O = oracle.Oracle(p.rowptr, p.col, p.val, **ORDERS[mode])
    S = Solver(p.rowptr, p.col, p.val, **ORDERS[mode])
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    return name, p, O, S, A


def test_aggregates_bit_exact(case):
    name, p, O, S, A = case
    agg = S.aggregates().cpu().numpy()
    assert np.array_equal(agg, O.aggregates())
    inf = S.info()
    assert inf["n_coarse"] == O.nc and inf["passes"] == O.passes and inf["rounds"] == O.rounds


def test_coarse_matrix_bit_exact(case):
    name, p, O, S, A = case
    rp, ci, v = (t.cpu().numpy() for t in S.coarse())
    orp, oci, ov = O.coarse()
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
    assert np.array_equal(v.view(np.uint64), ov.view(np.uint64))


def test_ilu0_bit_exact(case):
    name, p, O, S, A = case
    v = S.ilu0().cpu().numpy()
    assert np.array_equal(v.view(np.uint64), O.ilu0().view(np.uint64))


def test_ilut_bit_exact(case):
    name, p, O, S, A = case
    (lrp, lci, lv), (urp, uci, uv) = S.ilut()
    (olrp, olci, olv), (ourp, ouci, ouv) = O.ilut()
    assert np.array_equal(lrp.cpu().numpy(), olrp) and np.array_equal(lci.cpu().numpy(), olci)
    assert np.array_equal(urp.cpu().numpy(), ourp) and np.array_equal(uci.cpu().numpy(), ouci)
    assert np.array_equal(lv.cpu().numpy(), olv) and np.array_equal(uv.cpu().numpy(), ouv)


def test_spmv(case):
    name, p, O, S, A = case
    x = np.random.default_rng(1).uniform(-1, 1, p.n_rows)
    for tr in (False, True):
        y = S.spmv(torch.as_tensor(x, device="cuda"), transposed=tr).cpu().numpy()
        ref = O.spmv(x, transposed=tr)
        sc = np.abs(A).dot(np.abs(x)) if not tr else np.abs(A).T.dot(np.abs(x))
        assert np.all(np.abs(y - ref) <= 1e-14 * sc + 1e-300)


@pytest.mark.parametrize("adjoint", [False, True])
def test_preconditioner_fp64(case, adjoint):
    name, p, O, S, A = case
    rng = np.random.default_rng(2)
    for _ in range(2):
        z = rng.uniform(-1, 1, p.n_rows)
        q = S.apply(torch.as_tensor(z, device="cuda"), precision=0, adjoint=adjoint).cpu().numpy()
        ref = O.apply_adjoint(z) if adjoint else O.apply(z, 0)
        _elementwise(O, A, z, q, ref, 1e-13, f"{name} fp64 adjoint={adjoint}", adjoint=adjoint)


def test_preconditioner_fp32(case):
    """FP32 cycle vs the oracle's FP32 cycle (same roundings of the data, same
    operations, different summation order/contraction): agree to a few FP32
    ulps amplified by the sweeps; and both within FP32 accuracy of FP64."""
    name, p, O, S, A = case
    z = np.random.default_rng(3).uniform(-1, 1, p.n_rows)
    q = S.apply(torch.as_tensor(z, device="cuda"), precision=1).cpu().numpy()
    ref32 = O.apply(z, 1)
    ref64 = O.apply(z, 0)
    e32 = np.linalg.norm(q - ref32) / np.linalg.norm(ref32)
    e64 = np.linalg.norm(ref32 - ref64) / np.linalg.norm(ref64)
    assert e32 <= max(1e-4, 10 * e64), (e32, e64)
    _elementwise(O, A, z, q, ref32, 2e-5, f"{name} fp32")


def test_solve_converges_and_matches_oracle(case):
    name, p, O, S, A = case
    b = p.b[:, 0]
    tol = 1e-8
    x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=tol)
    xh = x.cpu().numpy()
    rel = np.linalg.norm(b - A @ xh) / np.linalg.norm(b)
    assert res.status == G.OK and rel < tol, (name, rel, res.info)
    xo, info = O.solve(b, tol=tol)
    assert abs(res.info["iters"] - info.steps) <= 1, (res.info["iters"], info.steps)
    assert np.linalg.norm(A @ (xh - xo)) / np.linalg.norm(b) <= 2 * tol


@pytest.mark.parametrize("steps", [1, 7, 45])
def test_iterates_equal_steps(case, steps):
    """Same number of FGMRES steps (tol = 0), including a restart at 30."""
    name, p, O, S, A = case
    b = p.b[:, 0]
    x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=0.0, maxit=steps)
    xo, info = O.solve(b, tol=0.0, maxit=steps)
    assert res.info["iters"] == info.steps == steps
    d = np.linalg.norm(A @ (x.cpu().numpy() - xo)) / np.linalg.norm(b)
    assert d <= 1e-10, (name, steps, d)


@pytest.mark.parametrize("steps,restart", [(40, 600), (120, 600), (400, 600), (800, 1000), (130, 45)])
def test_long_basis_iterates(steps, restart):
    """FGMRES past 32 basis vectors, where one Gram-corrected projection
    replaces the two Gram-Schmidt passes, past 384 and 768, where that
    projection runs over blocks of 384 vectors, and restarted at 45 (the Gram
    rows rebuilt every cycle): iterates at equal step counts within 1e-10 of
    the oracle's (modified Gram-Schmidt), the same bar as above."""
    _say(f"[case] long basis, {steps} steps, restart {restart}")
    p = W.scaled("fv2d_rot", 96)
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    S = Solver(p.rowptr, p.col, p.val)
    O = oracle.Oracle(p.rowptr, p.col, p.val)
    b = p.b[:, 0]
    x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=0.0, maxit=steps, restart=restart)
    xo, info = O.solve(b, tol=0.0, maxit=steps, restart=restart)
    assert res.info["iters"] == info.steps == steps
    d = np.linalg.norm(A @ (x.cpu().numpy() - xo)) / np.linalg.norm(b)
    assert d <= 1e-10, (steps, d)


def test_adjoint_solve(case):
    name, p, O, S, A = case
    g = np.random.default_rng(4).uniform(-1, 1, p.n_rows)
    lam, res = S.solve_adjoint(torch.as_tensor(g, device="cuda"), tol=1e-10)
    lh = lam.cpu().numpy()
    assert np.linalg.norm(g - A.T @ lh) / np.linalg.norm(g) < 1e-10
    lo, info = O.solve(g, tol=0.0, maxit=5, adjoint=True)
    l5, r5 = S.solve_adjoint(torch.as_tensor(g, device="cuda"), tol=0.0, maxit=5)
    assert np.linalg.norm(A.T @ (l5.cpu().numpy() - lo)) / np.linalg.norm(g) <= 1e-10


def test_fp32_preconditioned_solve(case):
    name, p, O, S, A = case
    b = p.b[:, 0]
    x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=1e-8, precond_fp32=1)
    xh = x.cpu().numpy()
    assert res.status == G.OK
    assert np.linalg.norm(b - A @ xh) / np.linalg.norm(b) < 1e-8
    xo, _ = O.solve(b, tol=1e-8)
    assert np.linalg.norm(A @ (xh - xo)) / np.linalg.norm(b) <= 2e-8


def test_multi_rhs_and_x0(case):
    name, p, O, S, A = case
    B = np.random.default_rng(5).uniform(-1, 1, (p.n_rows, 3))
    X, res = S.solve(torch.as_tensor(B, device="cuda"), tol=1e-9)
    Xh = X.cpu().numpy()
    for c in range(3):
        assert np.linalg.norm(B[:, c] - A @ Xh[:, c]) / np.linalg.norm(B[:, c]) < 1e-9
    # restart from the solution: converges with zero steps
    X2, res2 = S.solve(torch.as_tensor(B, device="cuda"), tol=1e-9, x0=X)
    assert res2.info["iters"] == 0


def test_deterministic(case):
    name, p, O, S, A = case
    b = torch.as_tensor(p.b[:, 0], device="cuda")
    x1, r1 = S.solve(b, tol=1e-8)
    x2, r2 = S.solve(b, tol=1e-8)
    assert torch.equal(x1, x2) and r1.info["iters"] == r2.info["iters"]


# ------------------------------------------------------------- edge cases
def test_sweep_waves_do_not_change_results():
    """The number of resident sweep waves changes scheduling only, not results
    (device-wide and one-workgroup sweeps)."""
    _say("[case] waves")
    p = W.scaled("fv2d", 48)
    b = torch.as_tensor(p.b[:, 0], device="cuda")
    xs = []
    for kern in (1, 2):
        for w in (0, 4, 64, 2048):
            s = Solver(p.rowptr, p.col, p.val, sweep_waves=w, sweep_kernel=kern)
            xs.append(s.apply(b))
    assert all(torch.equal(xs[0], x) for x in xs[1:])


@pytest.mark.parametrize("kind", ["fv2d_rot_96", "fv3d_20", "fv2d_37", "rgg_3001", "fv2d_150"])
def test_sweep_kernels_bitwise_equal(kind):
    """The level sweeps (single-CU ring, device-wide, one-workgroup LDS, in any
    mix of level ranges) and the wavefront sweep perform the same operations in
    the same order: bitwise-equal preconditioner applications, in FP64 and
    FP32, forward and adjoint.  The tree solve of the coarse factors (the
    default) adds the same terms in another order: within FP64 rounding."""
    _say(f"[case] sweep kernels {kind}")
    p = (CASES[kind] if kind in CASES else BAND_CASES[kind])()
    z = torch.as_tensor(np.random.default_rng(9).uniform(-1, 1, p.n_rows), device="cuda")
    variants = [dict(sweep_kernel=1), dict(sweep_kernel=3), dict(sweep_kernel=2),
                dict(sweep_kernel=3, sweep_wg_chunks=1), dict(sweep_kernel=3, sweep_wg_chunks=64)]
    solvers = [Solver(p.rowptr, p.col, p.val, **c) for c in variants]
    tree = Solver(p.rowptr, p.col, p.val, sweep_kernel=0)
    for prec, adj in ((0, False), (1, False), (0, True)):
        ref = solvers[0].apply(z, precision=prec, adjoint=adj)
        for c, s in zip(variants[1:], solvers[1:]):
            a = s.apply(z, precision=prec, adjoint=adj)
            assert torch.equal(a, ref), (kind, c, prec, adj)
        t = tree.apply(z, precision=prec, adjoint=adj)
        tol = 1e-12 if prec == 0 else 1e-5
        assert float(torch.linalg.norm(t - ref) / torch.linalg.norm(ref)) <= tol, (kind, prec, adj)


@pytest.mark.parametrize("kind", ["fv2d_64", "rgg_3001"])
def test_exact_coarse_solve(kind):
    """Exact coarse solve (the paper's EGMG variant): ILUT with tau = 0 is the
    complete LU of A_c without pivoting, so the preconditioner must equal the
    two-grid operator with A_c^{-1} itself.  Reference built without the
    oracle's ILUT: the oracle's ILU(0) smoother applied by scipy triangular
    solves, and A_c^{-1} by numpy's pivoted dense solve."""
    _say(f"[case] exact coarse solve {kind}")
    p = CASES[kind]()
    S = Solver(p.rowptr, p.col, p.val, ilut_tau=0.0)
    O = oracle.Oracle(p.rowptr, p.col, p.val, ilut_tau=0.0)
    (lrp, lci, lv), (urp, uci, uv) = S.ilut()
    (olrp, olci, olv), (ourp, ouci, ouv) = O.ilut()
    assert np.array_equal(lv.cpu().numpy(), olv) and np.array_equal(uv.cpu().numpy(), ouv)
    n = p.n_rows
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(n, n))
    f = sp.csr_matrix((O.ilu0(), p.col, p.rowptr), shape=(n, n))
    L0 = sp.tril(f, -1, format="csr") + sp.identity(n, format="csr")
    U0 = sp.triu(f, 0, format="csr")
    agg = O.aggregates()
    P = sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, O.nc))
    crp, cci, cv = O.coarse()
    Ac = sp.csr_matrix((cv, cci, crp), shape=(O.nc, O.nc)).toarray()
    z = np.random.default_rng(11).uniform(-1, 1, n)
    t = sp.linalg.spsolve_triangular(U0, sp.linalg.spsolve_triangular(L0, z, lower=True), lower=False)
    ref = t + P @ np.linalg.solve(Ac, P.T @ (z - A @ t))
    q = S.apply(torch.as_tensor(z, device="cuda"), precision=0).cpu().numpy()
    _elementwise(O, A, z, q, ref, 1e-12, f"exact coarse {kind}")
    # and the solve converges to tol
    b = p.b[:, 0]
    x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=1e-8)
    assert res.status == G.OK
    assert np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b) < 1e-8


@pytest.mark.parametrize("kind", ["fv2d_64", "fv3d_20", "rgg_3001"])
def test_jacobi_coarse_solve(kind):
    """Coarse solve by k Jacobi sweeps on each ILUT factor (the parallel
    inexact variant): one application against the oracle's same mode, with
    k = 3 and with k = N_c (then exact, equal to the triangular solves), and a
    converged solve."""
    _say(f"[case] jacobi coarse {kind}")
    p = CASES[kind]()
    z = np.random.default_rng(12).uniform(-1, 1, p.n_rows)
    zt = torch.as_tensor(z, device="cuda")
    S0 = Solver(p.rowptr, p.col, p.val)
    nc = S0.info()["n_coarse"]
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    for k in (3, nc):
        S = Solver(p.rowptr, p.col, p.val, coarse_mode=1, coarse_sweeps=k)
        O = oracle.Oracle(p.rowptr, p.col, p.val, coarse_mode=1, coarse_sweeps=k)
        q = S.apply(zt, precision=0).cpu().numpy()
        ref = O.apply(z, 0)
        _elementwise(O, A, z, q, ref, 1e-13, f"jacobi {kind} k={k}")
    exact = S0.apply(zt, precision=0).cpu().numpy()
    _elementwise(O, A, z, q, exact, 1e-12, f"jacobi {kind} k=N_c vs exact")
    S = Solver(p.rowptr, p.col, p.val, coarse_mode=1, coarse_sweeps=3)
    b = p.b[:, 0]
    x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=1e-8, restart=600)
    assert res.status == G.OK and np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b) < 1e-8


def test_profile_class_selection():
    """Event timing of selected kernel classes only, of all classes, and a
    rejected negative mask."""
    _say("[case] profile classes")
    p = W.make("fv2d_64")
    S = Solver(p.rowptr, p.col, p.val)
    b = torch.as_tensor(p.b[:, 0], device="cuda")
    S.profile(True, classes=["ortho"])
    S.solve(b, tol=1e-8)
    pr = S.profile_read()
    assert pr["ortho"]["launches"] > 0 and pr["ortho"]["ms"] > 0
    assert all(v["launches"] == 0 for k, v in pr.items() if k != "ortho")
    S.profile(True)
    S.solve(b, tol=1e-8)
    pr = S.profile_read()
    assert all(pr[k]["launches"] > 0 for k in ("spmv", "sweep_fine", "sweep_coarse", "ortho"))
    assert G.load().gmg_profile_enable(S._h, -1) == G.ERR_INVALID_ARG
    S.profile(False)


@pytest.mark.parametrize("case,n", [("dcc1_2d", 128), ("dcc2_3d", 30), ("dc1_2d", 128), ("dc1_3d", 30)])
def test_paper_problems_exact_vs_inexact(case, n):
    """The paper's analytic problems (Section 3.1) with GMRES(30), cf = 4:
    exact (tau = 0) and inexact (tau = 1e-4) coarse solves, each converged and
    within one step of the oracle's count.  With convection (DCC1, DCC2) the
    two converge in nearly the same number of steps while the inexact factor
    is several times smaller, as the paper reports; for pure diffusion (DC1)
    the inexact solve needs more steps under this drop rule (recorded, not a
    pass condition beyond exact <= inexact)."""
    _say(f"[case] paper problem {case} n={n}")
    p = W.paper_problem(case, n)
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    b = p.b[:, 0]
    steps, nnz = {}, {}
    for tau in (0.0, 1e-4):
        S = Solver(p.rowptr, p.col, p.val, cf=4.0, ilut_tau=tau)
        x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=1e-8, restart=30, maxit=600)
        assert res.status == G.OK, (case, tau, res.info)
        assert np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b) < 1e-8
        O = oracle.Oracle(p.rowptr, p.col, p.val, cf=4.0, ilut_tau=tau)
        xo, info = O.solve(b, tol=1e-8, restart=30, maxit=600)
        assert abs(res.info["iters"] - info.steps) <= 1, (case, tau, res.info["iters"], info.steps)
        steps[tau] = res.info["iters"]
        inf = S.info()
        nnz[tau] = inf["nnz_lc"] + inf["nnz_uc"]
    _say(f"[case] {case}: steps exact {steps[0.0]} inexact {steps[1e-4]}, factor storage ratio "
         f"{nnz[0.0] / nnz[1e-4]:.2f}")
    assert nnz[0.0] >= 1.5 * nnz[1e-4]
    assert steps[0.0] <= steps[1e-4]
    if case.startswith("dcc"):
        assert steps[1e-4] - steps[0.0] <= 2


def test_paper_curve_dc3d_50():
    """Figure F:curveJUMP regenerated from the GPU path: DC3D (DC1 3D) on
    50^3 cells, GMRES(30), cf = 4, exact (tau = 0) and inexact (tau = 1e-4
    and 1e-6) coarse solves.  Each GPU residual history (the FGMRES estimate after every
    step, read through gmg_get_history) follows the oracle's step by step
    (relative 1e-6 while above 1e-11) and ends within one step of it."""
    _say("[case] paper curve dc1_3d n=50")
    p = W.paper_problem("dc1_3d", 50)
    b = p.b[:, 0]
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    for tau in (0.0, 1e-4, 1e-6):
        S = Solver(p.rowptr, p.col, p.val, cf=4.0, ilut_tau=tau)
        x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=1e-8, restart=30, maxit=600)
        assert res.status == G.OK and np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b) < 1e-8
        h = S.history()
        assert len(h) == res.info["iters"]
        O = oracle.Oracle(p.rowptr, p.col, p.val, cf=4.0, ilut_tau=tau)
        _, info, ex = O.solve(b, tol=1e-8, restart=30, maxit=600, history=True)
        ho = ex["history"]
        assert abs(len(h) - len(ho)) <= 1, (tau, len(h), len(ho))
        m = min(len(h), len(ho))
        rel = np.abs(h[:m] - ho[:m]) / ho[:m]
        keep = ho[:m] > 1e-11
        _say(f"  tau={tau}: {len(h)} steps (oracle {len(ho)}), max relative curve difference {rel[keep].max():.2e}")
        assert np.all(rel[keep] <= 1e-6), (tau, rel.max())


def test_condition_estimates():
    """The cheap estimates of Section 3: max/min of |diag A_c| and of
    |diag L~U~|, against scipy on the oracle's A_c and ILUT factors; larger
    coefficient jumps give larger estimates (the paper's qualitative use)."""
    _say("[case] condition estimates")
    ests = []
    for lo, hi in ((-1, 1), (-4, 4)):
        p = W.fv_problem(48, 2, 8, lo, hi, W.velocity_const((1.0, 0.5)), 3)
        S = Solver(p.rowptr, p.col, p.val)
        O = oracle.Oracle(p.rowptr, p.col, p.val)
        ec, el = S.cond_estimate()
        crp, cci, cv = O.coarse()
        Ac = sp.csr_matrix((cv, cci, crp), shape=(O.nc, O.nc))
        (lrp, lci, lv), (urp, uci, uv) = O.ilut()
        L = sp.csr_matrix((lv, lci, lrp), shape=(O.nc, O.nc)) + sp.identity(O.nc, format="csr")
        U = sp.csr_matrix((uv, uci, urp), shape=(O.nc, O.nc))
        d = np.abs(Ac.diagonal())
        dlu = np.abs((L @ U).diagonal())
        assert np.isclose(ec, d.max() / d.min(), rtol=1e-12, atol=0)
        assert np.isclose(el, dlu.max() / dlu.min(), rtol=1e-10, atol=0)
        ests.append((ec, el))
    assert ests[1][0] > 100 * ests[0][0] and ests[1][1] > 100 * ests[0][1]


ND_CASES = {
    "fv2d_64": lambda: W.make("fv2d_64"),
    "fv3d_20": lambda: W.scaled("fv3d", 20),
    "rgg_3001": lambda: W.scaled("rgg", 3001),
}


@pytest.mark.parametrize("fo", [1, 2])
@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("name", list(ND_CASES))
def test_fine_nd_smoother(name, kernel, fo):
    """GMG-ND (Section 3.1 variants, fo = 1) and the multicolour smoother
    (fo = 2): the smoother's numbering and its ILU(0) factors bit-exact vs the
    oracle; one application in FP64 within 1e-13 of the magnitudes flowing into each entry, in FP32 within the FP32 bar;
    a converged solve within one step of the oracle's; the adjoint application
    entry by entry (its FP32 form refused).
    kernel 0: tree solves over the dissection tree (fo = 1) or the automatic
    level sweeps (fo = 2); 1: whole-device level sweeps."""
    _say(f"[case] fine_order={fo} {name} sweep_kernel={kernel}")
    p = ND_CASES[name]()
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    O = oracle.Oracle(p.rowptr, p.col, p.val, fine_order=fo)
    S = Solver(p.rowptr, p.col, p.val, fine_order=fo, sweep_kernel=kernel)
    perm, _ = O.fine()
    assert np.array_equal(S.fine_perm().cpu().numpy(), perm)
    assert np.array_equal(S.ilu0().cpu().numpy().view(np.uint64), O.ilu0().view(np.uint64))
    rng = np.random.default_rng(4)
    for _ in range(2):
        z = rng.uniform(-1, 1, p.n_rows)
        q = S.apply(torch.as_tensor(z, device="cuda"), precision=0).cpu().numpy()
        ref = O.apply(z, 0)
        _elementwise(O, A, z, q, ref, 1e-13, f"fine_order={fo} {name} fp64")
    q32 = S.apply(torch.as_tensor(z, device="cuda"), precision=1).cpu().numpy()
    ref32 = O.apply(z, 1)
    e32 = np.linalg.norm(q32 - ref32) / np.linalg.norm(ref32)
    e64 = np.linalg.norm(ref32 - ref) / np.linalg.norm(ref)
    assert e32 <= max(1e-4, 10 * e64), (e32, e64)
    _elementwise(O, A, z, q32, ref32, 2e-5, f"fine_order={fo} {name} fp32")
    b = p.b[:, 0]
    x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=1e-8)
    xh = x.cpu().numpy()
    assert res.status == G.OK and np.linalg.norm(b - A @ xh) / np.linalg.norm(b) < 1e-8, res.info
    _, info = O.solve(b, tol=1e-8)
    assert abs(res.info["iters"] - info.steps) <= 1, (res.info["iters"], info.steps)
    qa = S.apply(torch.as_tensor(z, device="cuda"), precision=0, adjoint=True).cpu().numpy()
    _elementwise(O, A, z, qa, O.apply_adjoint(z), 1e-13, f"fine_order={fo} {name} adjoint", adjoint=True)
    with pytest.raises(GmgError):
        S.apply(torch.as_tensor(z, device="cuda"), precision=1, adjoint=True)
    if kernel == 0 and fo == 1:
        S0 = Solver(p.rowptr, p.col, p.val)
        assert np.array_equal(S0.fine_perm().cpu().numpy(), np.arange(p.n_rows))


def test_fine_nd_large_separator():
    """GMG-ND on 64^3 cells: the first separator has more rows than one tree
    node may hold, so the tree layout cuts it into a chain of row blocks;
    same bars."""
    _say("[case] fine_order=1 fv3d_64 (level sweeps)")
    p = W.scaled("fv3d", 64)
    O = oracle.Oracle(p.rowptr, p.col, p.val, fine_order=1)
    S = Solver(p.rowptr, p.col, p.val, fine_order=1)
    perm, _ = O.fine()
    assert np.array_equal(S.fine_perm().cpu().numpy(), perm)
    assert np.array_equal(S.ilu0().cpu().numpy().view(np.uint64), O.ilu0().view(np.uint64))
    z = np.random.default_rng(6).uniform(-1, 1, p.n_rows)
    q = S.apply(torch.as_tensor(z, device="cuda"), precision=0).cpu().numpy()
    ref = O.apply(z, 0)
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    _elementwise(O, A, z, q, ref, 1e-13, "fine_order=1 fv3d_64")


@pytest.mark.parametrize("name", list(ND_CASES))
def test_spai_coarse_solve(name):
    """coarse_mode 2: the sparse approximate inverse of A_c bit-exact vs the
    oracle's (the same least-squares steps in the same order on the host);
    one application in FP64 within 1e-13 (entry by entry) and in FP32 within the FP32 bar; an
    unrestarted solve converged within one step of the oracle's."""
    _say(f"[case] coarse_mode=2 {name}")
    p = ND_CASES[name]()
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    O = oracle.Oracle(p.rowptr, p.col, p.val, coarse_mode=2)
    S = Solver(p.rowptr, p.col, p.val, coarse_mode=2)
    rp, ci, v = (t.cpu().numpy() for t in S.spai())
    orp, oci, ov = O.spai()
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
    assert np.array_equal(v.view(np.uint64), ov.view(np.uint64))
    z = np.random.default_rng(8).uniform(-1, 1, p.n_rows)
    q = S.apply(torch.as_tensor(z, device="cuda"), precision=0).cpu().numpy()
    ref = O.apply(z, 0)
    M = sp.csr_matrix((ov, oci, orp), shape=(O.nc, O.nc))
    _elementwise(O, A, z, q, ref, 1e-13, f"spai {name}", coarse=("spai", M))
    q32 = S.apply(torch.as_tensor(z, device="cuda"), precision=1).cpu().numpy()
    ref32 = O.apply(z, 1)
    e32 = np.linalg.norm(q32 - ref32) / np.linalg.norm(ref32)
    e64 = np.linalg.norm(ref32 - ref) / np.linalg.norm(ref)
    assert e32 <= max(1e-4, 10 * e64), (e32, e64)
    b = p.b[:, 0]
    x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=1e-8, restart=600, maxit=600)
    assert res.status == G.OK, res.info
    assert np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b) < 1e-8
    _, info = O.solve(b, tol=1e-8, restart=600, maxit=600)
    assert abs(res.info["iters"] - info.steps) <= 1, (res.info["iters"], info.steps)
    assert S.info()["nnz_lc"] == 0
    with pytest.raises(GmgError):
        S.cond_estimate()



DENSE_CASES = dict(ND_CASES, fv2d_8=lambda: W.scaled("fv2d", 8))


@pytest.mark.parametrize("name", list(DENSE_CASES))
def test_dense_coarse_inverse(name):
    """coarse_mode 3, the EGMG variant's exact coarse solve by a dense inverse
    (N_c from 11, one padded tile, to 1223, twenty tiles with a ragged tail):
    A_c^{-1} against numpy's pivoted inverse of the oracle's A_c (relative
    Frobenius error 1e-11: the same blocked no-pivot elimination run in
    numpy stays within 1.1e-13 of it on these cases, condition numbers up to
    2.6e8) and A_c X = I within 1e-9; one FP64 application against the
    oracle's exact (tau = 0) two-grid operator within 1e-10, the FP32 form
    within the FP32 bar; an unrestarted solve within one step of the oracle's
    exact-coarse solve."""
    _say(f"[case] coarse_mode=3 {name}")
    p = DENSE_CASES[name]()
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    O = oracle.Oracle(p.rowptr, p.col, p.val, ilut_tau=0.0)
    S = Solver(p.rowptr, p.col, p.val, coarse_mode=3)
    assert S.info()["n_coarse"] == O.nc and S.info()["nnz_lc"] == 0
    crp, cci, cv = O.coarse()
    Ac = sp.csr_matrix((cv, cci, crp), shape=(O.nc, O.nc)).toarray()
    X = S.coarse_inverse().cpu().numpy()
    R = np.linalg.inv(Ac)
    rel = np.linalg.norm(X - R) / np.linalg.norm(R)
    assert rel <= 1e-11, (name, rel)
    assert np.abs(Ac @ X - np.eye(O.nc)).max() <= 1e-9
    z = np.random.default_rng(9).uniform(-1, 1, p.n_rows)
    q = S.apply(torch.as_tensor(z, device="cuda"), precision=0).cpu().numpy()
    ref = O.apply(z, 0)
    _elementwise(O, A, z, q, ref, 1e-12, f"dense coarse {name}", coarse=("dense", R))
    q32 = S.apply(torch.as_tensor(z, device="cuda"), precision=1).cpu().numpy()
    ref32 = O.apply(z, 1)
    e32 = np.linalg.norm(q32 - ref) / np.linalg.norm(ref)
    e64 = np.linalg.norm(ref32 - ref) / np.linalg.norm(ref)
    assert e32 <= max(1e-4, 10 * e64), (e32, e64)
    b = p.b[:, 0]
    x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=1e-8, restart=600, maxit=600)
    assert res.status == G.OK, res.info
    assert np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b) < 1e-8
    _, info = O.solve(b, tol=1e-8, restart=600, maxit=600)
    assert abs(res.info["iters"] - info.steps) <= 1, (res.info["iters"], info.steps)
    with pytest.raises(GmgError):
        S.cond_estimate()


def _zero_leading_coarse_pivot(block_sum_zero=True):
    """8 unknowns in two strongly coupled chains of four, weakly coupled to
    each other: matching makes the chains the two aggregates, and the first
    chain's entries sum to zero, so A_c = [[0, -0.1], [-0.1, 4]] is invertible
    but has a zero leading pivot without pivoting; ILU(0) of A itself has
    nonzero pivots (3, 1.67, 2.35, -1.2, ...)."""
    A = np.zeros((8, 8))
    for o, d in ((0, (3.0, 3.0, 2.5, 0.5 if block_sum_zero else 1.5)), (4, (3.5, 3.0, 3.0, 3.5))):
        A[o, o + 1] = A[o + 1, o] = -2.0
        A[o + 1, o + 2] = A[o + 2, o + 1] = -0.5
        A[o + 2, o + 3] = A[o + 3, o + 2] = -2.0
        for k in range(4):
            A[o + k, o + k] = d[k]
    A[3, 4] = A[4, 3] = -0.1
    M = sp.csr_matrix(A)
    M.sort_indices()
    return M


def test_coarse_zero_pivot_reported():
    """The no-pivot elimination of A_c meets a zero pivot: the dense inverse
    (coarse_mode 3) and the complete LU (ILUT tau = 0) both report
    GMG_ERR_ZERO_PIVOT at setup, as the oracle does; with a nonzero pivot the
    same structure sets up and applies."""
    _say("[case] coarse zero pivot")
    M = _zero_leading_coarse_pivot()
    for kw in (dict(coarse_mode=3), dict(ilut_tau=0.0)):
        with pytest.raises(GmgError) as ei:
            Solver(M.indptr, M.indices, M.data, coarse_order=0, **kw)
        assert ei.value.code == G.ERR_ZERO_PIVOT, kw
    with pytest.raises(oracle.OracleError) as eo:
        oracle.Oracle(M.indptr, M.indices, M.data, coarse_order=0, ilut_tau=0.0)
    assert eo.value.code == oracle.ERR_ZERO_PIVOT
    M2 = _zero_leading_coarse_pivot(False)
    S = Solver(M2.indptr, M2.indices, M2.data, coarse_order=0, coarse_mode=3)
    O = oracle.Oracle(M2.indptr, M2.indices, M2.data, coarse_order=0, ilut_tau=0.0)
    z = np.random.default_rng(3).uniform(-1, 1, 8)
    q = S.apply(torch.as_tensor(z, device="cuda"), precision=0).cpu().numpy()
    assert np.allclose(q, O.apply(z, 0), rtol=1e-12, atol=1e-14)


def test_dense_coarse_inverse_size_limit():
    """coarse_mode 3 refuses N_c above 8192 at setup (fv2d 256^2: N_c ~ 16k)."""
    _say("[case] coarse_mode=3 size limit")
    p = W.scaled("fv2d", 256)
    with pytest.raises(GmgError):
        Solver(p.rowptr, p.col, p.val, coarse_mode=3)

def test_tiny_and_degenerate():
    _say("[case] tiny")
    # 1x1, diagonal matrices, a 2x2 that needs no pivoting
    for A in (np.array([[3.0]]), np.diag([1.0, 2.0, 3.0, 4.0]),
              np.array([[4.0, -1.0], [-2.0, 5.0]])):
        S_ = sp.csr_matrix(A)
        S_.sort_indices()
        rp, ci, v = S_.indptr.astype(np.int32), S_.indices.astype(np.int32), S_.data
        # default, GMG-ND smoother, SPAI coarse solve
        for opts in ({}, dict(fine_order=1), dict(coarse_mode=2)):
            s = Solver(rp, ci, v, **opts)
            o = oracle.Oracle(rp, ci, v, **opts)
            assert np.array_equal(s.aggregates().cpu().numpy(), o.aggregates())
            b = np.arange(1, A.shape[0] + 1, dtype=float)
            x, res = s.solve(torch.as_tensor(b, device="cuda"), tol=1e-12)
            assert np.allclose(A @ x.cpu().numpy(), b, rtol=1e-11), opts
            q = s.apply(torch.as_tensor(b, device="cuda")).cpu().numpy()
            assert np.allclose(q, o.apply(b), rtol=1e-12, atol=1e-15), opts
    # zero right-hand side: x = 0 without iterations
    p = W.scaled("fv2d", 16)
    s = Solver(p.rowptr, p.col, p.val)
    x, res = s.solve(torch.zeros(p.n_rows, dtype=torch.float64, device="cuda"))
    assert res.info["iters"] == 0 and float(x.abs().max()) == 0.0


def test_error_paths():
    _say("[case] errors")
    p = W.scaled("fv2d", 16)
    # unsorted columns
    ci = p.col.copy()
    ci[1], ci[2] = ci[2], ci[1]
    with pytest.raises(GmgError) as e:
        Solver(p.rowptr, ci, p.val)
    assert e.value.code == G.ERR_INVALID_ARG
    # missing diagonal
    rp = np.array([0, 1, 2], dtype=np.int32)
    with pytest.raises(GmgError) as e:
        Solver(rp, np.array([1, 0], dtype=np.int32), np.array([1.0, 1.0]))
    assert e.value.code == G.ERR_INVALID_ARG
    # non-finite entry
    v = p.val.copy()
    v[5] = np.inf
    with pytest.raises(GmgError) as e:
        Solver(p.rowptr, p.col, v)
    assert e.value.code == G.ERR_NONFINITE
    # zero pivot in ILU(0)
    with pytest.raises(GmgError) as e:      # explicit zero diagonal entry
        Solver(np.array([0, 2, 4], dtype=np.int32), np.array([0, 1, 0, 1], dtype=np.int32),
               np.array([0.0, 1.0, 1.0, 1.0]), cf=1.0)
    assert e.value.code == G.ERR_ZERO_PIVOT
    # NaN right-hand side, maxit, bad restart
    s = Solver(p.rowptr, p.col, p.val)
    b = np.ones(p.n_rows)
    b[3] = np.nan
    with pytest.raises(GmgError) as e:
        s.solve(torch.as_tensor(b, device="cuda"))
    assert e.value.code == G.ERR_NONFINITE
    x, res = s.solve(torch.as_tensor(p.b[:, 0], device="cuda"), tol=1e-14, maxit=2)
    assert res.status == G.NOT_CONVERGED and res.info["iters"] == 2
    with pytest.raises(GmgError):
        s.solve(torch.as_tensor(p.b[:, 0], device="cuda"), restart=5000)
    # the handle still works after errors
    x, res = s.solve(torch.as_tensor(p.b[:, 0], device="cuda"), tol=1e-8)
    assert res.status == G.OK


ADJ_VARIANTS = {
    "jacobi": dict(coarse_mode=1, coarse_sweeps=3),
    "spai": dict(coarse_mode=2),
    "dense": dict(coarse_mode=3),
    "nd": dict(fine_order=1),
    "color": dict(fine_order=2),
}


@pytest.mark.parametrize("variant", list(ADJ_VARIANTS))
@pytest.mark.parametrize("name", ["fv2d_64", "rgg_3001"])
def test_adjoint_variants(name, variant):
    """The adjoint cycle of every coarse solve (Jacobi sweeps, sparse
    approximate inverse, dense inverse) and reordered smoother (dissection
    tree, colour classes) against the oracle's transpose of the same
    operator (the dense inverse against the exact, tau = 0, coarse solve):
    one application entry by entry, adjoint FGMRES iterates after 5 steps
    (one and three right-hand sides), and a converged adjoint solve."""
    _say(f"[case] adjoint {variant} {name}")
    p = CASES[name]()
    opts = ADJ_VARIANTS[variant]
    S = Solver(p.rowptr, p.col, p.val, **opts)
    O = oracle.Oracle(p.rowptr, p.col, p.val, **(dict(ilut_tau=0.0) if variant == "dense" else opts))
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    coarse, bar, ibar = None, 1e-13, 1e-10
    if variant == "spai":
        coarse = ("spai", _spai_csr(O))
    if variant == "dense":
        crp, cci, cv = O.coarse()
        coarse = ("dense", np.linalg.inv(sp.csr_matrix((cv, cci, crp), shape=(O.nc, O.nc)).toarray()))
        bar, ibar = 1e-12, 1e-9
    rng = np.random.default_rng(21)
    z = rng.uniform(-1, 1, p.n_rows)
    q = S.apply(torch.as_tensor(z, device="cuda"), precision=0, adjoint=True).cpu().numpy()
    _elementwise(O, A, z, q, O.apply_adjoint(z), bar, f"adjoint {variant} {name}", adjoint=True, coarse=coarse)
    g = rng.uniform(-1, 1, p.n_rows)
    l5, _ = S.solve_adjoint(torch.as_tensor(g, device="cuda"), tol=0.0, maxit=5)
    lo, info = O.solve(g, tol=0.0, maxit=5, adjoint=True)
    assert info.steps == 5
    d = np.linalg.norm(A.T @ (l5.cpu().numpy() - lo)) / np.linalg.norm(g)
    assert d <= ibar, (variant, name, d)
    Gm = rng.uniform(-1, 1, (p.n_rows, 3))
    Lb, res_b = S.solve_adjoint(torch.as_tensor(Gm, device="cuda"), tol=0.0, maxit=5, restart=30)
    Lbh = Lb.cpu().numpy()
    for c in range(3):
        lo, _ = O.solve(Gm[:, c], tol=0.0, maxit=5, restart=30, adjoint=True)
        d = np.linalg.norm(A.T @ (Lbh[:, c] - lo)) / np.linalg.norm(Gm[:, c])
        assert d <= ibar, (variant, name, c, d)
    lam, res = S.solve_adjoint(torch.as_tensor(g, device="cuda"), tol=1e-9, restart=600, maxit=600)
    if res.status == G.OK:
        assert np.linalg.norm(g - A.T @ lam.cpu().numpy()) / np.linalg.norm(g) < 1e-9
    else:
        # an inexact coarse solve that does not converge forward either
        _, fres = S.solve(torch.as_tensor(g, device="cuda"), tol=1e-9, restart=600, maxit=600)
        assert fres.status != G.OK, (variant, name, res.info)


def _spai_csr(O):
    rp, ci, v = O.spai()
    return sp.csr_matrix((v, ci, rp), shape=(O.nc, O.nc))

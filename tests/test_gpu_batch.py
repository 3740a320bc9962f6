"""Several right-hand sides per launch: the batched FGMRES(m <= 32) path
(fine wavefront sweeps and coarse tree solves over all columns in one launch,
a CSR product over column batches, the fused residual + restriction, one
Krylov recurrence per column of each launch), against the oracle column by
column.  Bars as for one right-hand side: iterates at equal step counts within
||A (x - x_oracle)|| / ||b|| <= 1e-10; converged solves at true relative
residual < tol within one step per column of the oracle's count."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_1105_3468_amd import Solver  # noqa: E402
from paper_1105_3468_amd import gmg as G  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# 2D and 3D grids take the batched wavefront sweeps, the others the per-column level
# sweeps; the coarse factors follow the dissection tree in every case
CASES = {
    "fv2d_64": lambda: W.make("fv2d_64"),
    "fv2d_37": lambda: W.fv_problem(37, 2, 1, -2, 2, W.velocity_const((1.0, 0.5)), 5),
    "fv2d_150": lambda: W.fv_problem(150, 2, 1, -2, 2, W.velocity_const((1.0, 0.5)), 6),
    "fv3d_20": lambda: W.scaled("fv3d", 20),
    "rgg_3001": lambda: W.scaled("rgg", 3001),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    name = request.param
    _say(f"[case] batch {name}")
    p = CASES[name]()
    O = oracle.Oracle(p.rowptr, p.col, p.val)
    S = Solver(p.rowptr, p.col, p.val)
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    return name, p, O, S, A


def _rhs(n, k, seed):
    B = np.random.default_rng(seed).uniform(-1, 1, (n, k))
    B[:, 3] = B[:, 1]            # a repeated column
    return B


@pytest.mark.parametrize("steps", [7, 40])
def test_batched_iterates_match_oracle(case, steps):
    """5 columns, FGMRES(30), exactly `steps` steps each (40: one restart):
    every column against the oracle's iterate; a repeated column gives the
    same bits (the columns do not interact)."""
    name, p, O, S, A = case
    B = _rhs(p.n_rows, 5, 11)
    X, res = S.solve(torch.as_tensor(B, device="cuda"), tol=0.0, maxit=steps, restart=30)
    Xh = X.cpu().numpy()
    assert res.info["iters"] == 5 * steps, res.info
    for c in range(5):
        xo, info = O.solve(B[:, c], tol=0.0, maxit=steps, restart=30)
        d = np.linalg.norm(A @ (Xh[:, c] - xo)) / np.linalg.norm(B[:, c])
        assert info.steps == steps and d <= 1e-10, (name, c, d)
    assert np.array_equal(Xh[:, 1], Xh[:, 3])


def test_batched_converged_matches_oracle(case):
    name, p, O, S, A = case
    B = _rhs(p.n_rows, 6, 12)
    X, res = S.solve(torch.as_tensor(B, device="cuda"), tol=1e-8, restart=30)
    Xh = X.cpu().numpy()
    assert res.status == G.OK and res.info["converged"] == 6, res.info
    steps = 0
    for c in range(6):
        rel = np.linalg.norm(B[:, c] - A @ Xh[:, c]) / np.linalg.norm(B[:, c])
        assert rel < 1e-8, (name, c, rel)
        xo, info = O.solve(B[:, c], tol=1e-8, restart=30)
        steps += info.steps
        assert np.linalg.norm(A @ (Xh[:, c] - xo)) / np.linalg.norm(B[:, c]) <= 2e-8
    assert abs(res.info["iters"] - steps) <= 6, (res.info["iters"], steps)
    # the per-column residual histories, one column after another
    assert len(S.history()) == res.info["iters"]


def test_batched_adjoint_iterates(case):
    name, p, O, S, A = case
    B = _rhs(p.n_rows, 4, 13)
    L, res = S.solve_adjoint(torch.as_tensor(B, device="cuda"), tol=0.0, maxit=9, restart=30)
    Lh = L.cpu().numpy()
    for c in range(4):
        lo, info = O.solve(B[:, c], tol=0.0, maxit=9, restart=30, adjoint=True)
        d = np.linalg.norm(A.T @ (Lh[:, c] - lo)) / np.linalg.norm(B[:, c])
        assert d <= 1e-10, (name, c, d)
    L2, res2 = S.solve_adjoint(torch.as_tensor(B, device="cuda"), tol=1e-9, restart=30)
    L2h = L2.cpu().numpy()
    assert res2.status == G.OK
    for c in range(4):
        assert np.linalg.norm(B[:, c] - A.T @ L2h[:, c]) / np.linalg.norm(B[:, c]) < 1e-9


def test_batched_fp32_cycle(case):
    """The FP32 V-cycle for a batch: converged, and within 2 tol of the
    oracle's FP64 solution per column."""
    name, p, O, S, A = case
    B = _rhs(p.n_rows, 4, 14)
    X, res = S.solve(torch.as_tensor(B, device="cuda"), tol=1e-8, restart=30, precond_fp32=1)
    Xh = X.cpu().numpy()
    assert res.status == G.OK
    for c in range(4):
        assert np.linalg.norm(B[:, c] - A @ Xh[:, c]) / np.linalg.norm(B[:, c]) < 1e-8
        xo, _ = O.solve(B[:, c], tol=1e-8, restart=30)
        assert np.linalg.norm(A @ (Xh[:, c] - xo)) / np.linalg.norm(B[:, c]) <= 2e-8


def test_batched_two_batches_zero_column_and_x0():
    """20 columns (a batch of 16, then 4), one of them zero; then a restart
    from the solution with x0 (no step needed)."""
    _say("[case] batch fv2d_64 x20")
    p = W.make("fv2d_64")
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    S = Solver(p.rowptr, p.col, p.val)
    B = np.random.default_rng(15).uniform(-1, 1, (p.n_rows, 20))
    B[:, 17] = 0.0
    X, res = S.solve(torch.as_tensor(B, device="cuda"), tol=1e-9, restart=30)
    Xh = X.cpu().numpy()
    assert res.status == G.OK and res.info["converged"] == 20
    assert np.array_equal(Xh[:, 17], np.zeros(p.n_rows))
    for c in range(20):
        if c != 17:
            assert np.linalg.norm(B[:, c] - A @ Xh[:, c]) / np.linalg.norm(B[:, c]) < 1e-9
    X2, res2 = S.solve(torch.as_tensor(B, device="cuda"), tol=1e-9, restart=30, x0=X)
    assert res2.status == G.OK and res2.info["iters"] == 0
    assert np.array_equal(X2.cpu().numpy(), Xh)

"""Wavefront sweeps of fine factors with 3D-grid structure: a wave walks a
tile of 8 x 8 grid lines, neighbouring tiles exchange their faces through
memory.  The sweeps must perform the same operations in the same order as
the level sweeps (sweep_kernel 1): bitwise-equal preconditioner applications
in FP64 and FP32, forward and adjoint, on grids whose sides are not multiples
of the tile (padded lines), with a single plane of tiles in y or z, and with
two planes in z.  The solve against the oracle then follows from the parity
tests of the level sweeps."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_1105_3468_amd import Solver  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


grid7 = W.grid7_matrix


SHAPES = {
    "13x9x21": lambda: grid7(13, 9, 21, 1),
    "40x8x2": lambda: grid7(40, 8, 2, 2),
    "7x17x8": lambda: grid7(7, 17, 8, 3),
    "fv3d_20": lambda: (lambda p: (p.rowptr, p.col, p.val))(W.scaled("fv3d", 20)),
}


def _solver_3d(rp, ci, va, capfd, **opts):
    """A solver whose fine sweeps took the 3D wavefront layout (its setup log
    names the layout)."""
    os.environ["GMG_LOG"] = "1000000"
    try:
        S = Solver(rp, ci, va, **opts)
    finally:
        del os.environ["GMG_LOG"]
    err = capfd.readouterr().err
    assert "wavefront layout (3D)" in err, err[-2000:]
    return S


@pytest.mark.parametrize("shape", list(SHAPES))
def test_wave3_bitwise_equal_to_level_sweeps(shape, capfd):
    _say(f"[case] 3D wavefront {shape}")
    rp, ci, va = SHAPES[shape]()
    n = len(rp) - 1
    S3 = _solver_3d(rp, ci, va, capfd, sweep_kernel=3)
    S1 = Solver(rp, ci, va, sweep_kernel=1)
    rng = np.random.default_rng(5)
    for prec, adj in ((0, False), (1, False), (0, True)):
        for k in range(2):  # two applications in a row: the layout buffers are reset between them
            z = torch.as_tensor(rng.uniform(-1, 1, n), device="cuda")
            a = S3.apply(z, precision=prec, adjoint=adj)
            b = S1.apply(z, precision=prec, adjoint=adj)
            assert torch.equal(a, b), (shape, prec, adj, k, float((a - b).abs().max()))


@pytest.mark.parametrize("shape", ["13x9x21", "fv3d_20"])
def test_wave3_solve_matches_oracle(shape, capfd):
    """Default options (3D wavefront fine sweeps, tree-solved coarse factors):
    iterates after 8 steps within ||A (x - x_oracle)|| / ||b|| <= 1e-10, and
    a converged solve at the requested tolerance."""
    import scipy.sparse as sp
    _say(f"[case] 3D wavefront solve {shape}")
    rp, ci, va = SHAPES[shape]()
    n = len(rp) - 1
    S = _solver_3d(rp, ci, va, capfd)
    O = oracle.Oracle(rp, ci, va)
    A = sp.csr_matrix((va, ci, rp), shape=(n, n))
    b = np.random.default_rng(8).uniform(-1, 1, n)
    x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=0.0, maxit=8, restart=30)
    xo, info = O.solve(b, tol=0.0, maxit=8, restart=30)
    d = np.linalg.norm(A @ (x.cpu().numpy() - xo)) / np.linalg.norm(b)
    assert info.steps == 8 and d <= 1e-10, (shape, d)
    x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=1e-8, maxit=300, restart=300)
    r = np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b)
    assert r < 1e-8, (shape, r)

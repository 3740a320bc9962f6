"""Device memory reuse: freed library blocks are cached per device and handed
out again, at once to later work on the stream they were freed on, to other
streams only once their stream has been synchronised.  Solves on reused
memory, on other streams, with solvers alive side by side and after a stream
change must all give the bits of the first solve."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1105_3468_amd import Solver  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def problem():
    p = W.make("fv2d_64")
    rp, ci, va = (torch.as_tensor(a, device="cuda") for a in (p.rowptr, p.col, p.val))
    B = torch.as_tensor(np.random.default_rng(3).uniform(-1, 1, (p.n_rows, 3)), device="cuda")
    return p, rp, ci, va, B


def _solve(S, b, stream):
    with torch.cuda.stream(stream):
        x, res = S.solve(b, tol=1e-10, restart=30)
        xa, _ = S.solve_adjoint(b, tol=1e-10, restart=30)
    stream.synchronize()
    return x.clone(), xa.clone(), res.info["iters"]


def test_reuse_across_solvers_and_streams(problem):
    _say("[case] pool: reuse across solvers and streams")
    p, rp, ci, va, B = problem
    b = B[:, 0].contiguous()
    main = torch.cuda.current_stream()
    S0 = Solver(rp, ci, va)
    ref = _solve(S0, b, main)
    S0.close()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for st in (s1, s2, main, s1):
        with torch.cuda.stream(st):
            S = Solver(rp, ci, va, stream=st)
        got = _solve(S, b, st)
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]) and got[2] == ref[2]
        S.close()
    # two solvers alive on different streams, one destroyed and replaced
    # while the other keeps working
    with torch.cuda.stream(s1):
        Sa = Solver(rp, ci, va, stream=s1)
    with torch.cuda.stream(s2):
        Sb = Solver(rp, ci, va, stream=s2)
    ga = _solve(Sa, b, s1)
    gb = _solve(Sb, b, s2)
    Sa.close()
    with torch.cuda.stream(s1):
        Sc = Solver(rp, ci, va, stream=s1)
    gb2 = _solve(Sb, b, s2)
    gc = _solve(Sc, b, s1)
    for g in (ga, gb, gb2, gc):
        assert torch.equal(g[0], ref[0]) and torch.equal(g[1], ref[1])
    Sb.close()
    Sc.close()


def test_stream_change_and_batches(problem):
    """A solver moved to another stream (gmg_set_stream) and batched solves
    that allocate their column buffers on reused memory."""
    _say("[case] pool: stream change and batches")
    p, rp, ci, va, B = problem
    main = torch.cuda.current_stream()
    S0 = Solver(rp, ci, va)
    X0, _ = S0.solve(B, tol=1e-10, restart=30)
    X0 = X0.clone()
    S0.close()
    s1 = torch.cuda.Stream()
    S = Solver(rp, ci, va)
    S.set_stream(s1)
    with torch.cuda.stream(s1):
        X1, _ = S.solve(B, tol=1e-10, restart=30)
    s1.synchronize()
    assert torch.equal(X1, X0)
    S.set_stream(main)
    X2, _ = S.solve(B, tol=1e-10, restart=30)
    torch.cuda.synchronize()
    assert torch.equal(X2, X0)
    S.close()

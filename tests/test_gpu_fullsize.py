"""Parity at the full sizes of the benchmark workloads, with the options the
benchmark times (bench.SOLVE_OPTS: cf = 4, ILUT tau = 1e-6, no restart).

The oracle finishes the whole setup at these sizes in seconds, so the setup
outputs are compared in full: aggregates, A_c, ILU(0) and ILUT bit-exact.  A
full FGMRES run of the oracle on 1024^2 would take about a minute, so the solve
is checked by sampled outputs and properties: one preconditioner application
(FP64 within 1e-13 of the magnitudes that flow into each entry, entry by
entry, as in the small cases), the iterate after five
FGMRES steps (within 1e-10 in ||A dx|| / ||b||), and the converged GPU solve's
true residual.  rgg_500k converges in a few steps, so its converged solution is
compared with the oracle's as well, on each of its four seeds.  fv3d_128 runs the V-cycle in FP32 inside
FP64 FGMRES; its error against the FP64 oracle is bounded by FP32 rounding.
"""
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

import bench  # noqa: E402  (the timed options)
import oracle  # noqa: E402
from paper_1105_3468_amd import Solver  # noqa: E402
from paper_1105_3468_amd import gmg as G  # noqa: E402
from tests import _errbound as EB  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _elementwise(O, A, z, q, ref, tol, what):
    """|q - ref| <= tol * scale entry by entry (tests/_errbound.py)."""
    scale = EB.apply_scale(O, A, z)
    r = EB.check_elementwise(q, ref, scale, tol, what)
    _say(f"  {what}: max |diff|/scale = {r:.2e} (bar {tol:g})")


# workload -> (setup options, FGMRES restart, tolerance, maxit)
SETUPS = {
    "fv2d_1024": (dict(cf=bench.SOLVE_OPTS["cf"], ilut_tau=bench.SOLVE_OPTS["ilut_tau"]),
                  bench.SOLVE_OPTS["restart"], bench.TOL, bench.SOLVE_OPTS["maxit"]),
    "rgg_500k": (dict(cf=4.0, ilut_tau=1e-4), 30, 1e-8, 600),
    # the 3D problem needs a tighter coarse factor to converge without restart
    "fv3d_128": (dict(cf=4.0, ilut_tau=1e-5), 600, 1e-8, 600),
}
# the random geometric graph is specified on four seeds
CASES = ["fv2d_1024", "rgg_500k:0", "rgg_500k:1", "rgg_500k:2", "rgg_500k:3", "fv3d_128"]


@pytest.fixture(scope="module", params=CASES)
def big(request):
    name, _, seed = request.param.partition(":")
    seed = int(seed or 0)
    opts, restart, tol, maxit = SETUPS[name]
    _say(f"[fullsize] {name} seed {seed}: generating")
    p = W.make(name, seed=seed)
    _say(f"[fullsize] {name}: oracle setup")
    O = oracle.Oracle(p.rowptr, p.col, p.val, **opts)
    _say(f"[fullsize] {name}: GPU setup")
    S = Solver(p.rowptr, p.col, p.val, **opts)
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    return name, p, O, S, A, restart, tol, maxit


def test_setup_bit_exact(big):
    name, p, O, S, A, *_ = big
    _say(f"[fullsize] {name}: setup outputs")
    assert np.array_equal(S.aggregates().cpu().numpy(), O.aggregates())
    rp, ci, v = (t.cpu().numpy() for t in S.coarse())
    orp, oci, ov = O.coarse()
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
    assert np.array_equal(v.view(np.uint64), ov.view(np.uint64))
    assert np.array_equal(S.ilu0().cpu().numpy().view(np.uint64), O.ilu0().view(np.uint64))
    (lrp, lci, lv), (urp, uci, uv) = S.ilut()
    (olrp, olci, olv), (ourp, ouci, ouv) = O.ilut()
    assert np.array_equal(lrp.cpu().numpy(), olrp) and np.array_equal(lci.cpu().numpy(), olci)
    assert np.array_equal(urp.cpu().numpy(), ourp) and np.array_equal(uci.cpu().numpy(), ouci)
    assert np.array_equal(lv.cpu().numpy().view(np.uint64), olv.view(np.uint64))
    assert np.array_equal(uv.cpu().numpy().view(np.uint64), ouv.view(np.uint64))


def test_preconditioner_apply(big):
    name, p, O, S, A, *_ = big
    _say(f"[fullsize] {name}: preconditioner")
    z = np.random.default_rng(2).uniform(-1, 1, p.n_rows)
    q = S.apply(torch.as_tensor(z, device="cuda"), precision=0).cpu().numpy()
    ref = O.apply(z, 0)
    _elementwise(O, A, z, q, ref, 1e-13, f"{name} fp64")
    # FP32 cycle: against the oracle's FP32 cycle to a few FP32 ulps (amplified
    # by the sweeps), and its error against the FP64 oracle within FP32 accuracy
    q32 = S.apply(torch.as_tensor(z, device="cuda"), precision=1).cpu().numpy()
    ref32 = O.apply(z, 1)
    e_or = np.linalg.norm(ref32 - ref) / np.linalg.norm(ref)
    e_gpu = np.linalg.norm(q32 - ref) / np.linalg.norm(ref)
    _say(f"[fullsize] {name}: FP32 cycle error vs FP64 oracle {e_gpu:.2e} (oracle's own FP32 cycle {e_or:.2e})")
    assert np.linalg.norm(q32 - ref32) / np.linalg.norm(ref32) <= max(1e-4, 10 * e_or)
    assert e_gpu <= max(1e-4, 10 * e_or)
    _elementwise(O, A, z, q32, ref32, 2e-5, f"{name} fp32")


def test_five_step_iterates(big):
    name, p, O, S, A, restart, tol, maxit = big
    _say(f"[fullsize] {name}: five FGMRES steps")
    b = p.b[:, 0]
    x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=0.0, maxit=5, restart=restart)
    xo, info = O.solve(b, tol=0.0, maxit=5, restart=restart)
    assert res.info["iters"] == info.steps == 5
    d = np.linalg.norm(A @ (x.cpu().numpy() - xo)) / np.linalg.norm(b)
    assert d <= 1e-10, (name, d)


@pytest.mark.parametrize("fp32", [0, 1])
def test_converged_solve(big, fp32):
    name, p, O, S, A, restart, tol, maxit = big
    _say(f"[fullsize] {name}: solve to {tol} (FP32 cycle {fp32})")
    b = p.b[:, 0]
    x, res = S.solve(torch.as_tensor(b, device="cuda"), tol=tol, maxit=maxit, restart=restart, precond_fp32=fp32)
    xh = x.cpu().numpy()
    rel = np.linalg.norm(b - A @ xh) / np.linalg.norm(b)
    assert res.status == G.OK and rel < tol, (name, fp32, rel, res.info)
    if name == "rgg_500k":
        xo, info = O.solve(b, tol=tol, restart=restart)
        if not fp32:
            assert abs(res.info["iters"] - info.steps) <= 1, (res.info["iters"], info.steps)
        assert np.linalg.norm(A @ (xh - xo)) / np.linalg.norm(b) <= 2 * tol


VARIANTS = {"gmg_nd": dict(fine_order=1), "multicolour": dict(fine_order=2), "spai": dict(coarse_mode=2),
            "jacobi": dict(coarse_mode=1, coarse_sweeps=3)}


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_variants_full_size(variant):
    """The paper's variants at the benchmark's size and options (fv2d_1024,
    cf = 4, ILUT 1e-6): GMG-ND and the multicolour smoother (numbering and
    ILU(0) factors bit-exact), the SPAI coarse solve (inverse bit-exact), the
    coarse solve by three Jacobi sweeps per ILUT factor (factors bit-exact),
    and one preconditioner application within 1e-13 (entry by entry) of the oracle's, as for
    the default method above."""
    kw = VARIANTS[variant]
    opts = dict(SETUPS["fv2d_1024"][0], **kw)
    _say(f"[fullsize] fv2d_1024 {variant}: generating")
    p = W.make("fv2d_1024")
    _say(f"[fullsize] fv2d_1024 {variant}: oracle setup")
    O = oracle.Oracle(p.rowptr, p.col, p.val, **opts)
    _say(f"[fullsize] fv2d_1024 {variant}: GPU setup")
    S = Solver(p.rowptr, p.col, p.val, **opts)
    _say(f"[fullsize] fv2d_1024 {variant}: setup outputs")
    assert np.array_equal(S.fine_perm().cpu().numpy(), O.fine()[0])
    assert np.array_equal(S.ilu0().cpu().numpy().view(np.uint64), O.ilu0().view(np.uint64))
    if kw.get("coarse_mode") == 1:
        (lrp, lci, lv), (urp, uci, uv) = [[t.cpu().numpy() for t in f] for f in S.ilut()]
        (olrp, olci, olv), (ourp, ouci, ouv) = O.ilut()
        assert np.array_equal(lci, olci) and np.array_equal(lv.view(np.uint64), olv.view(np.uint64))
        assert np.array_equal(uci, ouci) and np.array_equal(uv.view(np.uint64), ouv.view(np.uint64))
    if kw.get("coarse_mode") == 2:
        rp, ci, v = (t.cpu().numpy() for t in S.spai())
        orp, oci, ov = O.spai()
        assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
        assert np.array_equal(v.view(np.uint64), ov.view(np.uint64))
    _say(f"[fullsize] fv2d_1024 {variant}: preconditioner")
    z = np.random.default_rng(12).uniform(-1, 1, p.n_rows)
    q = S.apply(torch.as_tensor(z, device="cuda"), precision=0).cpu().numpy()
    ref = O.apply(z, 0)
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows))
    coarse = None
    if kw.get("coarse_mode") == 2:
        coarse = ("spai", sp.csr_matrix((ov, oci, orp), shape=(O.nc, O.nc)))
    scale = EB.apply_scale(O, A, z, coarse=coarse)
    r = EB.check_elementwise(q, ref, scale, 1e-13, variant)
    _say(f"  {variant}: max |diff|/scale = {r:.2e} (bar 1e-13)")

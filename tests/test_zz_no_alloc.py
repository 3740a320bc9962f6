"""gmg_fv_assemble_noalloc, the allocation-free form of gmg_fv_assemble
(static device scratch instead of library allocations), against
gmg_fv_assemble itself through the C ABI: row pointers and columns bit-exact
and values bitwise equal (same kernels, same order), on two calls in a row,
the second on a smaller grid, then a 3D grid; the size limit is refused."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1105_3468_amd import autograd as AG  # noqa: E402
from paper_1105_3468_amd import gmg as G  # noqa: E402


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _assemble_both(n, dim, vel, seed):
    rng = np.random.default_rng(seed)
    kap = torch.as_tensor(10.0 ** rng.uniform(-4, 4, n ** dim), device="cuda")
    vt = AG.face_velocities(n, dim, vel)
    ref = G.fv_assemble(n, dim, kap, vt)
    # outputs pre-filled with garbage: every entry must be written
    N, nnz = n ** dim, G.load().gmg_fv_nnz(n, dim)
    out = (torch.full((N + 1,), -7, dtype=torch.int32, device="cuda"),
           torch.full((nnz,), -7, dtype=torch.int32, device="cuda"),
           torch.full((nnz,), float("nan"), dtype=torch.float64, device="cuda"))
    got = G.fv_assemble(n, dim, kap, vt, out=out, noalloc=True)
    torch.cuda.synchronize()
    return ref, got


def _same(ref, got):
    rp, ci, va = (t.cpu().numpy() for t in ref)
    grp, gci, gva = (t.cpu().numpy() for t in got)
    assert np.array_equal(grp, rp) and np.array_equal(gci, ci)
    assert np.array_equal(gva.view(np.uint64), va.view(np.uint64))


def test_noalloc_assembly_matches_allocating_entry_point():
    # first call on the device (the scratch lookup), then a smaller input,
    # which must not see stale block sums of the larger one
    for n, dim, vel, seed in [(1000, 2, W.velocity_rotating(10.0), 1), (37, 2, W.velocity_const((1.0, 0.5)), 2),
                              (48, 3, W.velocity_const((1.0, 1.0, 1.0)), 3), (1, 2, None, 4)]:
        _say(f"[case] noalloc assemble n={n} dim={dim}")
        ref, got = _assemble_both(n, dim, vel, seed)
        _same(ref, got)


def test_noalloc_assembly_rejects_too_many_cells():
    _say("[case] noalloc size limit")
    lib = G.load()
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda")
    p = dummy.data_ptr()
    n = 323   # 323^3 = 33,698,267 cells > the limit
    assert n ** 3 > G.FV_NOALLOC_MAX_CELLS
    st = lib.gmg_fv_assemble_noalloc(n, 3, p, p, p, p, p, p, p, None)
    assert st == G.ERR_INVALID_ARG
    assert b"exceed" in lib.gmg_last_error()

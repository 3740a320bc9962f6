"""CPU-side checks of the HIP library: it loads and exports every entry point
declared in include/gmg.h, and the binding's struct layouts match the header."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gmg_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1105_3468_amd import build as B
    B.build(force=False)
    return ctypes.CDLL(B.OUT)


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_all_symbols():
    from paper_1105_3468_amd import gmg
    assert sorted(gmg.EXPORTED) == _declared()


def test_default_options_and_struct_layout(lib):
    from paper_1105_3468_amd import gmg
    o = gmg.default_options()
    assert o.cf == 4.0 and o.restart == 30 and o.maxit == 600 and o.ilut_tau == 1e-4
    assert o.match_qbits == 4 and o.max_passes == 8
    # same default hash seed as the oracle's reading
    import oracle
    assert o.hash_seed == oracle.default_options()["seed"]
    assert o.sweep_kernel == 0 and o.sweep_wg_chunks == 8 and o.fine_order == 0
    # C layout: 13 ints, one uint64, two doubles, 4 bytes of tail padding
    assert ctypes.sizeof(gmg.Options) == 80
    assert ctypes.sizeof(gmg.Info) == 4 * 9 + 4 + 8 * 6 + 8 * 4


def test_fv_nnz_formula(lib):
    from paper_1105_3468_amd import gmg
    import workloads as W
    L = gmg.load()
    for n, dim in [(5, 2), (64, 2), (4, 3), (9, 3)]:
        if dim == 2:
            p = W.fv_problem(n, 2, 1, 0, 0, None, 0)
        else:
            p = W.fv_problem(n, 3, 1, 0, 0, None, 0)
        assert L.gmg_fv_nnz(n, dim) == p.nnz


def test_no_gpu_raises_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_1105_3468_amd import Solver
    import workloads as W
    p = W.scaled("fv2d", 8)
    with pytest.raises(RuntimeError):
        Solver(p.rowptr, p.col, p.val)


def test_struct_layout_matches_header(tmp_path):
    """Every field of the binding's Options and Info sits at the offset the C
    header gives it (compiled with gcc against include/gmg.h)."""
    import shutil
    import subprocess
    from paper_1105_3468_amd import gmg
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "gmg.h"', "int main(void) {"]
    for cname, py in (("gmg_options", gmg.Options), ("gmg_info", gmg.Info)):
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", inc, str(src), "-o", str(exe)])
    got = [int(t) for t in subprocess.check_output([str(exe)]).split()]
    want = []
    for py in (gmg.Options, gmg.Info):
        want.append(ctypes.sizeof(py))
        want += [getattr(py, f).offset for f, _ in py._fields_]
    assert got == want


def test_noalloc_assembly_limit_checked_before_device_work(lib):
    """gmg_fv_assemble_noalloc refuses grids beyond its scratch before it
    touches a device (so this runs without a GPU); the header's limit and the
    binding's agree."""
    from paper_1105_3468_amd import gmg
    src = open(os.path.join(ROOT, "include", "gmg.h")).read()
    assert re.search(r"GMG_FV_NOALLOC_MAX_CELLS\s+%dLL" % gmg.FV_NOALLOC_MAX_CELLS, src)
    assert re.search(r"GMG_FV_NOALLOC_SCRATCH_INTS\s+%d\b" % gmg.FV_NOALLOC_SCRATCH_INTS, src)
    # one block sum per 1024 cells (and the total) must fit the scratch
    assert (gmg.FV_NOALLOC_MAX_CELLS + 1 + 1023) // 1024 + 1 <= gmg.FV_NOALLOC_SCRATCH_INTS
    L = gmg.load()
    fake = ctypes.c_void_p(8)   # never dereferenced: the size check comes first
    assert L.gmg_fv_assemble_noalloc(323, 3, fake, fake, fake, fake, fake, fake, fake, None) == gmg.ERR_INVALID_ARG
    assert b"exceed" in L.gmg_last_error()
    assert L.gmg_fv_assemble_noalloc(0, 2, fake, fake, fake, None, fake, fake, fake, None) == gmg.ERR_INVALID_ARG

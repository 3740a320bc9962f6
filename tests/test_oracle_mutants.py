"""The oracle's pins catch plausible mistakes: each case builds a copy of
``oracle/gmg_oracle.c`` with one deliberate error (on the CPU, in a temporary
directory), runs the pin that should see it against that copy, and requires
the pin to fail.  The unmodified oracle passes the same pins in
``test_oracle_pins.py``."""
from __future__ import annotations

import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "gmg_oracle.c")

# (name, [(original text, replacement)], pin that must fail)
MUTANTS = [
    ("ilut_divide_then_drop",
     [("            if (fabs(w[k]) < ti) { w[k] = 0.0; in[k] = 2; continue; }   /* dropped */\n"
       "            double wk = w[k] / U->v[U->rp[k]];\n",
       "            double wk = w[k] / U->v[U->rp[k]];\n"
       "            if (fabs(wk) < ti) { w[k] = 0.0; in[k] = 2; continue; }\n")],
     pins.check_ilut_hand_fixture),
    ("ilut_one_norm_threshold",
     [("nrm = nrm + M->v[p] * M->v[p];", "nrm = nrm + fabs(M->v[p]);"),
      ("double ti = tau * sqrt(nrm);", "double ti = tau * nrm;")],
     pins.check_ilut_hand_fixture),
    ("ilut_no_final_u_drop",
     [("if (!(fabs(w[j]) < ti)) { U->ci[nu] = j;", "if (1) { U->ci[nu] = j;")],
     pins.check_ilut_hand_fixture),
    ("jacobi_in_place_update",
     [("            tmp[i] = a;        ", "            yc[i] = a;         ")],
     pins.check_jacobi_closed_form),
    ("jacobi_zero_start",
     [("for (int i = 0; i < nc; ++i) yc[i] = rc[i];  ", "for (int i = 0; i < nc; ++i) yc[i] = (T)0;   ")],
     pins.check_jacobi_closed_form),
    ("adjoint_jacobi_untransposed",
     [("t2[U->ci[p]] = t2[U->ci[p]] - U->v[p] * t1[j];", "t2[j] = t2[j] - U->v[p] * t1[U->ci[p]];")],
     pins.check_adjoint_transpose),
    ("adjoint_spai_untransposed",
     [("e[M->ci[p]] = e[M->ci[p]] + M->v[p] * b[i];", "e[i] = e[i] + M->v[p] * b[M->ci[p]];")],
     pins.check_adjoint_spai),
]


def _build_mutant(tmp_path, name, edits):
    text = open(SRC).read()
    for old, new in edits:
        assert text.count(old) == 1, f"{name}: target text not found exactly once: {old!r}"
        text = text.replace(old, new)
    src = tmp_path / f"{name}.c"
    lib = tmp_path / f"lib{name}.so"
    src.write_text(text)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", str(lib), str(src), "-lm"])
    return str(lib)


@pytest.mark.parametrize("name,edits,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_mutant(tmp_path, oracle_mod, name, edits, pin):
    lib = oracle._load(_build_mutant(tmp_path, name, edits))
    saved = oracle._lib
    oracle._lib = lib
    try:
        with pytest.raises(AssertionError):
            pin(oracle_mod)
    finally:
        oracle._lib = saved

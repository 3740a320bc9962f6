"""CPU oracle of the two-grid matching-AMG FGMRES method -- TEST INFRASTRUCTURE.

A plain, slow, sequential FP64 implementation written from the paper (see the
header of ``gmg_oracle.c`` for the passage each part follows).  Only the tests,
the package smoke check and the benchmark's CPU-baseline leg use it; the HIP
library never imports, links or calls anything here, and this module imports
nothing from the library.

Parity of every function here is pinned by ``tests/test_oracle_*.py`` against
brute force, dense linear algebra and the paper's worked example, except the
edge-key tie-break (quantised weight + hash), which is a design reading with no
external reference ("parity unpinned"; only its strict total order is checked).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, ERR_INVALID, ERR_OOM, ERR_ZERO_PIVOT, ERR_BREAKDOWN, ERR_NONFINITE = 0, 1, -1, -3, -4, -5, -6


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Opts(C.Structure):
    _fields_ = [("cf", C.c_double), ("max_passes", C.c_int), ("qbits", C.c_int),
                ("seed", C.c_uint64), ("ilut_tau", C.c_double), ("coarse_mode", C.c_int),
                ("coarse_sweeps", C.c_int), ("coarse_order", C.c_int), ("fine_order", C.c_int)]


_lib = None


def _load(path: str):
    """Open an oracle library built from gmg_oracle.c and declare its entry
    points (also used by the tests that build deliberately broken copies of
    the oracle to show that its pins catch them)."""
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.or_setup.argtypes = [C.c_int, P, P, P, C.POINTER(_Opts), P, C.POINTER(P)]
    lib.or_setup.restype = C.c_int
    lib.or_destroy.argtypes = [P]
    lib.or_sizes.argtypes = [P, P]
    lib.or_get_agg.argtypes = [P, P]
    lib.or_get_members.argtypes = [P, P, P]
    lib.or_get_graph.argtypes = [P, P, P, P]
    lib.or_get_coarse.argtypes = [P, P, P, P]
    lib.or_get_ilut.argtypes = [P, P, P, P, P, P, P]
    lib.or_get_ilu0.argtypes = [P, P]
    lib.or_get_fine.argtypes = [P, P, P, P, P]
    lib.or_get_spai.argtypes = [P, P, P, P]
    lib.or_precond_apply.argtypes = [P, C.c_int, P, P]
    lib.or_precond_apply_twosolve.argtypes = [P, P, P]
    lib.or_precond_apply_adjoint.argtypes = [P, P, P]
    lib.or_fgmres.argtypes = [P, C.c_int, C.c_int, P, P, C.c_double, C.c_int, C.c_int,
                              C.c_int, P, P, P, C.c_int]
    lib.or_fgmres.restype = C.c_int
    lib.or_match_once.argtypes = [C.c_int, P, P, P, C.c_int, C.c_uint64, P, P]
    lib.or_match_once.restype = C.c_int
    lib.or_spmv.argtypes = [P, C.c_int, P, P]
    lib.or_default_opts.argtypes = [C.POINTER(_Opts)]
    return lib


def _L():
    global _lib
    if _lib is None:
        _lib = _load(build())
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def default_options() -> dict:
    o = _Opts()
    _L().or_default_opts(C.byref(o))
    return {f: getattr(o, f) for f, _ in _Opts._fields_}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: status {code}")
        self.code = code


@dataclass
class SolveInfo:
    status: int
    steps: int
    restarts: int
    relres: float
    relres_est: float


class Oracle:
    """Setup of the two-grid hierarchy on A (CSR, int32 indices, float64 values)."""

    def __init__(self, rowptr, col, val, agg=None, **opts):
        lib = _L()
        self._lib = lib
        o = _Opts()
        lib.or_default_opts(C.byref(o))
        for k, v in opts.items():
            setattr(o, k, v)
        self.opts = o
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.n = len(self.rowptr) - 1
        h = C.c_void_p()
        ag = None if agg is None else np.ascontiguousarray(agg, dtype=np.int32)
        st = lib.or_setup(self.n, _p(self.rowptr), _p(self.col), _p(self.val), C.byref(o),
                          None if ag is None else _p(ag), C.byref(h))
        if st != OK:
            raise OracleError(st, "oracle setup")
        self._h = h
        s = np.zeros(9, dtype=np.int64)
        lib.or_sizes(h, _p(s))
        (self.n, self.nc, self.nnz, self.nnz_c, self.nnz_lc, self.nnz_uc, self.passes,
         self.rounds, self.nnz_graph) = (int(t) for t in s)

    def __del__(self):
        if getattr(self, "_h", None) is not None and getattr(self, "_lib", None) is not None:
            self._lib.or_destroy(self._h)
            self._h = None

    # --- setup products ----------------------------------------------------
    def aggregates(self):
        a = np.empty(self.n, dtype=np.int32)
        self._lib.or_get_agg(self._h, _p(a))
        return a

    def members(self):
        aptr = np.empty(self.nc + 1, dtype=np.int32)
        amem = np.empty(self.n, dtype=np.int32)
        self._lib.or_get_members(self._h, _p(aptr), _p(amem))
        return aptr, amem

    def graph(self):
        rp = np.empty(self.n + 1, dtype=np.int32)
        ci = np.empty(self.nnz_graph, dtype=np.int32)
        w = np.empty(self.nnz_graph, dtype=np.float64)
        self._lib.or_get_graph(self._h, _p(rp), _p(ci), _p(w))
        return rp, ci, w

    def coarse(self):
        rp = np.empty(self.nc + 1, dtype=np.int32)
        ci = np.empty(self.nnz_c, dtype=np.int32)
        v = np.empty(self.nnz_c, dtype=np.float64)
        self._lib.or_get_coarse(self._h, _p(rp), _p(ci), _p(v))
        return rp, ci, v

    def spai(self):
        """(rowptr, col, val) of the sparse approximate inverse of A_c
        (coarse_mode = 2; the pattern of A_c)."""
        if self.opts.coarse_mode != 2:
            raise ValueError("spai needs coarse_mode = 2")
        rp = np.empty(self.nc + 1, dtype=np.int32)
        ci = np.empty(self.nnz_c, dtype=np.int32)
        v = np.empty(self.nnz_c, dtype=np.float64)
        self._lib.or_get_spai(self._h, _p(rp), _p(ci), _p(v))
        return rp, ci, v

    def fine(self):
        """The smoother's numbering perm (position -> fine unknown; identity
        unless fine_order is 1, nested dissection, or 2, colour classes) and its
        matrix F = Q A Q^T as (rowptr, col, val)."""
        perm = np.empty(self.n, dtype=np.int32)
        rp = np.empty(self.n + 1, dtype=np.int32)
        ci = np.empty(self.nnz, dtype=np.int32)
        v = np.empty(self.nnz, dtype=np.float64)
        self._lib.or_get_fine(self._h, _p(perm), _p(rp), _p(ci), _p(v))
        return perm, (rp, ci, v)

    def ilu0(self):
        """ILU(0) values on the pattern of the smoother's matrix F (A itself
        unless fine_order = 1; strict lower part = L0, rest = U0)."""
        v = np.empty(self.nnz, dtype=np.float64)
        self._lib.or_get_ilu0(self._h, _p(v))
        return v

    def ilut(self):
        """(L rowptr, col, val) strictly lower, (U rowptr, col, val) with the diagonal first."""
        lrp = np.empty(self.nc + 1, dtype=np.int32)
        lci = np.empty(self.nnz_lc, dtype=np.int32)
        lv = np.empty(self.nnz_lc, dtype=np.float64)
        urp = np.empty(self.nc + 1, dtype=np.int32)
        uci = np.empty(self.nnz_uc, dtype=np.int32)
        uv = np.empty(self.nnz_uc, dtype=np.float64)
        self._lib.or_get_ilut(self._h, _p(lrp), _p(lci), _p(lv), _p(urp), _p(uci), _p(uv))
        return (lrp, lci, lv), (urp, uci, uv)

    # --- solve-phase operations -------------------------------------------
    def apply(self, z, precision: int = 0):
        z = np.ascontiguousarray(z, dtype=np.float64)
        q = np.empty(self.n)
        self._lib.or_precond_apply(self._h, precision, _p(z), _p(q))
        return q

    def apply_twosolve(self, z):
        z = np.ascontiguousarray(z, dtype=np.float64)
        q = np.empty(self.n)
        self._lib.or_precond_apply_twosolve(self._h, _p(z), _p(q))
        return q

    def apply_adjoint(self, z):
        z = np.ascontiguousarray(z, dtype=np.float64)
        q = np.empty(self.n)
        self._lib.or_precond_apply_adjoint(self._h, _p(z), _p(q))
        return q

    def spmv(self, x, transposed=False):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.n)
        self._lib.or_spmv(self._h, int(transposed), _p(x), _p(y))
        return y

    def solve(self, b, tol=1e-8, maxit=600, restart=30, x0=None, adjoint=False, precision=0,
              zdump=False, history=False):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64)
        info = np.zeros(4)
        zd = np.zeros((restart, self.n)) if zdump else None
        hist = np.zeros(maxit) if history else None
        st = self._lib.or_fgmres(self._h, int(adjoint), int(precision), _p(b), _p(x), float(tol),
                            int(maxit), int(restart), int(x0 is not None), _p(info),
                            None if zd is None else _p(zd), None if hist is None else _p(hist),
                            0 if hist is None else len(hist))
        if st < 0:
            raise OracleError(st, "oracle solve")
        si = SolveInfo(st, int(info[0]), int(info[1]), float(info[2]), float(info[3]))
        extra = {}
        if zdump:
            extra["Z"] = zd
        if history:
            extra["history"] = hist[: si.steps]
        return (x, si, extra) if extra else (x, si)


def match_once(rowptr, col, w, qbits=4, seed=None):
    """One handshake matching pass on a symmetric weighted graph; returns (mate, rounds)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    nv = len(rowptr) - 1
    mate = np.empty(max(nv, 1), dtype=np.int32)
    rounds = C.c_int(0)
    if seed is None:
        seed = default_options()["seed"]
    st = _L().or_match_once(nv, _p(rowptr), _p(col), _p(w), int(qbits), C.c_uint64(seed),
                            _p(mate), C.cast(C.pointer(rounds), C.c_void_p))
    if st != OK:
        raise OracleError(st, "match")
    return mate[:nv], rounds.value

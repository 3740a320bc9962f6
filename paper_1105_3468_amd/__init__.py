"""MI355X-native two-grid matching-aggregation AMG with an inexact ILUT coarse
solve, as a preconditioner of flexible GMRES (one GPU, HIP kernels for gfx950).

The compute lives in ``libgmg.so`` (C ABI: ``include/gmg.h``); this package
only binds it (``gmg``) and wraps it for autograd (``autograd``).
"""
from .gmg import (GmgError, Solver, default_options, fv_assemble, fv_kappa_grad, load,
                  pattern_grad)

__all__ = ["Solver", "GmgError", "default_options", "load", "fv_assemble", "fv_kappa_grad",
           "pattern_grad"]

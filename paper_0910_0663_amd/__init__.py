"""MI355X-native Virtual Transmission Method (Wei and Yang, arXiv 0910.0663).

The solver is the C-ABI library ``libvtm.so`` (include/vtm.h) with hand-written
HIP kernels for gfx950; this package is its Python binding.
"""
from .binding import (  # noqa: F401
    Solver,
    SolveReport,
    VTMError,
    plan,
    line_admittance,
    split_vertex,
    vertex_admittance,
    vertex_sca,
    lib,
    LIB_PATH,
    EXPORTS,
)

__all__ = ["Solver", "SolveReport", "VTMError", "plan", "line_admittance", "split_vertex", "vertex_admittance", "vertex_sca", "lib", "LIB_PATH", "EXPORTS", "VTMSolve", "Circuit"]


def __getattr__(name):
    if name in ("VTMSolve", "Circuit"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)

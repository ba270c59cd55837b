"""CPU oracle for the Virtual Transmission Method (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never does, and this
package never touches the library.
"""
from .vtm import (  # noqa: F401
    Torn,
    Result,
    RefineResult,
    Sweeper,
    UntearableError,
    tear_at_vertices,
    tear_wires,
    cut_wires,
    expand_midpoints,
    line_matrix,
    vtm_solve,
    vtm_refine,
    sweep_operator,
    interface_schur,
    partial_schur,
    reflection,
    spectral_radius,
    relative_residual,
    eliminate_twins,
    vtm_solve_eliminated,
    interface_residual,
    direct_solve,
    direct_adjoint,
    branch_gradient,
    matrix_gradient,
    jacobi_matrix,
    gauss_seidel_matrix,
)

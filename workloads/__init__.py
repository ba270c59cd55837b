"""Seeded synthetic circuits for the VTM solver and its oracle.

This package only builds problem instances: resistor grids, their nodal-analysis
matrix ``A`` (eq. 1), current-source right-hand sides, node partitions and line
impedances.  It contains none of the iteration's arithmetic, so both the HIP
path and the CPU oracle may import it.
"""
from .grids import (  # noqa: F401
    Workload,
    CONFIGS,
    make,
    grid2d_edges,
    grid3d_edges,
    nodal_matrix,
    block_partition_2d,
    block_partition_3d,
    random_cut_widths,
    separator_strips,
    GROUND_S,
)

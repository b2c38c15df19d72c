"""MI355X-native short-range Lennard-Jones MD over a cell list.

The compute path is the HIP library ``libmdlj.so`` (C-ABI in include/md.h);
this package is its ctypes binding plus a small owner class. Importing it
loads the library and fails if it has not been built.
"""
from ._lib import (  # noqa: F401
    MDError,
    MDParams,
    SYMBOLS,
    lib,
    make_params,
    md_build_cells,
    md_cell_grid,
    md_cell_lists,
    md_check,
    md_energy_virial,
    md_forces,
    md_get_state,
    md_neighbors,
    md_step,
    md_step_every,
    md_step_list,
    md_tile_capacity,
    md_workspace_bytes,
)
from .system import LJSystem, occupancy_cell_min  # noqa: F401
from .adjoint import LJTrajectory, trajectory_gradients  # noqa: F401
from .batch import BatchedLJ  # noqa: F401
from .tune import grid_options, tile_options, tune_batch, tune_cell_min, tune_system  # noqa: F401

lib()

"""RGDBEK (randomized greedy double block extended Kaczmarz, arXiv
2509.19267) for AMD Instinct MI355X (gfx950).

The solver lives in the HIP library librgdbek.so (C-ABI in
include/rgdbek.h); this package only marshals arguments to it.
"""
from ._binding import RgdbekError, LIB_PATH, load  # noqa: F401
from .solver import (Solver, BatchSolver, MultiRhsSolver,  # noqa: F401
                     block_diagonal, select, select_threshold,
                     select_block_law, select_iid, select_noalloc, solve,
                     RGDBEKFunction)

__all__ = ["Solver", "BatchSolver", "MultiRhsSolver", "block_diagonal", "select",
           "select_threshold", "select_block_law", "select_iid",
           "select_noalloc", "solve", "RGDBEKFunction", "RgdbekError",
           "LIB_PATH", "load"]

"""MI355X-native PCG state solver with the M_EH+Rot two-level Schwarz
preconditioner (arXiv:2006.13387), behind the C ABI of include/msp.h.

The compute path is the HIP library libmsp.so built from csrc/ for gfx950;
this package only marshals arguments (see binding.py).
"""
from .binding import (EXPORTS, LIB_PATH, Batch, MspError, ProblemDesc,
                      Server, SolveInfo, Solver, load_library, make_desc,
                      vec_dot)

__all__ = ["EXPORTS", "LIB_PATH", "Batch", "MspError", "ProblemDesc",
           "Server", "SolveInfo", "Solver", "load_library", "make_desc",
           "vec_dot"]

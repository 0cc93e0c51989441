"""LS-AMG-DD solve phase for MI355X (gfx950): C-ABI library + thin binding.

``liblsamg.so`` (built in-tree by ``paper_2601_04112_amd.build``) holds the
host setup of the hierarchy and the HIP kernels of the solve; ``lsamg``
marshals arguments to it.
"""
from .lsamg import (Solver, LsamgError, load, make_params, FP64, MIXED, OP_A,
                    OP_RAS, OP_RAST, OP_VCYCLE)

__all__ = ["Solver", "LsamgError", "load", "make_params", "FP64", "MIXED",
           "OP_A", "OP_RAS", "OP_RAST", "OP_VCYCLE"]

"""Seeded synthetic inputs for least-squares systems ``A = G^T G``.

This package builds the *problems* the solver is run on: the sparse
factor ``G`` of a finite-difference diffusion operator (section 4.1 of the
paper, the rotated anisotropic Laplacian written as ``G = B^T grad+``; and
the ``D1 + B^T D2^{-1} B`` form of the introduction) and the random
right-hand sides.  It holds none of the solver's arithmetic: no
aggregation, splitting, eigenproblem or cycle.  Both the CPU oracle and
the HIP library consume what it returns.
"""
from .grids import (Problem, aniso2d, ls3d, rhs_uniform, config1, config2,
                    config3, CONFIG_RHS_SEED)

__all__ = ["Problem", "aniso2d", "ls3d", "rhs_uniform", "config1", "config2",
           "config3", "CONFIG_RHS_SEED"]

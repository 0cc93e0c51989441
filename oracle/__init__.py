"""Plain FP64 CPU oracle of least-squares AMG-DD (test infrastructure only).

This package is test infrastructure.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the library and its
Python binding never do.  It shares no code with the HIP path: the two meet
only in the seeded problem generators of the ``problems`` package.

Every function follows the paper's definitions step by step, in FP64, with
NumPy/SciPy primitives (sparse products, dense Cholesky, symmetric
generalized eigensolver) and no blocking, fusion or reordering beyond what the
definitions state.  Where the paper is silent or ambiguous the reading taken
is stated at the point of use.

Parity status: every function is pinned by a test in ``tests/test_oracle_*``
(closed forms, exact invariants, special cases that reduce to a direct
solve, brute force on tiny inputs), except the iteration counts /
convergence factors of the large configurations, which are parity unpinned
(the paper's printed factors are for a different aggregation).
"""
from .lsamg import (Params, Level, Hierarchy, setup, vcycle, pcg, ras, ras_t,
                    apply_A, dense_preconditioner, stats, AssembledVcycle,
                    additive_schwarz, acycle, block_pcg)

__all__ = ["Params", "Level", "Hierarchy", "setup", "vcycle", "pcg", "ras",
           "ras_t", "apply_A", "dense_preconditioner", "stats", "AssembledVcycle",
           "additive_schwarz", "acycle", "block_pcg"]

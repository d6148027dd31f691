"""CPU FP64 oracle for recycling BiCGSTAB -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import or run anything in this package.  The product path (the
HIP library and its Python binding) never routes through it and shares no
code with it: the only thing both sides consume is the seeded input module
``workloads``.

Contents (each function cites the passage of the paper it follows):

* ``krylov.bicgstab``   -- van der Vorst's BiCGSTAB (the non-recycling baseline).
* ``krylov.rbicgstab``  -- RBiCGSTAB, Section 4 (BiCGSTAB on the projected operator).
* ``krylov.rbicg``      -- RBiCG, Section 3 (BiCG on the projected pair), with the cycle store
                           of Lanczos vectors described in Section 6.2.
* ``recycle.make_blocks``     -- the recycle blocks of Section 3, eq. (CcheckChat).
* ``recycle.recycle_space``   -- recycle-space selection (our reading; the
                                 paper defers it to its reference on RBiCG):
                                 harmonic right / two-sided left Ritz vectors.
* ``sequence.run_sequence``   -- the Section 6.2 driver (RBiCG on a matrix
                                 change, RBiCGSTAB for the other right-hand sides).
* ``adjoint.adjoint_solve``   -- A^T lambda = c by RBiCGSTAB with the swapped
                                 recycle space; ``adjoint.gradients`` -- dL/db,
                                 dL/dsigma, dL/dK for A(sigma) = K + sigma M.

Parity status: every function here is pinned by a CPU test (dense LU, SciPy's
BiCGSTAB, invariants of Theorems 1-2, closed forms, finite differences of
dense solves); see tests/test_oracle*.py.
"""
from .krylov import (OK, MAXIT, BREAKDOWN_RHO, BREAKDOWN_ALPHA, BREAKDOWN_OMEGA,
                     NONFINITE, SolveInfo, bicgstab, rbicgstab, rbicg)
from .recycle import (Blocks, make_blocks, empty_blocks, two_sided_ritz, harmonic_ritz,
                      recycle_space)
from .sequence import run_sequence, SequenceResult
from .adjoint import adjoint_solve, gradients, transposed_blocks

__all__ = ["OK", "MAXIT", "BREAKDOWN_RHO", "BREAKDOWN_ALPHA", "BREAKDOWN_OMEGA",
           "NONFINITE", "SolveInfo", "bicgstab", "rbicgstab", "rbicg", "Blocks",
           "make_blocks", "empty_blocks", "two_sided_ritz", "harmonic_ritz", "recycle_space",
           "run_sequence", "SequenceResult", "adjoint_solve", "gradients", "transposed_blocks"]

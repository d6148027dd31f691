"""Adjoint of a recycled solve -- oracle side (TEST INFRASTRUCTURE ONLY).

Model: the parametrised family of Section 6.1 with one parameter,
A(sigma) = K + sigma M (M diagonal), a solve A x = b, and a scalar loss
L = c^T x.  Differentiating A x = b gives, with the adjoint solution
lambda of A^T lambda = c,

    dL/db = lambda,
    dL/dA = -lambda x^T        (restricted to A's stored entries, which are K's),
    dL/dsigma = <dL/dA, M> = -sum_i lambda_i m_i x_i.

The adjoint system is solved by RBiCGSTAB (Section 4) on A^T with the recycle space
of A with the roles of U and Ut exchanged: for A^T the right space is Ut and
the left space U, so its blocks are built by ``make_blocks(A^T, A, Ut, U)``
(the same construction as for A, applied to the transposed operator).
"""
from __future__ import annotations

import numpy as np

from .krylov import rbicgstab
from .recycle import Blocks, make_blocks


def transposed_blocks(A, At, U: np.ndarray, Ut: np.ndarray, **kw) -> Blocks:
    """The recycle blocks (eq. CcheckChat) of the operator A^T with right space Ut, left space U."""
    return make_blocks(At, A, Ut, U, **kw)


def adjoint_solve(A, At, U: np.ndarray, Ut: np.ndarray, c: np.ndarray, rtol: float = 1e-10,
                  shadow=None, max_it: int = 20000):
    """lambda with A^T lambda = c by RBiCGSTAB on A^T (swapped recycle space)."""
    blocks = transposed_blocks(A, At, U, Ut)
    return rbicgstab(At, blocks, c, shadow_m1=shadow, rtol=rtol, max_it=max_it)


def gradients(rowptr: np.ndarray, colidx: np.ndarray, mdiag: np.ndarray, x: np.ndarray,
              lam: np.ndarray):
    """(dL/db, dL/dsigma, dL/dK values on the CSR pattern) from x and lambda."""
    n = x.shape[0]
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    g_val = -lam[rows] * x[colidx]
    g_sigma = -float(np.sum(lam * mdiag * x))
    return lam.copy(), g_sigma, g_val

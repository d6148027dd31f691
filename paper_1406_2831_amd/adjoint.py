"""Differentiable recycled solves for A(sigma) = K + sigma M.

``RecycledSolve`` is a ``torch.autograd.Function`` computing x = A(sigma)^-1 b
with the HIP library; its backward solves the adjoint system
A(sigma)^T lambda = dL/dx with RBiCGSTAB reusing the recycle space with the
roles of U and Ut swapped (``RBS_TRANSPOSE``: the left space Ut is the right
space of A^T), then forms

    dL/db = lambda,  dL/dsigma = -lambda^T M x,  dL/dK_ij = -lambda_i x_j

(the last on K's stored entries) in the library.  The matrix family is the
parametrised form of Section 6.1 with one parameter and M diagonal.  The
recycle space is treated as a constant: x does not depend on it.

This module orders library calls and marshals tensors; every arithmetic step
(value assembly, solves, gradients) runs in librbicgstab.so.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import scipy.sparse as sp
import torch

from .rbicgstab import Context, RbsError, rbicgstab_shifted_values


def transpose_pattern(rowptr: np.ndarray, colidx: np.ndarray, n: int):
    """CSR pattern of the transpose and the map perm with valT = val[perm]."""
    nnz = colidx.shape[0]
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    # entries are numbered 1..nnz so that no stored entry is an explicit zero
    t = sp.coo_matrix((np.arange(1, nnz + 1, dtype=np.float64), (colidx.astype(np.int64), rows)),
                      shape=(n, n)).tocsr()
    t.sort_indices()
    if t.nnz != nnz:
        raise ValueError("pattern has duplicate entries")
    return (t.indptr.astype(np.int32), t.indices.astype(np.int32),
            (t.data.astype(np.int64) - 1))


class ShiftedSystem:
    """A(sigma) = K + sigma diag(m) on one library context (device resident).

    K is a CSR object with ``rowptr``, ``colidx``, ``val`` (every row stores
    its diagonal); ``mdiag`` the diagonal of M.  ``bind(kval, sigma)`` forms
    A's values on the device and binds A, A^T to the context (keeping its
    recycle space).
    """

    def __init__(self, K, mdiag, k_max: int = 20, s_max: int = 512, device: str = "cuda",
                 secant_max: float = 0.0):
        n = int(K.n)
        rp, ci = np.asarray(K.rowptr), np.asarray(K.colidx)
        rows = np.repeat(np.arange(n), np.diff(rp))
        hit = np.nonzero(ci == rows)[0]
        diag = np.full(n, -1, dtype=np.int64)
        diag[rows[hit]] = hit
        if np.any(diag < 0):
            raise ValueError("K must store every diagonal entry")
        rpt, cit, perm = transpose_pattern(rp, ci, n)
        self.n, self.nnz, self.device = n, int(ci.shape[0]), device
        d = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
        self.rowptr, self.colidx = d(rp, torch.int32), d(ci, torch.int32)
        self.rowptrT, self.colidxT = d(rpt, torch.int32), d(cit, torch.int32)
        self.diag_pos, self.perm_t = d(diag, torch.int64), d(perm, torch.int64)
        self.mdiag = d(mdiag, torch.float64)
        self.kval0 = d(K.val, torch.float64)
        self.val = torch.empty(self.nnz, dtype=torch.float64, device=device)
        self.valT = torch.empty_like(self.val)
        mrow = int(max(np.diff(rp).max(), np.diff(rpt).max()))
        self.ctx = Context(n, mrow, k_max, s_max, device, secant_max)
        self._bound = None

    def bind(self, kval: Optional[torch.Tensor] = None, sigma: float = 0.0):
        kval = self.kval0 if kval is None else kval.detach()
        if self._bound is not None:
            bk, bver, bsig = self._bound
            # the bound tensor stays referenced, so its storage cannot be reused:
            # same address + same version counter means the same values
            if (bk.data_ptr() == kval.data_ptr() and bk.numel() == kval.numel()
                    and bver == kval._version and bsig == float(sigma)):
                return self
        kc = kval.contiguous()
        rbicgstab_shifted_values(kc, self.diag_pos, self.mdiag, float(sigma), self.perm_t,
                                 self.val, self.valT)
        self.ctx.setup((self.rowptr, self.colidx, self.val), (self.rowptrT, self.colidxT, self.valT))
        self._bound = (kval, kval._version, float(sigma))
        return self

    def solve(self, b, sigma, kval=None, rtol=1e-10, max_it=20000, mode="rbicgstab",
              transpose=False, shadow=None):
        self.bind(kval, sigma)
        x, st = self.ctx.solve(b.contiguous(), rtol=rtol, max_it=max_it, mode=mode,
                               transpose=transpose, shadow=shadow)
        if st.status != 0:
            raise RbsError(st.status, f"solve did not converge: {st.as_dict()}")
        return x, st

    def grads(self, lam, x):
        """(dL/dK values, dL/dsigma) for the bound matrix."""
        return self.ctx.adjoint_grads(self.rowptr, self.colidx, lam, x, self.mdiag)

    def close(self):
        self.ctx.close()


class RecycledSolve(torch.autograd.Function):
    """x = A(sigma)^-1 b with A(sigma) = K + sigma M (K's values ``kval``).

    ``mode`` picks the forward solver: "rbicgstab" (installed space),
    "bicgstab", or "rbicg" (RBiCG, whose space is installed for the adjoint
    solve and for later systems).  The adjoint is always RBiCGSTAB on A^T with
    the swapped space (plain BiCGSTAB when no space is installed).
    """

    @staticmethod
    def forward(ctx, system: ShiftedSystem, b, sigma, kval, rtol: float = 1e-10,
                max_it: int = 20000, mode: str = "rbicgstab"):
        sig = float(sigma)
        x, st = system.solve(b.detach(), sig, kval, rtol=rtol, max_it=max_it, mode=mode)
        if mode == "rbicg":
            system.ctx.recycle("from_last_solve")
        ctx.system, ctx.sig, ctx.rtol, ctx.max_it = system, sig, rtol, max_it
        ctx.kval = kval.detach()
        ctx.save_for_backward(x)
        ctx.forward_stats = st.as_dict()
        return x.clone()

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        system = ctx.system
        lam, _ = system.solve(gx.detach().contiguous(), ctx.sig, ctx.kval, rtol=ctx.rtol,
                              max_it=ctx.max_it, mode="rbicgstab", transpose=True)
        gval, gsig = system.grads(lam, x)
        need_b, need_sigma, need_k = ctx.needs_input_grad[1:4]
        g_sigma = torch.tensor(gsig, dtype=torch.float64, device=x.device) if need_sigma else None
        return (None, lam if need_b else None, g_sigma, gval if need_k else None, None, None, None)


def recycled_solve(system: ShiftedSystem, b, sigma, kval, rtol: float = 1e-10,
                   max_it: int = 20000, mode: str = "rbicgstab"):
    return RecycledSolve.apply(system, b, sigma, kval, rtol, max_it, mode)

"""Sequence driver on the GPU library (Section 6.2 strategy).

For each matrix A(i) of a shifted sequence: bind it (``rbicgstab_setup``,
which recomputes C = A U, Ct = A^T Ut and the projection blocks for the new
matrix), solve its first right-hand side with RBiCG (``RBS_RBICG_GEN``) and
install the space built from its Lanczos vectors (``recycle_update``), then
solve the remaining right-hand sides with RBiCGSTAB.  ``mode="bicgstab"``
solves every system with plain BiCGSTAB on the same kernels.

All arithmetic runs in the HIP library; this module only orders the calls.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import time

import numpy as np
import torch

from .rbicgstab import Context, device_csr


@dataclass
class GpuSequenceResult:
    x: List[torch.Tensor] = field(default_factory=list)
    status: List[int] = field(default_factory=list)
    iters: List[int] = field(default_factory=list)
    matvecs: List[int] = field(default_factory=list)
    solver: List[str] = field(default_factory=list)
    rel_res_true: List[float] = field(default_factory=list)
    k_used: List[int] = field(default_factory=list)
    ms: List[float] = field(default_factory=list)        # host wall time of each solve call
                                                         # (a multi-RHS call: on its first system)
    ritz_ms: List[float] = field(default_factory=list)   # of which Ritz steps (RBiCG solves)
    ritz_m: List[int] = field(default_factory=list)      # stored vectors of the last Ritz step
    setup_matvecs: int = 0
    setup_ms: float = 0.0      # matrix binds and recycle-space installs (host wall time)

    @property
    def total_matvecs(self) -> int:
        return int(sum(self.matvecs)) + int(self.setup_matvecs)


def max_row_nnz(*mats) -> int:
    return int(max(np.diff(m.rowptr).max() for m in mats))


class GpuSequence:
    """Device-resident inputs of a ``workloads.ShiftedSequence`` plus a solver context."""

    def __init__(self, seq, k: Optional[int] = None, s_max: int = 512, device: str = "cuda",
                 secant_max: float = 0.0, keep_x: bool = True):
        self.seq = seq
        self.k = seq.k if k is None else k
        self.device = device
        self.keep_x = keep_x
        mats = [seq.matrix(i) for i in range(len(seq.sigmas))]
        self.mrow = max_row_nnz(*[m for pair in mats for m in pair])
        self.mats = [(device_csr(A, device), device_csr(At, device)) for A, At in mats]
        self.rhs = [torch.as_tensor(b, device=device) for b in seq.rhs]
        self.shadows = [torch.as_tensor(s, device=device) for s in seq.shadows]
        self.ctx = Context(seq.n, self.mrow, max(self.k, 1), s_max, device, secant_max)
        # per-system solutions; rows of one (systems, n) block so that the
        # right-hand sides of one matrix can also be solved together
        self.xblock = torch.zeros((seq.num_systems, seq.n), dtype=torch.float64, device=device)
        self.xbuf = [self.xblock[i] for i in range(seq.num_systems)]
        self.rhs_block = torch.stack(self.rhs).contiguous()
        self.shadow_block = torch.stack(self.shadows).contiguous()

    def run(self, mode: str = "rbicgstab", rtol: float = 1e-8, max_it: int = 20000,
            systems: Optional[int] = None, precision: str = "fp64",
            multi_rhs: bool = False, rbicg_stop: str = "both") -> GpuSequenceResult:
        """precision applies to the RBiCGSTAB / BiCGSTAB solves ("fp64" or
        "fp32_ir"); RBiCG and the recycle-space update always run in FP64.
        multi_rhs: the RBiCGSTAB right-hand sides of each matrix (all of them
        for BiCGSTAB) are solved together by rbicgstab_solve_multi (FP64).
        rbicg_stop: RBiCG's stopping rule, "both" residuals or "primary" alone."""
        seq, ctx = self.seq, self.ctx
        out = GpuSequenceResult()
        last = seq.num_systems if systems is None else min(systems, seq.num_systems)
        if multi_rhs and precision != "fp64":
            raise ValueError("multi-RHS solves are FP64")
        if ctx.handle is not None:
            ctx.recycle("clear")
        results = {}
        idx = 0
        while idx < last:
            si, j = seq.system(idx)
            if j == 0:
                A, At = self.mats[si]
                t0 = time.perf_counter()
                ctx.setup(A, At)
                out.setup_ms += (time.perf_counter() - t0) * 1e3
                ma, mat = ctx.setup_matvecs()
                out.setup_matvecs += ma + mat
            gen = mode != "bicgstab" and j == 0 and self.k > 0
            end = min((si + 1) * seq.nrhs, last)   # systems of this matrix
            if multi_rhs and not gen and end - idx > 1:
                grp = list(range(idx, end))
                X = self.xblock[idx:end]
                X.zero_()
                _, sts = ctx.solve_multi(self.rhs_block[idx:end], X, self.shadow_block[idx:end],
                                         rtol=rtol, max_it=max_it, mode=mode)
                for g, st in zip(grp, sts):   # one call: its time counted once
                    results[g] = (st, mode, st.ms if g == grp[0] else 0.0)
                idx = end
                continue
            b, sh, x = self.rhs[idx], self.shadows[idx], self.xbuf[idx]
            x.zero_()
            if mode == "bicgstab":
                _, st = ctx.solve(b, x, shadow=sh, rtol=rtol, max_it=max_it, mode="bicgstab",
                                  precision=precision)
                solver = "bicgstab"
            elif gen:
                _, st = ctx.solve(b, x, shadow=sh, rtol=rtol, max_it=max_it, mode="rbicg",
                                  stop=rbicg_stop)
                t0 = time.perf_counter()
                ctx.recycle("from_last_solve")
                out.setup_ms += (time.perf_counter() - t0) * 1e3
                ma, mat = ctx.setup_matvecs()
                out.setup_matvecs += ma + mat
                solver = "rbicg"
            else:
                _, st = ctx.solve(b, x, shadow=sh, rtol=rtol, max_it=max_it, mode="rbicgstab",
                                  precision=precision)
                solver = "rbicgstab"
            results[idx] = (st, solver, st.ms)
            idx += 1
        for i in range(last):
            st, solver, call_ms = results[i]
            if self.keep_x:
                out.x.append(self.xbuf[i])
            out.status.append(st.status)
            out.iters.append(st.total_iters)
            out.matvecs.append(st.matvecs_A + st.matvecs_At)
            out.solver.append(solver)
            out.rel_res_true.append(st.rel_res_true)
            out.k_used.append(st.k_used)
            out.ms.append(call_ms)
            out.ritz_ms.append(st.ritz_ms if solver == "rbicg" else 0.0)
            out.ritz_m.append(st.ritz_m if solver == "rbicg" else 0)
        return out

    def close(self):
        self.ctx.close()

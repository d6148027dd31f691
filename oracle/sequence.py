"""Sequence driver of Section 6.2 (oracle, FP64) -- TEST INFRASTRUCTURE ONLY.

For each matrix ``A(i)`` (shift-major order of Section 6.1): the first
right-hand side is solved with RBiCG (Section 3; dual right-hand side of
all ones), whose Lanczos vectors build or improve the recycle space in
cycles of ``s`` iterations; every other right-hand side of the same matrix
is solved with RBiCGSTAB (Section 4) using that space.  The first system
starts with an empty space.  ``mode="bicgstab"`` runs the non-recycling
baseline on every system.

The space is updated by ``recycle.recycle_space`` (harmonic right, two-sided
left Ritz vectors).  Readings: the projection used inside a solve is fixed; the improved space is
installed (``make_blocks``) after the RBiCG solve ends, and only if that
solve converged.  Cycle updates combine the space being built with the
cycle's Lanczos vectors, ``W = [U_new, V_s]``, ``Wt = [Ut_new, Vt_s]``,
starting from the current space.  ``s=None`` uses cycles of ``S_DEFAULT``
vectors, long enough to hold a whole RBiCG solve on these workloads (one
update at its end): short cycles discard the small-eigenvalue information
on these operators (see the design notes).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List

import numpy as np

from .krylov import OK, bicgstab, rbicg, rbicgstab
from .recycle import make_blocks, empty_blocks, recycle_space


@dataclass
class SequenceResult:
    x: List[np.ndarray] = field(default_factory=list)
    status: List[int] = field(default_factory=list)
    iters: List[int] = field(default_factory=list)
    matvecs: List[int] = field(default_factory=list)
    solver: List[str] = field(default_factory=list)
    rel_res_true: List[float] = field(default_factory=list)
    seconds: List[float] = field(default_factory=list)
    k_used: List[int] = field(default_factory=list)   # recycle dimension each solve projects with
    # largest condition number of the column-scaled Lanczos stores whose Ritz
    # steps built the space each solve projects with, and the spaces upstream
    # of it (nan: no space, or not tracked)
    store_cond: List[float] = field(default_factory=list)

    @property
    def total_matvecs(self) -> int:
        return int(sum(self.matvecs))


S_DEFAULT = 512   # Lanczos vectors kept per cycle (a whole solve at these sizes)


def run_sequence(seq, mode: str = "rbicgstab", k: int = None, s: int = None,
                 rtol: float = 1e-8, max_it: int = 20000, systems=None,
                 rbicg_stop: str = "both", secant_max: float = 1e2,
                 track_store_cond: bool = False) -> SequenceResult:
    """Solve the systems of ``seq`` (a ``workloads.ShiftedSequence``) in order.

    ``systems`` limits the run to the first ``systems`` systems (a bounded sample).
    ``rbicg_stop`` is RBiCG's stopping rule (``krylov.rbicg``'s ``stop``);
    ``secant_max`` the oblique-projector cap of ``recycle.make_blocks``.
    ``track_store_cond`` records, per solve, the condition number of the
    (column-scaled) stored Lanczos basis its recycle space was computed from:
    the Ritz step is only as well determined as that basis.
    """
    k = seq.k if k is None else k
    if s is None:
        s = S_DEFAULT
    n = seq.n
    out = SequenceResult()
    U = np.zeros((n, 0))
    Ut = np.zeros((n, 0))
    last = seq.num_systems if systems is None else min(systems, seq.num_systems)
    cur_shift = -1
    A = At = None
    blocks = empty_blocks(n)
    space_cond = np.nan
    for idx in range(last):
        si, j = seq.system(idx)
        t0 = time.perf_counter()
        mv = 0
        if si != cur_shift:
            Acsr, Atcsr = seq.matrix(si)
            A, At = Acsr.to_scipy(), Atcsr.to_scipy()
            cur_shift = si
            if mode != "bicgstab":
                blocks = make_blocks(A, At, U, Ut, secant_max=secant_max)
                mv += blocks.matvecs_A + blocks.matvecs_At
        b = seq.rhs[idx]
        k_solve = blocks.k if mode != "bicgstab" else 0   # the projection this solve uses
        cond_solve = space_cond if k_solve > 0 else np.nan
        if mode == "bicgstab":
            x, info = bicgstab(A, b, shadow=seq.shadows[idx], rtol=rtol, max_it=max_it)
            mv += info.matvecs_A
            solver = "bicgstab"
        elif j == 0:
            state = {"U": blocks.U, "Ut": blocks.Ut, "mv": 0}

            def on_cycle(V, Vt):
                W = np.hstack([state["U"], V])
                Wt = np.hstack([state["Ut"], Vt])
                if track_store_cond:
                    state["cond"] = max(np.linalg.cond(W / np.linalg.norm(W, axis=0)),
                                        np.linalg.cond(Wt / np.linalg.norm(Wt, axis=0)))
                Un, Utn, m = recycle_space(A, W, Wt, k)
                state["U"], state["Ut"] = Un, Utn
                state["mv"] += m

            x, _, info = rbicg(A, At, blocks, b, rtol=rtol, max_it=max_it, s=s,
                               on_cycle=on_cycle, stop=rbicg_stop)
            mv += info.matvecs_A + info.matvecs_At + state["mv"]
            solver = "rbicg"
            converged = info.status == OK
            if not converged:
                # finish from the RBiCG iterate with RBiCGSTAB on the old space
                x, info2 = rbicgstab(A, blocks, b, x_m1=x, shadow_m1=seq.shadows[idx],
                                     rtol=rtol, max_it=max_it)
                mv += info2.matvecs_A
                info.iters += info2.total_iters
                info.status = info2.status
                info.rel_res_true = info2.rel_res_true
            if converged:
                U, Ut = state["U"], state["Ut"]
                # a space is as well determined as its store and every space upstream
                space_cond = np.nanmax([state.get("cond", np.nan), cond_solve])
                blocks = make_blocks(A, At, U, Ut, secant_max=secant_max)
                U, Ut = blocks.U, blocks.Ut
                mv += blocks.matvecs_A + blocks.matvecs_At
        else:
            x, info = rbicgstab(A, blocks, b, shadow_m1=seq.shadows[idx], rtol=rtol,
                                max_it=max_it)
            mv += info.matvecs_A
            solver = "rbicgstab"
        out.seconds.append(time.perf_counter() - t0)
        out.x.append(x)
        out.status.append(info.status)
        out.iters.append(info.total_iters if solver != "rbicg" else info.iters)
        out.matvecs.append(mv)
        out.solver.append(solver)
        out.rel_res_true.append(info.rel_res_true)
        out.k_used.append(k_solve)
        out.store_cond.append(cond_solve)
    return out

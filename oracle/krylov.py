"""BiCGSTAB, RBiCGSTAB (Section 4) and RBiCG (Section 3) in plain FP64 -- TEST INFRASTRUCTURE ONLY.

Real arithmetic throughout, so the paper's ``*`` is a transpose and complex
conjugates of scalars are the scalars themselves (Section 1 notation).

Readings of points the paper leaves open (listed again in the design notes):

* convergence: ``||r_i|| <= rtol * ||b||`` on the recurrence residual; after
  the final ``x <- x - U x_c`` the true residual ``b - A x`` is checked and,
  if it is above ``rtol * ||b||``, the solve restarts from that ``x`` (at most
  ``max_restarts`` times);
* breakdowns are only detected and reported (the paper assumes they do not
  happen): an exactly zero ``(rt0, r)``, ``(rt0, q)``, ``(t, t)`` or
  ``omega``, and any non-finite scalar, is reported; if
  ``(t, t) = 0`` while ``||s|| <= tol`` the half step ``x + alpha p`` is
  accepted;
* RBiCG stops when the primary and the dual residual both meet the
  relative tolerance (each against its own right-hand side).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from .recycle import Blocks, empty_blocks

OK = 0
MAXIT = 1
BREAKDOWN_RHO = 2
BREAKDOWN_ALPHA = 3
BREAKDOWN_OMEGA = 4
NONFINITE = -5


def _zero(val: float, a: np.ndarray, b: np.ndarray) -> bool:
    """Breakdown test of the start (r_0, rt_0) = 0 and of the recurrences: an exact zero."""
    return val == 0.0


@dataclass
class SolveInfo:
    status: int = OK
    iters: int = 0                 # iterations of the final (accepted) pass
    total_iters: int = 0           # summed over restarts
    matvecs_A: int = 0
    matvecs_At: int = 0
    restarts: int = 0
    rel_res_recur: float = np.nan
    rel_res_true: float = np.nan
    rel_res_dual: float = np.nan   # RBiCG: true relative residual of the dual system
    res_hist: List[float] = field(default_factory=list)
    trace: dict = field(default_factory=dict)   # optional per-iteration vectors (tests)


def _bad(*vals) -> bool:
    return any((not np.isfinite(v)) for v in vals)


def bicgstab(A, b: np.ndarray, x0: Optional[np.ndarray] = None,
             shadow: Optional[np.ndarray] = None, rtol: float = 1e-8,
             max_it: int = 10000, max_restarts: int = 3, record: bool = False):
    """van der Vorst's BiCGSTAB (the baseline named in Section 1; the k = 0 case of Section 4).

    ``shadow`` is the fixed vector ``r^`` of the inner products (defaults to
    the initial residual).  Returns ``(x, SolveInfo)``.
    """
    n = b.shape[0]
    info = SolveInfo()
    bnorm = np.linalg.norm(b)
    if _bad(bnorm):
        info.status = NONFINITE
        return np.zeros(n), info
    tol = rtol * bnorm
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    started_nonzero = x0 is not None and np.any(x != 0)
    trace = {"r": [], "x": []} if record else {}
    for attempt in range(max_restarts + 1):
        if started_nonzero or attempt > 0:
            r = b - A @ x
            info.matvecs_A += 1
        else:
            r = b.copy()
        rhat = r.copy() if shadow is None else np.array(shadow, dtype=np.float64)
        rho_prev = alpha = omega = 1.0
        p = np.zeros(n)
        v = np.zeros(n)
        info.iters = 0
        status = MAXIT
        rho = rhat @ r
        for i in range(1, max_it + 1):
            if _bad(rho) or _zero(rho, rhat, r):
                status = NONFINITE if _bad(rho) else BREAKDOWN_RHO
                break
            if i == 1:
                p = r.copy()
            else:
                beta = (rho / rho_prev) * (alpha / omega)
                p = r + beta * (p - omega * v)
            v = A @ p
            den = rhat @ v
            if _bad(den) or _zero(den, rhat, v):
                status = NONFINITE if _bad(den) else BREAKDOWN_ALPHA
                break
            alpha = rho / den
            s = r - alpha * v
            t = A @ s
            info.matvecs_A += 2
            tt = t @ t
            info.iters = i
            if tt == 0.0:
                if np.linalg.norm(s) <= tol:
                    x = x + alpha * p
                    r = s
                    status = OK
                else:
                    status = BREAKDOWN_OMEGA
                break
            omega = (t @ s) / tt
            x = x + alpha * p + omega * s
            r = s - omega * t
            rn = np.linalg.norm(r)
            info.res_hist.append(rn / bnorm)
            if record:
                trace["r"].append(r.copy())
                trace["x"].append(x.copy())
            if _bad(rn):
                status = NONFINITE
                break
            if rn <= tol:
                status = OK
                break
            if omega == 0.0:
                status = BREAKDOWN_OMEGA
                break
            rho_prev = rho
            rho = rhat @ r
        info.total_iters += info.iters
        info.rel_res_recur = np.linalg.norm(r) / bnorm
        rt = np.linalg.norm(b - A @ x) / bnorm
        info.matvecs_A += 1
        info.rel_res_true = rt
        info.status = status
        if status != OK or rt <= rtol or attempt == max_restarts:
            if status == OK and rt > rtol:
                info.status = MAXIT
            break
        info.restarts += 1
    info.trace = trace
    return x, info


class _Projected:
    """The projected operators of Sections 3 and 4 built from recycle blocks.

    ``B v = (I - C Chat^T) A v`` (primary side) and
    ``Bt v = (I - Ct Ccheck^T) A^T v`` (dual side).  Each application also
    returns the coefficient vector that the projection removed
    (``Chat^T A v`` or ``Ccheck^T A^T v``): because ``C = A U`` (and
    ``Ct = A^T Ut``), the removed part is ``A U`` times that vector, so a
    running sum of the coefficients is the ``U`` component that the final
    correction ``x - U x_c`` takes back out.
    """

    def __init__(self, A, At, blocks: Blocks):
        self.A, self.At, self.bl = A, At, blocks
        self.k = blocks.k

    def primary(self, v):
        Av = self.A @ v
        coef = self.bl.Chat.T @ Av
        return Av - self.bl.C @ coef, coef

    def dual(self, v):
        Atv = self.At @ v
        coef = self.bl.Ccheck.T @ Atv
        return Atv - self.bl.Ct @ coef, coef


def _initial_projection(blocks: Blocks, r_m1: np.ndarray, x: np.ndarray):
    """eq. (minusXR), primary side: x_0 = x_{-1} + U Chat^T r_{-1}, r_0 = r_{-1} - C Chat^T r_{-1}."""
    coef = blocks.Chat.T @ r_m1
    return x + blocks.U @ coef, r_m1 - blocks.C @ coef


def _initial_projection_dual(blocks: Blocks, rt_m1: np.ndarray, xt: np.ndarray):
    """eq. (minusXR), dual side: xt_0 = xt_{-1} + Ut Ccheck^T rt_{-1}, rt_0 = rt_{-1} - Ct Ccheck^T rt_{-1}."""
    coef = blocks.Ccheck.T @ rt_m1
    return xt + blocks.Ut @ coef, rt_m1 - blocks.Ct @ coef


def rbicgstab(A, blocks: Blocks, b: np.ndarray, x_m1: Optional[np.ndarray] = None,
              shadow_m1: Optional[np.ndarray] = None, rtol: float = 1e-8,
              max_it: int = 10000, max_restarts: int = 3, record: bool = False):
    """RBiCGSTAB (Section 4): BiCGSTAB applied to the projected operator.

    Section 4 derives the method as van der Vorst's BiCGSTAB run on
    ``B = (I - C Chat^T) A`` from the projected start of eq. (minusXR), with
    the shadow vector projected by ``I - Ct Ccheck^T``.  Every product with
    ``B`` leaves behind the coefficients ``Chat^T A v``; weighted by the step
    lengths they accumulate into the k-vector ``x_c``, and the solution is
    ``x - U x_c`` (``C = A U``).  ``blocks`` carries ``U``, ``C``,
    ``Chat = Ct D_c^{-1}`` and, for the shadow, ``Ct`` and ``Ccheck``.
    ``shadow_m1`` is the random shadow before projection (defaults to the
    initial residual).  Returns ``(x, SolveInfo)``, ``x`` corrected.
    """
    n = b.shape[0]
    Bop = _Projected(A, None, blocks)
    k = blocks.k
    info = SolveInfo()
    bnorm = np.linalg.norm(b)
    if _bad(bnorm):
        info.status = NONFINITE
        return np.zeros(n), info
    tol = rtol * bnorm
    x = np.zeros(n) if x_m1 is None else np.array(x_m1, dtype=np.float64)
    started_nonzero = x_m1 is not None and np.any(x != 0)
    trace = {"r": [], "x": [], "xc": [], "s": [], "q": [], "t": []} if record else {}
    for attempt in range(max_restarts + 1):
        if started_nonzero or attempt > 0:
            r_m1 = b - A @ x
            info.matvecs_A += 1
        else:
            r_m1 = b.copy()
        shadow = r_m1.copy() if shadow_m1 is None else np.array(shadow_m1, dtype=np.float64)
        x, r = _initial_projection(blocks, r_m1, x)
        _, rt0 = _initial_projection_dual(blocks, shadow, np.zeros(n))
        if record:
            trace["r0"], trace["x0"], trace["rt0"] = r.copy(), x.copy(), rt0.copy()
        rho = rt0 @ r
        status = MAXIT
        info.iters = 0
        xc = np.zeros(k)
        if np.linalg.norm(r) <= tol:
            status = OK              # r_0 already small: the projection solved it (b in range(C))
        elif _bad(rho) or _zero(rho, rt0, r):
            status = NONFINITE if _bad(rho) else BREAKDOWN_RHO
        else:
            beta = omega = 0.0
            p = np.zeros(n)
            q = np.zeros(n)          # the previous B p
            for i in range(1, max_it + 1):
                p = r + beta * (p - omega * q)
                q, zeta = Bop.primary(p)
                den = rt0 @ q
                if _bad(den) or _zero(den, rt0, q):
                    status = NONFINITE if _bad(den) else BREAKDOWN_ALPHA
                    break
                alpha = rho / den
                s = r - alpha * q
                t, gamma = Bop.primary(s)
                info.matvecs_A += 2
                info.iters = i
                tt = t @ t
                if tt == 0.0:
                    if np.linalg.norm(s) <= tol:
                        x = x + alpha * p
                        xc = xc + alpha * zeta
                        r = s
                        status = OK
                    else:
                        status = BREAKDOWN_OMEGA
                    break
                omega = (s @ t) / tt
                x = x + alpha * p + omega * s
                xc = xc + alpha * zeta + omega * gamma
                r_new = s - omega * t
                rn = np.linalg.norm(r_new)
                info.res_hist.append(rn / bnorm)
                if record:
                    for key, val in (("r", r_new), ("x", x), ("xc", xc), ("s", s),
                                     ("q", q), ("t", t)):
                        trace[key].append(val.copy())
                r = r_new
                if _bad(rn):
                    status = NONFINITE
                    break
                if rn <= tol:
                    status = OK
                    break
                if omega == 0.0:
                    status = BREAKDOWN_OMEGA
                    break
                rho_new = rt0 @ r
                if _zero(rho_new, rt0, r):
                    status = BREAKDOWN_RHO
                    break
                beta = (rho_new / rho) * (alpha / omega)
                rho = rho_new
        x = x - blocks.U @ xc
        info.total_iters += info.iters
        info.rel_res_recur = np.linalg.norm(r) / bnorm
        rt = np.linalg.norm(b - A @ x) / bnorm
        info.matvecs_A += 1
        info.rel_res_true = rt
        info.status = status
        if status != OK or rt <= rtol or attempt == max_restarts:
            if status == OK and rt > rtol:
                info.status = MAXIT
            break
        info.restarts += 1
    info.trace = trace
    return x, info


def rbicg(A, At, blocks: Blocks, b: np.ndarray, bt: Optional[np.ndarray] = None,
          x_m1: Optional[np.ndarray] = None, xt_m1: Optional[np.ndarray] = None,
          rtol: float = 1e-8, max_it: int = 10000, s: int = 0,
          on_cycle: Optional[Callable[[np.ndarray, np.ndarray], None]] = None,
          stop: str = "both", record: bool = False):
    """RBiCG (Section 3): BiCG on the primary and dual systems with the
    projected operators ``B = (I - C Chat^T) A`` and ``Bt = (I - Ct Ccheck^T) A^T``
    (augmented bi-Lanczos, Theorem 1), started by eq. (minusXR) on both sides.

    Both solutions are corrected at the end by the accumulated ``U`` and
    ``Ut`` components.  The solve stops when both residuals meet their
    tolerance (``||r|| <= rtol ||b||`` and ``||rt|| <= rtol ||bt||``), the
    rule of the RBiCG algorithm in Section 3; ``stop="primary"`` stops on the
    primary residual alone (an option, not the paper's rule).  The dual
    right-hand side ``bt`` defaults to the vector of all ones (the choice of
    Section 6.2).  The Lanczos vectors are the normalised residuals
    ``r_{i-1}/||r_{i-1}||`` and ``rt_{i-1}/||rt_{i-1}||``; every ``s``
    iterations (and once more at the end for a partial cycle) they are
    handed to ``on_cycle(V, Vt)`` and discarded.  ``info.rel_res_dual`` is the
    dual system's true relative residual.  Returns ``(x, xt, SolveInfo)``.
    """
    if stop not in ("both", "primary"):
        raise ValueError("stop must be 'both' or 'primary'")
    n = b.shape[0]
    ops = _Projected(A, At, blocks)
    k = blocks.k
    info = SolveInfo()
    if bt is None:
        bt = np.ones(n)
    bnorm = np.linalg.norm(b)
    btnorm = np.linalg.norm(bt)
    if _bad(bnorm) or _bad(btnorm):
        info.status = NONFINITE
        return np.zeros(n), np.zeros(n), info
    tol = rtol * bnorm
    tol_dual = rtol * btnorm if stop == "both" else np.inf
    x = np.zeros(n) if x_m1 is None else np.array(x_m1, dtype=np.float64)
    xt = np.zeros(n) if xt_m1 is None else np.array(xt_m1, dtype=np.float64)
    if np.any(x != 0):
        r_m1 = b - A @ x
        info.matvecs_A += 1
    else:
        r_m1 = b.copy()
    if np.any(xt != 0):
        rt_m1 = bt - At @ xt
        info.matvecs_At += 1
    else:
        rt_m1 = np.array(bt, dtype=np.float64)
    x, r = _initial_projection(blocks, r_m1, x)
    xt, rt = _initial_projection_dual(blocks, rt_m1, xt)
    trace = {"r": [r.copy()], "rt": [rt.copy()]} if record else {}
    p = np.zeros(n)
    pt = np.zeros(n)
    zc = np.zeros(k)      # accumulated U coefficients of x
    ztc = np.zeros(k)     # accumulated Ut coefficients of xt
    beta = 0.0
    rho = rt @ r
    status = MAXIT
    V, Vt = [], []

    def flush():
        if on_cycle is not None and V:
            on_cycle(np.array(V).T, np.array(Vt).T)
        V.clear()
        Vt.clear()

    def converged(rn, rtn):
        return rn <= tol and rtn <= tol_dual

    if converged(np.linalg.norm(r), np.linalg.norm(rt)):
        status = OK
    elif _bad(rho) or _zero(rho, rt, r):   # the caller re-chooses the dual start
        status = NONFINITE if _bad(rho) else BREAKDOWN_RHO
    else:
        for i in range(1, max_it + 1):
            if s > 0:
                V.append(r / np.linalg.norm(r))
                Vt.append(rt / np.linalg.norm(rt))
            p = r + beta * p
            pt = rt + beta * pt
            q, zeta = ops.primary(p)
            qt, zetat = ops.dual(pt)
            info.matvecs_A += 1
            info.matvecs_At += 1
            den = pt @ q
            info.iters = i
            if _bad(den) or _zero(den, pt, q):
                status = NONFINITE if _bad(den) else BREAKDOWN_ALPHA
                break
            alpha = rho / den        # real arithmetic: the dual step is the same alpha
            zc = zc + alpha * zeta
            ztc = ztc + alpha * zetat
            x = x + alpha * p
            xt = xt + alpha * pt
            r = r - alpha * q
            rt = rt - alpha * qt
            rn, rtn = np.linalg.norm(r), np.linalg.norm(rt)
            info.res_hist.append(rn / bnorm)
            if record:
                trace["r"].append(r.copy())
                trace["rt"].append(rt.copy())
            if _bad(rn) or _bad(rtn):
                status = NONFINITE
                break
            if converged(rn, rtn):
                status = OK
                break
            rho_new = rt @ r
            if _zero(rho_new, rt, r):
                status = BREAKDOWN_RHO
                break
            beta = rho_new / rho
            rho = rho_new
            if s > 0 and len(V) == s:
                flush()
    if s > 0:
        flush()
    x = x - blocks.U @ zc
    xt = xt - blocks.Ut @ ztc
    info.total_iters = info.iters
    info.rel_res_recur = np.linalg.norm(r) / bnorm
    info.rel_res_true = np.linalg.norm(b - A @ x) / bnorm
    info.rel_res_dual = np.linalg.norm(bt - At @ xt) / btnorm
    info.matvecs_A += 1
    info.matvecs_At += 1
    if status == OK and info.rel_res_true > rtol:
        status = MAXIT
    info.status = status
    info.trace = trace
    return x, xt, info

"""Thin Python binding of librbicgstab.so (argument marshalling only).

The functions ``rbicgstab_workspace_bytes``, ``rbicgstab_setup``,
``rbicgstab_solve``, ``recycle_update``, ``rbicgstab_get_blocks`` and
``rbicgstab_destroy`` mirror the C entry points of include/rbicgstab.h and
take torch tensors (device memory) plus a torch stream.  ``Context`` bundles
a handle with the workspace tensor it lives in.  Every computation runs in
the HIP library: if it is not built, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbicgstab.so")

RBS_OK = 0
RBS_MAXIT = 1
RBS_BREAKDOWN_RHO = 2
RBS_BREAKDOWN_ALPHA = 3
RBS_BREAKDOWN_OMEGA = 4
RBS_ERR_ARG = -1
RBS_ERR_HIP = -2
RBS_ERR_WORKSPACE = -3
RBS_ERR_SINGULAR_DC = -4
RBS_ERR_NONFINITE = -5

RBS_RBICGSTAB = 0
RBS_BICGSTAB = 1
RBS_RBICG_GEN = 2
RBS_TRANSPOSE = 8
RBS_FP32_IR = 16
RBS_STOP_PRIMARY = 32

RBS_RECYCLE_SET = 0
RBS_RECYCLE_FROM_LAST_SOLVE = 1
RBS_RECYCLE_CLEAR = 2

EXPORTS = ("rbicgstab_workspace_bytes", "rbicgstab_setup", "rbicgstab_solve", "recycle_update",
           "rbicgstab_get_blocks", "rbicgstab_time_pass", "rbicgstab_time_stream", "rbicgstab_setup_matvecs",
           "rbicgstab_adjoint_grads", "rbicgstab_shifted_values", "rbicgstab_solve_multi",
           "rbicgstab_destroy", "rbicgstab_last_error", "rbicgstab_batch_workspace_bytes",
           "rbicgstab_batch_create", "rbicgstab_batch_solve", "rbicgstab_batch_config",
           "rbicgstab_batch_destroy", "rbicgstab_batch_last_error", "rbicgstab_adjoint_grads_noalloc",
           "rbicgstab_gram_workspace_bytes", "rbicgstab_gram")
RBS_BATCH_TUNE = 1
RBS_BATCH_GRAPH = 2


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("total_iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("matvecs_A", ctypes.c_int32), ("matvecs_At", ctypes.c_int32),
                ("k_used", ctypes.c_int32), ("ritz_updates", ctypes.c_int32),
                ("rel_res_recur", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("ms", ctypes.c_double), ("ir_steps", ctypes.c_int32), ("ritz_m", ctypes.c_int32),
                ("ritz_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librbicgstab.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1406_2831_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, f64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                             ctypes.c_size_t)
    lib.rbicgstab_workspace_bytes.argtypes = [i64, i32, i32, i32]
    lib.rbicgstab_workspace_bytes.restype = sz
    lib.rbicgstab_setup.argtypes = [ctypes.POINTER(vp), i64, i64, vp, vp, vp, i64, vp, vp, vp,
                                    i32, i32, i32, f64, vp, sz, vp]
    lib.rbicgstab_setup.restype = ctypes.c_int
    lib.rbicgstab_solve.argtypes = [vp, vp, vp, i32, vp, f64, i32, i32, ctypes.POINTER(Stats)]
    lib.rbicgstab_solve.restype = ctypes.c_int
    lib.rbicgstab_solve_multi.argtypes = [vp, i32, vp, i64, vp, i64, vp, f64, i32, i32,
                                          ctypes.POINTER(Stats)]
    lib.rbicgstab_solve_multi.restype = ctypes.c_int
    lib.rbicgstab_batch_workspace_bytes.argtypes = [i32, ctypes.POINTER(i64)]
    lib.rbicgstab_batch_workspace_bytes.restype = sz
    lib.rbicgstab_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), vp, sz, i32]
    lib.rbicgstab_batch_create.restype = ctypes.c_int
    lib.rbicgstab_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), f64,
                                          i32, i32, ctypes.POINTER(Stats)]
    lib.rbicgstab_batch_solve.restype = ctypes.c_int
    lib.rbicgstab_batch_config.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(f64)]
    lib.rbicgstab_batch_config.restype = ctypes.c_int
    lib.rbicgstab_batch_destroy.argtypes = [vp]
    lib.rbicgstab_batch_destroy.restype = ctypes.c_int
    lib.rbicgstab_batch_last_error.argtypes = [vp]
    lib.rbicgstab_batch_last_error.restype = ctypes.c_char_p
    lib.recycle_update.argtypes = [vp, i32, vp, vp, i32]
    lib.recycle_update.restype = ctypes.c_int
    lib.rbicgstab_get_blocks.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(i32)]
    lib.rbicgstab_get_blocks.restype = ctypes.c_int
    lib.rbicgstab_time_pass.argtypes = [vp, i32, i32, i32, ctypes.POINTER(f64), ctypes.POINTER(f64)]
    lib.rbicgstab_time_pass.restype = ctypes.c_int
    lib.rbicgstab_time_stream.argtypes = [i32, i64, vp, vp, i32, i32, vp, ctypes.POINTER(f64), ctypes.POINTER(f64)]
    lib.rbicgstab_time_stream.restype = ctypes.c_int
    lib.rbicgstab_adjoint_grads.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, ctypes.POINTER(f64)]
    lib.rbicgstab_adjoint_grads.restype = ctypes.c_int
    lib.rbicgstab_adjoint_grads_noalloc.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.rbicgstab_adjoint_grads_noalloc.restype = ctypes.c_int
    lib.rbicgstab_gram_workspace_bytes.argtypes = [i64, i32, i32]
    lib.rbicgstab_gram_workspace_bytes.restype = sz
    lib.rbicgstab_gram.argtypes = [i64, vp, i64, i32, vp, i64, i32, vp, vp, sz, vp]
    lib.rbicgstab_gram.restype = ctypes.c_int
    lib.rbicgstab_shifted_values.argtypes = [i64, i64, vp, vp, vp, f64, vp, vp, vp, vp]
    lib.rbicgstab_shifted_values.restype = ctypes.c_int
    lib.rbicgstab_setup_matvecs.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.rbicgstab_setup_matvecs.restype = ctypes.c_int
    lib.rbicgstab_destroy.argtypes = [vp]
    lib.rbicgstab_destroy.restype = ctypes.c_int
    lib.rbicgstab_last_error.argtypes = [vp]
    lib.rbicgstab_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


class RbsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"librbicgstab error {code}: {msg}")
        self.code = code


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(lib, handle, rc: int) -> int:
    if rc < 0:
        msg = lib.rbicgstab_last_error(handle)
        raise RbsError(rc, msg.decode() if msg else "")
    return rc


# ----------------------------------------------------------------- C-named functions

def rbicgstab_workspace_bytes(n: int, max_row_nnz: int, k_max: int, s_max: int) -> int:
    return int(load_library().rbicgstab_workspace_bytes(n, max_row_nnz, k_max, s_max))


def rbicgstab_setup(handle: Optional[ctypes.c_void_p], n: int, A, At, max_row_nnz: int, k_max: int,
                    s_max: int, workspace: torch.Tensor, secant_max: float = 0.0, stream=None):
    """A, At: (rowptr int32, colidx int32, val float64) device tensors.  Returns the handle."""
    lib = load_library()
    h = handle if handle is not None else ctypes.c_void_p(None)
    rc = lib.rbicgstab_setup(ctypes.byref(h), n, A[1].numel(), _ptr(A[0]), _ptr(A[1]), _ptr(A[2]),
                             At[1].numel(), _ptr(At[0]), _ptr(At[1]), _ptr(At[2]), max_row_nnz,
                             k_max, s_max, secant_max, _ptr(workspace), workspace.numel(),
                             _stream(stream))
    _check(lib, h, rc)
    return h


def rbicgstab_solve(handle, b: torch.Tensor, x: torch.Tensor, x_nonzero: bool = False,
                    shadow: Optional[torch.Tensor] = None, rtol: float = 1e-8, max_it: int = 10000,
                    flags: int = RBS_RBICGSTAB) -> Stats:
    lib = load_library()
    st = Stats()
    rc = lib.rbicgstab_solve(handle, _ptr(b), _ptr(x), int(bool(x_nonzero)), _ptr(shadow), rtol,
                             max_it, flags, ctypes.byref(st))
    _check(lib, handle, rc)
    return st


def rbicgstab_solve_multi(handle, B: torch.Tensor, X: torch.Tensor, shadows: Optional[torch.Tensor] = None,
                          rtol: float = 1e-8, max_it: int = 10000, flags: int = RBS_RBICGSTAB):
    """B, X, shadows: (nrhs, n) row-major tensors == column-major n x nrhs blocks (ld = n)."""
    lib = load_library()
    nrhs, n = B.shape
    stats = (Stats * nrhs)()
    rc = lib.rbicgstab_solve_multi(handle, nrhs, _ptr(B), n, _ptr(X), X.shape[1], _ptr(shadows), rtol,
                                   max_it, flags, stats)
    _check(lib, handle, rc)
    return list(stats)


def recycle_update(handle, mode: int, U: Optional[torch.Tensor] = None,
                   Ut: Optional[torch.Tensor] = None) -> int:
    """U, Ut: (k, n) row-major torch tensors == column-major n x k blocks with ld = n."""
    lib = load_library()
    k = 0 if U is None else U.shape[0]
    return _check(lib, handle, lib.recycle_update(handle, mode, _ptr(U), _ptr(Ut), k))


def rbicgstab_get_blocks(handle, n: int, k_max: int, device="cuda"):
    """Returns dict of (k, n) tensors U, Ut, C, Ct, Chat, Ccheck (column j = row j)."""
    lib = load_library()
    out = {name: torch.zeros((k_max, n), dtype=torch.float64, device=device)
           for name in ("U", "Ut", "C", "Ct", "Chat", "Ccheck")}
    kk = ctypes.c_int32(0)
    _check(lib, handle, lib.rbicgstab_get_blocks(handle, *[_ptr(out[k]) for k in
                                                            ("U", "Ut", "C", "Ct", "Chat", "Ccheck")],
                                                 ctypes.byref(kk)))
    return {name: t[: kk.value].clone() for name, t in out.items()}, kk.value


def rbicgstab_time_pass(handle, which: int, k: int, reps: int):
    """(mean ms per launch, algorithmic bytes per launch) of one fused pass; for the
    Ritz-step matrix-core kernels (which 40..42) the second value is useful flops."""
    lib = load_library()
    ms, by = ctypes.c_double(0), ctypes.c_double(0)
    _check(lib, handle, lib.rbicgstab_time_pass(handle, which, k, reps, ctypes.byref(ms),
                                                ctypes.byref(by)))
    return ms.value, by.value


def rbicgstab_time_stream(kind: int, a: torch.Tensor, b: torch.Tensor, grid: int, reps: int, stream=None):
    """(mean ms per launch, bytes per launch) of a streaming reference kernel over the
    float64 device tensors a and b (kind 0 read, 1 copy, 2 seven-read / three-write mix)."""
    lib = load_library()
    ms, by = ctypes.c_double(0), ctypes.c_double(0)
    _check(lib, None, lib.rbicgstab_time_stream(kind, a.numel(), _ptr(a), _ptr(b), grid, reps,
                                                _stream(stream), ctypes.byref(ms), ctypes.byref(by)))
    return ms.value, by.value


def rbicgstab_adjoint_grads(handle, rowptr: torch.Tensor, colidx: torch.Tensor, lam: torch.Tensor,
                            x: torch.Tensor, mdiag: Optional[torch.Tensor], grad_val: torch.Tensor):
    """Fills grad_val (device, nnz) and returns dL/dsigma (host float)."""
    lib = load_library()
    gs = ctypes.c_double(0)
    _check(lib, handle, lib.rbicgstab_adjoint_grads(handle, colidx.numel(), _ptr(rowptr), _ptr(colidx),
                                                    _ptr(lam), _ptr(x), _ptr(mdiag), _ptr(grad_val),
                                                    ctypes.byref(gs)))
    return gs.value


def rbicgstab_adjoint_grads_noalloc(rowptr: torch.Tensor, colidx: torch.Tensor, lam: torch.Tensor,
                                    x: torch.Tensor, mdiag: Optional[torch.Tensor], grad_val: torch.Tensor,
                                    grad_sigma: torch.Tensor, stream=None) -> None:
    """The same gradients without a context or any allocation: grad_val (nnz) and
    grad_sigma (one double) are device tensors; the work is enqueued on `stream`."""
    lib = load_library()
    _check(lib, None, lib.rbicgstab_adjoint_grads_noalloc(lam.numel(), colidx.numel(), _ptr(rowptr),
                                                          _ptr(colidx), _ptr(lam), _ptr(x), _ptr(mdiag),
                                                          _ptr(grad_val), _ptr(grad_sigma), _stream(stream)))


def rbicgstab_gram(X: torch.Tensor, Y: torch.Tensor, stream=None) -> torch.Tensor:
    """X^T Y with the library's Gram kernels.  X (mx, n) and Y (my, n) are device
    tensors whose rows are the columns of the n x mx and n x my column-major
    operands (leading dimension n); passing the same tensor twice gives the
    symmetric product.  Returns the (my, mx) tensor whose rows are the columns
    of X^T Y, i.e. its transpose Y^T X in row-major terms (synchronised)."""
    lib = load_library()
    mx, n = X.shape
    my = Y.shape[0]
    out = torch.empty((my, mx), dtype=torch.float64, device=X.device)
    ws = torch.empty(max(1, lib.rbicgstab_gram_workspace_bytes(n, mx, my) // 8 + 32), dtype=torch.float64,
                     device=X.device)
    base = ws.data_ptr()
    aligned = (base + 255) // 256 * 256
    nbytes = ws.numel() * 8 - (aligned - base)
    _check(lib, None, lib.rbicgstab_gram(n, _ptr(X), n, mx, _ptr(Y), n, my, _ptr(out),
                                         ctypes.c_void_p(aligned), nbytes, _stream(stream)))
    torch.cuda.synchronize(X.device)
    return out


def rbicgstab_shifted_values(kval: torch.Tensor, diag_pos: torch.Tensor, mdiag: torch.Tensor,
                             sigma: float, perm_t: Optional[torch.Tensor], val: torch.Tensor,
                             valT: Optional[torch.Tensor], stream=None) -> None:
    """val = kval + sigma * mdiag on the diagonal entries; valT = val[perm_t] (device)."""
    lib = load_library()
    _check(lib, None, lib.rbicgstab_shifted_values(mdiag.numel(), kval.numel(), _ptr(kval),
                                                   _ptr(diag_pos), _ptr(mdiag), float(sigma),
                                                   _ptr(perm_t), _ptr(val), _ptr(valT),
                                                   _stream(stream)))


def rbicgstab_setup_matvecs(handle):
    lib = load_library()
    a, b = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib, handle, lib.rbicgstab_setup_matvecs(handle, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def rbicgstab_destroy(handle) -> None:
    if handle is not None and handle.value:
        load_library().rbicgstab_destroy(handle)


# ----------------------------------------------------------------- convenience wrapper

def device_csr(csr, device="cuda"):
    """Upload a CSR (rowptr, colidx, val numpy arrays, or an object with those fields)."""
    rp, ci, va = (csr.rowptr, csr.colidx, csr.val) if hasattr(csr, "rowptr") else csr
    return (torch.as_tensor(rp, dtype=torch.int32, device=device),
            torch.as_tensor(ci, dtype=torch.int32, device=device),
            torch.as_tensor(va, dtype=torch.float64, device=device))


@dataclass
class Context:
    """A recycling-BiCGSTAB context: workspace tensor + library handle."""
    n: int
    max_row_nnz: int
    k_max: int
    s_max: int
    device: str = "cuda"
    secant_max: float = 0.0

    def __post_init__(self):
        self.ws_bytes = rbicgstab_workspace_bytes(self.n, self.max_row_nnz, self.k_max, self.s_max)
        if self.ws_bytes == 0:
            raise RbsError(RBS_ERR_ARG, "invalid context sizes")
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.handle = None

    def setup(self, A, At, stream=None):
        """Bind A(i) (and its transpose); device tensors or host CSR objects."""
        if not isinstance(A[0] if isinstance(A, tuple) else None, torch.Tensor):
            A = device_csr(A, self.device)
            At = device_csr(At, self.device)
        self.handle = rbicgstab_setup(self.handle, self.n, A, At, self.max_row_nnz, self.k_max,
                                      self.s_max, self.workspace, self.secant_max, stream)
        return self

    def solve(self, b, x=None, x_nonzero=False, shadow=None, rtol=1e-8, max_it=10000,
              mode: str = "rbicgstab", transpose: bool = False, precision: str = "fp64",
              stop: str = "both"):
        """precision: "fp64", or "fp32_ir" (FP32 storage under FP64 iterative refinement).
        stop (mode "rbicg"): "both" residuals (the default), or "primary" alone."""
        flags = {"rbicgstab": RBS_RBICGSTAB, "bicgstab": RBS_BICGSTAB,
                 "rbicg": RBS_RBICG_GEN}[mode] | (RBS_TRANSPOSE if transpose else 0)
        flags |= {"fp64": 0, "fp32_ir": RBS_FP32_IR}[precision]
        flags |= {"both": 0, "primary": RBS_STOP_PRIMARY}[stop] if mode == "rbicg" else 0
        if x is None:
            x = torch.zeros_like(b)
        st = rbicgstab_solve(self.handle, b, x, x_nonzero, shadow, rtol, max_it, flags)
        return x, st

    def solve_multi(self, B, X=None, shadows=None, rtol=1e-8, max_it=10000, mode: str = "rbicgstab"):
        """B: (nrhs, n) device tensor (row j = right-hand side j); returns (X, [Stats])."""
        flags = {"rbicgstab": RBS_RBICGSTAB, "bicgstab": RBS_BICGSTAB}[mode]
        B = B.contiguous()
        if X is None:
            X = torch.zeros_like(B)
        st = rbicgstab_solve_multi(self.handle, B, X, None if shadows is None else shadows.contiguous(),
                                   rtol, max_it, flags)
        return X, st

    def recycle(self, mode: str = "from_last_solve", U=None, Ut=None):
        m = {"set": RBS_RECYCLE_SET, "from_last_solve": RBS_RECYCLE_FROM_LAST_SOLVE,
             "clear": RBS_RECYCLE_CLEAR}[mode]
        return recycle_update(self.handle, m, U, Ut)

    def blocks(self):
        return rbicgstab_get_blocks(self.handle, self.n, self.k_max, self.device)

    def setup_matvecs(self):
        return rbicgstab_setup_matvecs(self.handle)

    def adjoint_grads(self, rowptr, colidx, lam, x, mdiag=None, grad_val=None):
        if grad_val is None:
            grad_val = torch.empty(colidx.numel(), dtype=torch.float64, device=lam.device)
        gs = rbicgstab_adjoint_grads(self.handle, rowptr, colidx, lam, x, mdiag, grad_val)
        return grad_val, gs


    def time_pass(self, which: int, k: int, reps: int = 50):
        return rbicgstab_time_pass(self.handle, which, k, reps)

    def close(self):
        rbicgstab_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A batch of bound contexts solved together (rbicgstab_batch_*)."""

    def __init__(self, contexts, tune: bool = True, graph: bool = True, device: str = "cuda"):
        lib = load_library()
        self.contexts = list(contexts)
        nsys = len(self.contexts)
        n = (ctypes.c_int64 * nsys)(*[c.n for c in self.contexts])
        ws = int(lib.rbicgstab_batch_workspace_bytes(nsys, n))
        if ws == 0:
            raise RbsError(RBS_ERR_ARG, "invalid batch sizes")
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=device)
        handles = (ctypes.c_void_p * nsys)(*[c.handle.value for c in self.contexts])
        h = ctypes.c_void_p(None)
        flags = (RBS_BATCH_TUNE if tune else 0) | (RBS_BATCH_GRAPH if graph else 0)
        rc = lib.rbicgstab_batch_create(ctypes.byref(h), nsys, handles, _ptr(self.workspace), ws, flags)
        if rc < 0:
            msg = lib.rbicgstab_batch_last_error(None)
            raise RbsError(rc, msg.decode() if msg else "")
        self.handle = h

    def _check(self, rc):
        if rc < 0:
            msg = load_library().rbicgstab_batch_last_error(self.handle)
            raise RbsError(rc, msg.decode() if msg else "")
        return rc

    def config(self):
        rows, grid, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0)
        self._check(load_library().rbicgstab_batch_config(self.handle, ctypes.byref(rows), ctypes.byref(grid),
                                                          ctypes.byref(ms)))
        return {"tile_rows": rows.value, "grid": grid.value, "tuned_ms_per_iter": ms.value}

    def solve(self, bs, xs, shadows=None, rtol=1e-8, max_it=10000, mode: str = "rbicgstab",
              precision: str = "fp64"):
        """bs, xs (, shadows): lists of device tensors, one per system; precision
        "fp64" or "fp32_ir" (FP32 storage under FP64 iterative refinement)."""
        lib = load_library()
        nsys = len(self.contexts)
        P = ctypes.c_void_p * nsys
        pb = P(*[t.data_ptr() for t in bs])
        px = P(*[t.data_ptr() for t in xs])
        ps = P(*[t.data_ptr() for t in shadows]) if shadows is not None else None
        stats = (Stats * nsys)()
        flags = {"rbicgstab": RBS_RBICGSTAB, "bicgstab": RBS_BICGSTAB}[mode]
        flags |= {"fp64": 0, "fp32_ir": RBS_FP32_IR}[precision]
        torch.cuda.current_stream().synchronize()
        rc = lib.rbicgstab_batch_solve(self.handle, pb, px, ps, rtol, max_it, flags, stats)
        self._check(rc)
        return list(stats)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load_library().rbicgstab_batch_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

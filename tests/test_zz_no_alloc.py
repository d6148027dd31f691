"""The no-allocation gradient entry point against the context-based one.

rbicgstab_adjoint_grads_noalloc keeps its block partials in a file-scope
device array instead of a context's workspace; with the same kernels and the
same grid it must give bit-identical gradients.  Two calls in a row, the
second on a smaller system, check that the array's leftover contents from the
first call do not leak into the second.
"""
import sys

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _case(torch, rb, N, seed):
    """A shifted 3D system of N^3 rows with random lambda and x (device tensors)."""
    K = w.convdiff((N, N, N), w.VEL3, w.PECLET)
    rng = np.random.default_rng(seed)
    mdiag = rng.uniform(0.5, 1.5, size=K.n)
    lam = rng.standard_normal(K.n)
    x = rng.standard_normal(K.n)
    dev = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    return (K, dev(K.rowptr, torch.int32), dev(K.colidx, torch.int32), dev(lam), dev(x), dev(mdiag))


def test_noalloc_gradients_match_context_gradients():
    import torch
    from paper_1406_2831_amd import rbicgstab as rb
    from paper_1406_2831_amd.sequence import max_row_nnz
    assert torch.cuda.is_available()
    rb.load_library()
    for N, seed in ((48, 1), (20, 2)):       # the second call is smaller
        _say(f"adjoint gradients without allocation, N={N}")
        K, rowptr, colidx, lam, x, mdiag = _case(torch, rb, N, seed)
        # the context-based entry point
        ctx = rb.Context(K.n, max_row_nnz(K), 1, 0)
        ctx.setup(K, K.transpose())
        g_ref, s_ref = ctx.adjoint_grads(rowptr, colidx, lam, x, mdiag)
        # the no-allocation entry point
        g = torch.full_like(g_ref, np.nan)
        s = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
        rb.rbicgstab_adjoint_grads_noalloc(rowptr, colidx, lam, x, mdiag, g, s)
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref)
        assert float(s.item()) == s_ref
        # and both against the formula on the host
        ln, xn, mn = lam.cpu().numpy(), x.cpu().numpy(), mdiag.cpu().numpy()
        rows = np.repeat(np.arange(K.n), np.diff(K.rowptr))
        assert np.array_equal(g.cpu().numpy(), -ln[rows] * xn[K.colidx])
        ref = -float(np.dot(ln * mn, xn))
        assert abs(float(s.item()) - ref) <= 1e-12 * abs(ref) * np.sqrt(K.n)
        ctx.close()


def test_noalloc_rejects_bad_arguments():
    import torch
    from paper_1406_2831_amd import rbicgstab as rb
    rb.load_library()
    lib = rb.load_library()
    rc = lib.rbicgstab_adjoint_grads_noalloc(0, 0, None, None, None, None, None, None, None, None)
    assert rc == rb.RBS_ERR_ARG
    assert b"n < 2^31" in lib.rbicgstab_last_error(None)

"""GPU parity of the adjoint path (RBS_TRANSPOSE solves, gradient kernel,
torch.autograd.Function) against the CPU FP64 oracle and finite differences.

Tolerances: adjoint solutions versus the oracle / a direct solve within 1e-6
relative (solves at rtol 1e-10 or tighter, kappa * rtol <= 1e-6 on these
grids); the gradient kernel versus the oracle formula on the same inputs to
1e-13 relative (one product per entry, one reduction for dL/dsigma);
directional derivatives versus central differences (step 1e-6, solves at
rtol 1e-12) to 1e-4 of the typical (RMS over the directions) derivative: the
finite-difference noise is about kappa * rtol / step in absolute terms, so a
direction whose derivative happens to be small is not held to a relative bar.
"""
import sys

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle as o
import workloads as w

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def adj():
    from paper_1406_2831_amd import adjoint
    from paper_1406_2831_amd import rbicgstab as rbm
    rbm.load_library()
    return adjoint


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _t(torch_mod, a):
    return torch_mod.as_tensor(np.ascontiguousarray(a), dtype=torch_mod.float64, device="cuda")


def test_transpose_solve_exact_space_2d(adj, torch_mod):
    """A^T lambda = c with the swapped exact eigenvector space vs the oracle."""
    seq = w.seq_2d()
    sigma = float(seq.sigmas[1])
    A, At = seq.matrix(1)
    As, Ats = A.to_scipy(), At.to_scipy()
    ev, vl, vr = sla.eig(As.toarray(), left=True, right=True)
    order = np.argsort(np.abs(ev))
    U, Ut = vr[:, order[:8]].real.copy(), vl[:, order[:8]].real.copy()
    c = np.random.default_rng(21).standard_normal(seq.n)
    _say("transpose 2d exact space")
    sysm = adj.ShiftedSystem(seq.K, seq.mdiag, k_max=8, s_max=0)
    sysm.bind(None, sigma)
    sysm.ctx.recycle("set", _t(torch_mod, U.T), _t(torch_mod, Ut.T))
    lam, st = sysm.solve(_t(torch_mod, c), sigma, rtol=1e-10, transpose=True)
    lo, info = o.adjoint_solve(As, Ats, U, Ut, c, rtol=1e-12)
    assert info.status == o.OK and st.status == 0 and st.k_used == 8
    assert st.rel_res_true <= 1e-10
    assert _rel(lam.cpu().numpy(), lo) <= 1e-6
    # products with A^T are the solve's operator: counted in matvecs_At
    assert st.matvecs_At >= 2 * st.iters and st.matvecs_A >= 8
    # plain BiCGSTAB on A^T as well
    lam0, st0 = sysm.solve(_t(torch_mod, c), sigma, rtol=1e-10, transpose=True, mode="bicgstab")
    assert st0.status == 0 and _rel(lam0.cpu().numpy(), lo) <= 1e-6
    sysm.close()


def test_gradient_kernel_matches_formula(adj, torch_mod):
    seq = w.seq_3d(N=23, nshift=2, nrhs=1, k=8)
    sysm = adj.ShiftedSystem(seq.K, seq.mdiag, k_max=8, s_max=0)
    sysm.bind(None, float(seq.sigmas[0]))
    rng = np.random.default_rng(2)
    x, lam = rng.standard_normal(seq.n), rng.standard_normal(seq.n)
    _say("gradient kernel 23^3")
    gv, gs = sysm.grads(_t(torch_mod, lam), _t(torch_mod, x))
    _, gs_o, gv_o = o.gradients(seq.K.rowptr, seq.K.colidx, seq.mdiag, x, lam)
    assert np.max(np.abs(gv.cpu().numpy() - gv_o)) <= 1e-14 * np.max(np.abs(gv_o))
    assert abs(gs - gs_o) <= 1e-12 * np.sum(np.abs(lam * seq.mdiag * x))
    sysm.close()


def test_autograd_matches_oracle_gradient_2d(adj, torch_mod):
    """L = c^T x through RecycledSolve: gradients vs the oracle's (dense) ones."""
    seq = w.seq_2d()
    sigma0 = float(seq.sigmas[2])
    K = seq.K
    c = np.random.default_rng(31).standard_normal(seq.n)
    b = seq.rhs[0]
    _say("autograd 2d rbicg forward + transposed rbicgstab backward")
    sysm = adj.ShiftedSystem(K, seq.mdiag, k_max=8, s_max=256)
    bt = _t(torch_mod, b).requires_grad_(True)
    sg = torch_mod.tensor(sigma0, dtype=torch_mod.float64, device="cuda", requires_grad=True)
    kv = _t(torch_mod, K.val).requires_grad_(True)
    for mode in ("rbicg", "rbicgstab", "bicgstab"):
        for t in (bt, sg, kv):
            t.grad = None
        x = adj.recycled_solve(sysm, bt, sg, kv, 1e-11, 20000, mode)
        loss = (x * _t(torch_mod, c)).sum()
        loss.backward()
        A = K.to_scipy().toarray() + sigma0 * np.diag(seq.mdiag)
        xd = np.linalg.solve(A, b)
        ld = np.linalg.solve(A.T, c)
        g_b, g_s, g_v = o.gradients(K.rowptr, K.colidx, seq.mdiag, xd, ld)
        assert _rel(x.detach().cpu().numpy(), xd) <= 1e-6, mode
        assert _rel(bt.grad.cpu().numpy(), g_b) <= 1e-6, mode
        assert abs(sg.grad.item() - g_s) <= 1e-6 * abs(g_s), mode
        assert _rel(kv.grad.cpu().numpy(), g_v) <= 1e-6, mode
    assert sysm.ctx.blocks()[1] > 0   # the RBiCG forward installed a space
    sysm.close()


def test_ragged_3d_generated_space_adjoint(adj, torch_mod):
    """Forward RBiCG on a ragged grid builds (U, Ut); the transposed solve reuses it."""
    seq = w.seq_3d(N=23, nshift=1, nrhs=1, k=12)
    sigma = float(seq.sigmas[0])
    A, At = seq.matrix(0)
    c = np.random.default_rng(41).standard_normal(seq.n)
    _say("ragged 23^3 rbicg forward, transposed rbicgstab")
    sysm = adj.ShiftedSystem(seq.K, seq.mdiag, k_max=12, s_max=512)
    x, st = sysm.solve(_t(torch_mod, seq.rhs[0]), sigma, rtol=1e-10, mode="rbicg")
    sysm.ctx.recycle("from_last_solve")
    lam, stl = sysm.solve(_t(torch_mod, c), sigma, rtol=1e-10, transpose=True)
    lam_ref = spla.spsolve(At.to_scipy().tocsc(), c)
    x_ref = spla.spsolve(A.to_scipy().tocsc(), seq.rhs[0])
    print(f"forward iters {st.iters}, adjoint iters {stl.iters} k {stl.k_used}", flush=True)
    assert stl.k_used > 0 and stl.status == 0
    assert _rel(lam.cpu().numpy(), lam_ref) <= 1e-6
    assert _rel(x.cpu().numpy(), x_ref) <= 1e-6
    # the same adjoint by plain BiCGSTAB on A^T
    lam0, st0 = sysm.solve(_t(torch_mod, c), sigma, rtol=1e-10, transpose=True, mode="bicgstab")
    print(f"adjoint bicgstab iters {st0.iters}", flush=True)
    assert _rel(lam0.cpu().numpy(), lam_ref) <= 1e-6
    sysm.close()


def test_directional_derivatives_vs_central_differences(adj, torch_mod):
    """16 random directions in (b, sigma, K values), step 1e-6, solves at 1e-12."""
    N = 32
    seq, c, bdirs = w.adjoint_problem(N=N, ndirs=16)
    K, mdiag, sigma, b = seq.K, seq.mdiag, float(seq.sigmas[0]), seq.rhs[0]
    _say(f"finite differences {N}^3")
    sysm = adj.ShiftedSystem(K, mdiag, k_max=20, s_max=512)
    bt = _t(torch_mod, b).requires_grad_(True)
    sg = torch_mod.tensor(sigma, dtype=torch_mod.float64, device="cuda", requires_grad=True)
    kv = _t(torch_mod, K.val).requires_grad_(True)
    ct = _t(torch_mod, c)
    x = adj.recycled_solve(sysm, bt, sg, kv, 1e-12, 50000, "rbicg")
    (x * ct).sum().backward()
    gb, gs, gk = bt.grad.cpu().numpy(), sg.grad.item(), kv.grad.cpu().numpy()
    dirs = w.generator(3, 1, "dirs")
    h = 1e-6
    fds, ans = [], []
    for i in range(16):
        db = bdirs[i]
        ds = dirs.standard_normal()
        dk = dirs.standard_normal(K.nnz) * np.abs(K.val)
        vals = []
        for sgn in (1.0, -1.0):
            with torch_mod.no_grad():
                xp, _ = sysm.solve(_t(torch_mod, b + sgn * h * db), sigma + sgn * h * ds,
                                   _t(torch_mod, K.val + sgn * h * dk), rtol=1e-12, max_it=50000)
                vals.append(float((xp * ct).sum().item()))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = gb @ db + gs * ds + gk @ dk
        fds.append(fd)
        ans.append(an)
        print(f"dir {i}: fd {fd:.10e} adjoint {an:.10e} rel {abs(fd - an) / abs(an):.2e}", flush=True)
    fds, ans = np.array(fds), np.array(ans)
    scale = np.sqrt(np.mean(ans ** 2))
    worst = np.max(np.abs(fds - ans)) / scale
    print(f"max |fd - adjoint| / rms = {worst:.2e}", flush=True)
    assert worst <= 1e-4
    sysm.close()

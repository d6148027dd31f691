"""GPU parity at full sizes and at the large recycle dimensions.

* Algorithm 2 at the full 64^3 size with an exact recycle space: at sigma = 0
  the 7-point operator is a Kronecker sum of tridiagonal Toeplitz factors, so
  its left and right eigenvectors have a closed form
  (``workloads.separable_eigenpairs``); GPU and oracle run RBiCGSTAB on the
  same installed space and must take the same iterations to the same answer.
* RBiCG started from an installed space (the space-improving solve of
  Section 6.2) at 64^3, against the oracle's RBiCG on the same space.
* Recycle dimensions 30, 40 and 64 (buckets 32, 40 and 64 of the fused
  kernels) on the 27-point stencil, through the single-system, multi-RHS,
  batched and FP32-storage paths, with a well-conditioned space: U has
  orthonormal columns and Ut = A^-T A U, so Ct = C and the projector is
  orthogonal.
* The 128^3 adjoint configuration by properties the oracle can check one by
  one: FP64 true residuals of the forward and transposed solves, the
  sigma-gradient as a dot product, sampled entries of the value gradient.

Tolerances as in test_gpu_parity: solves at rtol 1e-10, solutions within
1e-6 relative (kappa * rtol <= 1e-6), iteration counts within a few percent.
"""
import sys

import numpy as np
import pytest
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
def rb():
    from paper_1406_2831_amd import rbicgstab as rbm
    rbm.load_library()
    return rbm


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _dev(torch_mod, a):
    return torch_mod.as_tensor(np.ascontiguousarray(a), dtype=torch_mod.float64, device="cuda")


def _context(rb, A, At, k_max, s_max=64, secant_max=float("inf")):
    from paper_1406_2831_amd.sequence import max_row_nnz
    ctx = rb.Context(A.n, max_row_nnz(A, At), k_max, s_max, secant_max=secant_max)
    ctx.setup(A, At)
    return ctx


def _install(ctx, torch_mod, U, Ut):
    ctx.recycle("set", _dev(torch_mod, U.T), _dev(torch_mod, Ut.T))


def _solve(ctx, torch_mod, b, sh, mode="rbicgstab", rtol=1e-10, precision="fp64"):
    bt = _dev(torch_mod, b)
    x = torch_mod.zeros_like(bt)
    _, st = ctx.solve(bt, x, shadow=None if sh is None else _dev(torch_mod, sh), rtol=rtol,
                      max_it=20000, mode=mode, precision=precision)
    return x.cpu().numpy(), st


@pytest.fixture(scope="module")
def exact64():
    """sigma = 0 operator at 64^3 and its 20 lowest eigenpairs in closed form."""
    dims = (64, 64, 64)
    K = w.convdiff(dims, w.VEL3, w.PECLET)
    Kt = K.transpose()
    lam, U, Ut = w.separable_eigenpairs(dims, w.VEL3, w.PECLET, 20)
    b = w.generator(1, 0, "b").standard_normal(K.n)
    sh = w.generator(1, 0, "shadow").standard_normal(K.n)
    return K, Kt, lam, U, Ut, b, sh


def test_closed_form_space_is_exact_at_full_size(exact64):
    """The installed space is an exact invariant pair of the 64^3 operator."""
    K, Kt, lam, U, Ut, _, _ = exact64
    As, Ats = K.to_scipy(), Kt.to_scipy()
    assert np.max(np.linalg.norm(As @ U - U * lam, axis=0) / lam) < 1e-12
    assert np.max(np.linalg.norm(Ats @ Ut - Ut * lam, axis=0) / lam) < 1e-12


def test_algorithm2_exact_space_full_size(rb, torch_mod, exact64):
    """RBiCGSTAB at 64^3 with the 20 exact eigenpairs installed: GPU and oracle on the
    same space take the same number of iterations to the same solution, and the
    deflation of the 20 smallest eigenvalues cuts iterations against BiCGSTAB."""
    K, Kt, lam, U, Ut, b, sh = exact64
    As, Ats = K.to_scipy(), Kt.to_scipy()
    _say("algorithm 2, 64^3, exact closed-form space k=20")
    ctx = _context(rb, K, Kt, 20, secant_max=0.0)   # the default cap keeps every exact pair
    _install(ctx, torch_mod, U, Ut)
    k = ctx.blocks()[1]
    assert k == 20
    x, st = _solve(ctx, torch_mod, b, sh)
    xb, stb = _solve(ctx, torch_mod, b, sh, mode="bicgstab")
    bl = o.make_blocks(As, Ats, U, Ut)
    assert bl.k == 20
    xo, io = o.rbicgstab(As, bl, b, shadow_m1=sh, rtol=1e-10)
    print(f"exact space 64^3: gpu iters {st.iters} oracle {io.iters}, gpu bicgstab {stb.iters}", flush=True)
    assert st.status == 0 and io.status == o.OK and st.k_used == 20
    assert np.linalg.norm(b - As @ x) / np.linalg.norm(b) <= 1e-10
    assert abs(st.iters - io.iters) <= max(2, 0.05 * io.iters)
    assert _rel(x, xo) <= 1e-6
    assert stb.status == 0 and _rel(xb, xo) <= 1e-6
    assert st.iters < stb.iters
    ctx.close()


def test_rbicg_from_installed_space_full_size(rb, torch_mod, exact64):
    """RBiCG (dual right-hand side of ones, both residuals to tolerance) started from
    an installed space at 64^3: the GPU's iteration count and solution are the
    oracle's; the space it builds drives a converging RBiCGSTAB solve."""
    K, Kt, lam, U, Ut, b, sh = exact64
    As, Ats = K.to_scipy(), Kt.to_scipy()
    _say("rbicg from an installed space, 64^3")
    ctx = _context(rb, K, Kt, 20, s_max=512, secant_max=0.0)
    # four exact pairs: with ten, the oracle's RBiCG stalls near 1e-8 and then
    # diverges (the BiCG recurrences of the projected pair lose their accuracy),
    # so rtol 1e-10 would test that instability rather than the kernels
    _install(ctx, torch_mod, U[:, :4], Ut[:, :4])
    x, st = _solve(ctx, torch_mod, b, None, mode="rbicg")
    bl = o.make_blocks(As, Ats, U[:, :4], Ut[:, :4])
    xo, xto, io = o.rbicg(As, Ats, bl, b, rtol=1e-10)
    print(f"rbicg 64^3 from k=4: gpu iters {st.iters} oracle {io.iters} "
          f"(dual residual {io.rel_res_dual:.2e})", flush=True)
    assert st.status == 0 and io.status == o.OK and st.k_used == 4
    assert io.rel_res_dual <= 1e-9
    assert abs(st.iters - io.iters) <= max(2, 0.05 * io.iters)
    assert np.linalg.norm(b - As @ x) / np.linalg.norm(b) <= 1e-10
    assert _rel(x, xo) <= 1e-6
    ctx.recycle("from_last_solve")
    knew = ctx.blocks()[1]
    assert knew > 0
    b2 = w.generator(1, 1, "b").standard_normal(K.n)
    x2, st2 = _solve(ctx, torch_mod, b2, sh)
    assert st2.status == 0 and np.linalg.norm(b2 - As @ x2) / np.linalg.norm(b2) <= 1e-10
    ctx.close()


@pytest.fixture(scope="module")
def stencil27():
    """27-point stencil at N = 24 (n = 13,824; several tiles and 216 slices), one
    shift, three right-hand sides, and a well-conditioned 64-column space."""
    seq = w.seq_3d27(N=24, nshift=1, nrhs=3, k=64)
    A, At = seq.matrix(0)
    As, Ats = A.to_scipy(), At.to_scipy()
    rng = w.generator(4, 0, "U")
    U, _ = np.linalg.qr(rng.standard_normal((A.n, 64)))
    lu = spla.splu(As.tocsc())
    Ut = lu.solve(As @ U, trans="T")   # A^T Ut = A U: Ct = C
    refs = [lu.solve(b) for b in seq.rhs]
    return seq, A, At, As, Ats, U, Ut, refs


@pytest.mark.parametrize("k", [30, 40, 64])
def test_large_recycle_dimension_single_and_fp32(rb, torch_mod, stencil27, k):
    """Buckets 32, 40, 64: single-system FP64 RBiCGSTAB vs the oracle and the direct
    solve; FP32 storage under FP64 refinement vs the direct solve."""
    seq, A, At, As, Ats, U, Ut, refs = stencil27
    _say(f"27-point N=24, k={k}: single FP64 and FP32-IR")
    ctx = _context(rb, A, At, 64)
    _install(ctx, torch_mod, U[:, :k], Ut[:, :k])
    assert ctx.blocks()[1] == k
    bl = o.make_blocks(As, Ats, U[:, :k], Ut[:, :k], secant_max=np.inf)
    assert bl.k == k
    b, sh = seq.rhs[0], seq.shadows[0]
    x, st = _solve(ctx, torch_mod, b, sh)
    xo, io = o.rbicgstab(As, bl, b, shadow_m1=sh, rtol=1e-10)
    print(f"k={k}: gpu iters {st.iters} oracle {io.iters}", flush=True)
    assert st.status == 0 and st.k_used == k and io.status == o.OK
    assert abs(st.iters - io.iters) <= max(2, 0.05 * io.iters)
    assert _rel(x, refs[0]) <= 1e-6 and _rel(x, xo) <= 1e-6
    x32, st32 = _solve(ctx, torch_mod, b, sh, precision="fp32_ir")
    print(f"k={k}: fp32-ir inner iters {st32.iters}, outer steps {st32.ir_steps}, "
          f"fallbacks {st32.restarts}", flush=True)
    assert st32.status == 0 and st32.rel_res_true <= 1e-10
    assert _rel(x32, refs[0]) <= 1e-6
    ctx.close()


@pytest.mark.parametrize("k", [20, 22, 30, 64])
def test_large_recycle_dimension_multi_rhs(rb, torch_mod, stencil27, k):
    """Three right-hand sides solved together at buckets 20, 24 (block columns read
    in the row's arithmetic part), 32 and 64 (64: the largest fused reduction,
    3 x 67 sums per workgroup) vs one-at-a-time solves."""
    seq, A, At, As, Ats, U, Ut, refs = stencil27
    _say(f"27-point N=24, k={k}: multi-RHS")
    ctx = _context(rb, A, At, 64)
    _install(ctx, torch_mod, U[:, :k], Ut[:, :k])
    Bm = np.stack(seq.rhs)
    Sm = np.stack(seq.shadows)
    X, sts = ctx.solve_multi(_dev(torch_mod, Bm), shadows=_dev(torch_mod, Sm), rtol=1e-10)
    Xn = X.cpu().numpy()
    for j in range(3):
        x1, st1 = _solve(ctx, torch_mod, seq.rhs[j], seq.shadows[j])
        print(f"k={k} rhs {j}: multi iters {sts[j].iters} single {st1.iters}", flush=True)
        assert sts[j].status == 0 and sts[j].rel_res_true <= 1e-10 and sts[j].k_used == k
        assert abs(sts[j].iters - st1.iters) <= max(3, 0.05 * st1.iters)
        assert _rel(Xn[j], refs[j]) <= 1e-6 and _rel(Xn[j], x1) <= 1e-6
    ctx.close()


def test_large_recycle_dimension_batched(rb, torch_mod, stencil27):
    """A batch of three systems with recycle dimensions 30, 40 and 64 (bucket 64 of the
    batched passes, systems of different k in one launch) vs the direct solves."""
    seq, A, At, As, Ats, U, Ut, refs = stencil27
    _say("27-point N=24: batched k = 30, 40, 64")
    ctxs = []
    for k in (30, 40, 64):
        ctx = _context(rb, A, At, 64)
        _install(ctx, torch_mod, U[:, :k], Ut[:, :k])
        ctxs.append(ctx)
    bs = [_dev(torch_mod, b) for b in seq.rhs]
    shs = [_dev(torch_mod, s) for s in seq.shadows]
    batch = rb.Batch(ctxs, tune=False, graph=False)
    xs = [torch_mod.zeros_like(b) for b in bs]
    sts = batch.solve(bs, xs, shs, rtol=1e-10)
    for j, (x, st) in enumerate(zip(xs, sts)):
        x1, st1 = _solve(ctxs[j], torch_mod, seq.rhs[j], seq.shadows[j])
        print(f"batched system {j} (k={st.k_used}): iters {st.iters} alone {st1.iters}", flush=True)
        assert st.status == 0 and st.rel_res_true <= 1e-10
        assert abs(st.iters - st1.iters) <= max(3, 0.05 * st1.iters)
        assert _rel(x.cpu().numpy(), refs[j]) <= 1e-6
    # FP32 storage under FP64 refinement, batched
    xs = [torch_mod.zeros_like(b) for b in bs]
    sts = batch.solve(bs, xs, shs, rtol=1e-10, precision="fp32_ir")
    for j, (x, st) in enumerate(zip(xs, sts)):
        print(f"batched fp32-ir system {j}: inner iters {st.iters}, outer {st.ir_steps}", flush=True)
        assert st.status == 0 and st.rel_res_true <= 1e-10 and st.ir_steps >= 2
        assert _rel(x.cpu().numpy(), refs[j]) <= 1e-6
    batch.close()
    for c in ctxs:
        c.close()


def test_adjoint_full_size_128(rb, torch_mod):
    """The 128^3 adjoint configuration (n = 2,097,152): forward RBiCG building the space,
    then the forward RBiCGSTAB solve and the transposed solve reusing the space
    swapped, checked by properties computed on the host in FP64."""
    from paper_1406_2831_amd.sequence import max_row_nnz
    seq, c, _ = w.adjoint_problem(N=128, ndirs=1)
    A, At = seq.matrix(0)
    As, Ats = A.to_scipy(), At.to_scipy()
    b, sh = seq.rhs[0], seq.shadows[0]
    _say("adjoint 128^3: rbicg, rbicgstab, transposed rbicgstab, gradients")
    ctx = rb.Context(A.n, max_row_nnz(A, At), 20, 512)
    ctx.setup(A, At)
    _, st0 = _solve(ctx, torch_mod, b, sh, mode="rbicg", rtol=1e-10)
    assert st0.status == 0
    ctx.recycle("from_last_solve")
    k = ctx.blocks()[1]
    bt = _dev(torch_mod, b)
    x = torch_mod.zeros_like(bt)
    _, st = ctx.solve(bt, x, shadow=_dev(torch_mod, sh), rtol=1e-10, max_it=20000)
    ct = _dev(torch_mod, c)
    lam = torch_mod.zeros_like(ct)
    _, stl = ctx.solve(ct, lam, rtol=1e-10, max_it=20000, transpose=True)
    print(f"128^3: k={k}, forward iters {st.iters}, adjoint iters {stl.iters}", flush=True)
    assert st.status == 0 and stl.status == 0 and st.k_used == k and stl.k_used == k
    xn, ln = x.cpu().numpy(), lam.cpu().numpy()
    assert np.linalg.norm(b - As @ xn) / np.linalg.norm(b) <= 1e-10
    assert np.linalg.norm(c - Ats @ ln) / np.linalg.norm(c) <= 1e-10
    rowptr = torch_mod.as_tensor(A.rowptr, dtype=torch_mod.int32, device="cuda")
    colidx = torch_mod.as_tensor(A.colidx, dtype=torch_mod.int32, device="cuda")
    gval, gsig = ctx.adjoint_grads(rowptr, colidx, lam, x, _dev(torch_mod, seq.mdiag))
    ref_sig = -float(np.dot(ln * seq.mdiag, xn))
    assert abs(gsig - ref_sig) <= 1e-10 * abs(ref_sig)
    idx = w.generator(3, 1, "dirs").integers(0, A.nnz, size=4096)
    rows = np.searchsorted(A.rowptr, idx, side="right") - 1
    g = gval.cpu().numpy()[idx]
    assert np.array_equal(g, -ln[rows] * xn[A.colidx[idx]])
    ctx.close()

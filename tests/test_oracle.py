"""Pins of the CPU oracle against things other than itself.

Each test ties an oracle function to a fact fixed by the mathematics or by
an independent implementation: SciPy's BiCGSTAB, dense LU, the projector
identities of Section 3 (eq. CcheckChat, Theorem 2, eq. minusXR), the
polynomial argument of Section 4 (RBiCGSTAB is BiCGSTAB applied to
``B = (I - C Chat^T) A``), deflation of exact eigenvectors, closed forms.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle as o
import workloads as w


@pytest.fixture(scope="module")
def c0():
    seq = w.seq_2d()
    A, At = seq.matrix(1)
    return seq, A.to_scipy(), At.to_scipy()


@pytest.fixture(scope="module")
def eig_c0(c0):
    _, A, _ = c0
    lam, vl, vr = sla.eig(A.toarray(), left=True, right=True)
    order = np.argsort(np.abs(lam))
    return lam[order], vl[:, order].real, vr[:, order].real


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# --------------------------------------------------------------------------- inputs

def test_workload_sizes():
    s = w.seq_2d()
    assert (s.n, s.K.nnz) == (1024, 4992)
    K = w.convdiff((64, 64, 64), w.VEL3, w.PECLET)
    assert (K.n, K.nnz) == (262144, 1810432)
    K27 = w.convdiff27(12, w.VEL3, w.PECLET)
    assert K27.nnz == (3 * 12 - 2) ** 3
    Kt = K27.transpose()
    assert abs(Kt.to_scipy() - K27.to_scipy().T).max() == 0.0


def test_workload_operator_closed_form():
    """1D factor eigenvalues: tridiagonal Toeplitz closed form a + 2 sqrt(bc) cos(j pi h)."""
    N, c = 20, 7.0
    h = 1.0 / (N + 1)
    K = w.convdiff((N, 1), (c / w.PECLET, 0.0), w.PECLET).to_scipy().toarray()
    # with a single point on y the y-factor adds 2/h_y^2 = 8 (h_y = 1/2)
    a, lo, up = 2 / h**2 + c / h, -1 / h**2 - c / h, -1 / h**2
    j = np.arange(1, N + 1)
    ref = np.sort(a + 2 * np.sqrt(lo * up) * np.cos(j * np.pi * h) + 8.0)
    got = np.sort(np.linalg.eigvals(K).real)
    assert np.allclose(got, ref, rtol=1e-10)


# --------------------------------------------------------------------------- BiCGSTAB

def test_bicgstab_iterates_match_scipy(c0):
    seq, A, _ = c0
    b = seq.rhs[1]
    xs = []
    spla.bicgstab(A, b, rtol=1e-14, maxiter=30, callback=lambda xk: xs.append(xk.copy()))
    _, info = o.bicgstab(A, b, rtol=1e-14, max_it=30, max_restarts=0, record=True)
    assert len(xs) == 30 and len(info.trace["x"]) == 30
    for i in range(30):
        assert _rel(info.trace["x"][i], xs[i]) < 1e-9, i


def test_bicgstab_dense_lu(c0):
    seq, A, _ = c0
    b = seq.rhs[1]
    x, info = o.bicgstab(A, b, shadow=seq.shadows[1], rtol=1e-12)
    xd = np.linalg.solve(A.toarray(), b)
    kappa = np.linalg.cond(A.toarray())
    assert info.status == o.OK
    assert _rel(x, xd) < kappa * 1e-12 * 10
    assert info.rel_res_true <= 1e-12


# --------------------------------------------------------------------------- RBiCGSTAB

def test_rbicgstab_k0_is_bicgstab(c0):
    """Algorithm 2 with an empty recycle space is van der Vorst's BiCGSTAB, step for step."""
    seq, A, _ = c0
    b, sh = seq.rhs[1], seq.shadows[1]
    _, i0 = o.bicgstab(A, b, shadow=sh, rtol=1e-10)
    _, i1 = o.rbicgstab(A, o.empty_blocks(A.shape[0]), b, shadow_m1=sh, rtol=1e-10)
    h0, h1 = np.array(i0.res_hist[:20]), np.array(i1.res_hist[:20])
    assert np.max(np.abs(h0 - h1) / h0) < 1e-8
    assert abs(i0.iters - i1.iters) <= 1


def _random_blocks(A, At, k, seed):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((A.shape[0], k))
    Ut = rng.standard_normal((A.shape[0], k))
    return o.make_blocks(A, At, U, Ut, secant_max=np.inf)


def test_rbicgstab_is_bicgstab_on_projected_operator(c0, eig_c0):
    """Section 4: RBiCGSTAB's residuals are BiCGSTAB's for B = (I - C Chat^T) A from r_0, shadow rt_0."""
    seq, A, At = c0
    lam, vl, vr = eig_c0
    # exact eigenvector spaces keep the projector well posed (perturbed spaces make B so
    # non-normal that rounding alone separates the two histories after a few steps)
    bl = o.make_blocks(A, At, vr[:, :6], vl[:, :6], secant_max=np.inf)
    assert bl.k == 6
    b, sh = seq.rhs[1], seq.shadows[1]
    _, info = o.rbicgstab(A, bl, b, shadow_m1=sh, rtol=1e-10, record=True)
    r0, rt0 = info.trace["r0"], info.trace["rt0"]
    B = A.toarray() - bl.C @ (bl.Chat.T @ A.toarray())
    _, ib = o.bicgstab(B, r0, shadow=rt0, rtol=1e-10, max_restarts=0)
    hr = np.array(info.res_hist[:25]) * np.linalg.norm(b)
    hb = np.array(ib.res_hist[:25]) * np.linalg.norm(r0)
    assert np.max(np.abs(hr - hb) / hb) < 1e-9


def test_rbicgstab_invariants(c0, eig_c0):
    seq, A, At = c0
    lam, vl, vr = eig_c0
    bl = o.make_blocks(A, At, vr[:, :8], vl[:, :8], secant_max=np.inf)
    b, sh = seq.rhs[1], seq.shadows[1]
    x, info = o.rbicgstab(A, bl, b, shadow_m1=sh, rtol=1e-10, record=True)
    k = bl.k
    tr = info.trace
    # eq. (CcheckChat): Chat^T C = I and Ccheck^T Ct = I; D_c = Ct^T C = I after bi-orthogonalisation
    assert np.abs(bl.Chat.T @ bl.C - np.eye(k)).max() < 1e-10
    assert np.abs(bl.Ccheck.T @ bl.Ct - np.eye(k)).max() < 1e-10
    assert np.abs(bl.Ct.T @ bl.C - np.eye(k)).max() < 1e-8
    # eq. (minusXR): rt_0 orthogonal to C; Theorem 2: Ct^T B x = 0 for r, s, q
    assert np.abs(bl.C.T @ tr["rt0"]).max() < 1e-10 * np.linalg.norm(bl.C) * np.linalg.norm(tr["rt0"])
    scale = np.linalg.norm(bl.Ct, axis=0)
    for key in ("r", "s", "q"):
        for v in tr[key][:20]:
            assert np.max(np.abs(bl.Ct.T @ v) / scale) < 1e-8 * np.linalg.norm(b)
    # the recurrence residual is the true residual of x_i - U x_c (C = A U)
    for xi, xci, ri in list(zip(tr["x"], tr["xc"], tr["r"]))[:20]:
        true = b - A @ (xi - bl.U @ xci)
        assert np.linalg.norm(true - ri) < 1e-9 * np.linalg.norm(b)
    assert info.status == o.OK and info.rel_res_true <= 1e-10


def test_rbicgstab_dense_lu(c0, eig_c0):
    seq, A, At = c0
    lam, vl, vr = eig_c0
    bl = o.make_blocks(A, At, vr[:, :8], vl[:, :8])
    b, sh = seq.rhs[1], seq.shadows[1]
    x, info = o.rbicgstab(A, bl, b, shadow_m1=sh, rtol=1e-12)
    xd = np.linalg.solve(A.toarray(), b)
    kappa = np.linalg.cond(A.toarray())
    assert info.status == o.OK
    assert _rel(x, xd) < kappa * 1e-12 * 10


def test_exact_eigenvectors_deflate(c0, eig_c0):
    """Recycling exact left/right eigenvectors removes their eigenvalues from B's spectrum."""
    seq, A, At = c0
    lam, vl, vr = eig_c0
    k = 8
    bl = o.make_blocks(A, At, vr[:, :k], vl[:, :k], secant_max=np.inf)
    Ad = A.toarray()
    B = Ad - bl.C @ (bl.Chat.T @ Ad)
    mu = np.linalg.eigvals(B)
    mu = mu[np.argsort(np.abs(mu))]
    assert np.all(np.abs(mu[:k]) < 1e-8 * np.abs(lam).max())
    rest = np.sort_complex(mu[k:])
    ref = np.sort_complex(lam[k:])
    assert np.max(np.abs(rest - ref) / np.abs(ref)) < 1e-8
    _, i0 = o.bicgstab(A, seq.rhs[1], shadow=seq.shadows[1], rtol=1e-10)
    _, i1 = o.rbicgstab(A, bl, seq.rhs[1], shadow_m1=seq.shadows[1], rtol=1e-10)
    assert i1.iters < i0.iters


def test_rhs_in_range_of_C(c0):
    """b = C y gives r_0 = 0: no iteration and x = U Chat^T b exactly (eq. minusXR)."""
    seq, A, At = c0
    bl = _random_blocks(A, At, 5, 7)
    b = bl.C @ np.arange(1.0, 6.0)
    x, info = o.rbicgstab(A, bl, b, rtol=1e-10)
    assert info.status == o.OK and info.iters == 0
    assert np.linalg.norm(A @ x - b) < 1e-10 * np.linalg.norm(b)


def test_failure_paths(c0):
    seq, A, At = c0
    b = seq.rhs[1]
    n = A.shape[0]
    # disjoint supports make (r_0, rt_0) exactly zero in floating point
    bz = b.copy()
    bz[n // 2:] = 0.0
    sh = seq.shadows[1].copy()
    sh[: n // 2] = 0.0
    _, info = o.rbicgstab(A, o.empty_blocks(n), bz, shadow_m1=sh)
    assert info.status == o.BREAKDOWN_RHO
    _, info = o.rbicgstab(A, o.empty_blocks(n), b, max_it=1, max_restarts=0)
    assert info.status == o.MAXIT and info.iters == 1
    bad = b.copy()
    bad[3] = np.nan
    _, info = o.rbicgstab(A, o.empty_blocks(n), bad)
    assert info.status == o.NONFINITE
    # skew-symmetric operator: (s, A s) = 0 so omega = 0
    R = np.array([[0.0, 1.0], [-1.0, 0.0]])
    _, info = o.bicgstab(R, np.array([1.0, 0.0]), shadow=np.array([1.0, 1.0]), max_restarts=0)
    assert info.status == o.BREAKDOWN_OMEGA


# --------------------------------------------------------------------------- RBiCG

def test_bicg_biorthogonality_and_solution(c0):
    """Algorithm 1 with an empty space is BiCG: (rt_j, r_i) = 0 for j != i, x = A^-1 b."""
    seq, A, At = c0
    b = seq.rhs[1]
    x, xt, info = o.rbicg(A, At, o.empty_blocks(A.shape[0]), b, rtol=1e-12, record=True)
    R = np.array(info.trace["r"][:8]).T
    Rt = np.array(info.trace["rt"][:8]).T
    Gm = Rt.T @ R
    off = Gm - np.diag(np.diag(Gm))
    norms = np.outer(np.linalg.norm(Rt, axis=0), np.linalg.norm(R, axis=0))
    assert np.max(np.abs(off) / norms) < 1e-8
    xd = np.linalg.solve(A.toarray(), b)
    assert info.status == o.OK
    assert _rel(x, xd) < np.linalg.cond(A.toarray()) * 1e-12 * 10
    # dual system: A^T xt = ones
    assert np.linalg.norm(At @ xt - np.ones(A.shape[0])) < 1e-6 * np.sqrt(A.shape[0])


def test_rbicg_projected_orthogonality(c0, eig_c0):
    """eq. (CVBiOrth): Ct^T V = 0 and C^T Vt = 0 for the recycled Lanczos vectors."""
    seq, A, At = c0
    lam, vl, vr = eig_c0
    bl = o.make_blocks(A, At, vr[:, :8], vl[:, :8], secant_max=np.inf)
    b = seq.rhs[1]
    x, xt, info = o.rbicg(A, At, bl, b, rtol=1e-12, record=True)
    for r, rt in list(zip(info.trace["r"], info.trace["rt"]))[:25]:
        assert np.max(np.abs(bl.Ct.T @ r)) < 1e-8 * np.linalg.norm(r) * np.linalg.norm(bl.Ct)
        assert np.max(np.abs(bl.C.T @ rt)) < 1e-8 * np.linalg.norm(rt) * np.linalg.norm(bl.C)
    xd = np.linalg.solve(A.toarray(), b)
    assert info.status == o.OK
    assert _rel(x, xd) < np.linalg.cond(A.toarray()) * 1e-12 * 10


def test_rbicg_dual_solution_with_recycle_space(c0, eig_c0):
    """RBiCG solves the dual system A^T xt = bt too (Section 3): with a recycle
    space the dual iterate is corrected by the accumulated Ut component, and the
    solve stops only when both residuals meet the tolerance."""
    seq, A, At = c0
    # an inexact space: with exact eigenvectors the dual coefficients vanish
    # identically (A Ccheck is a multiple of C, and C^T pt = 0), so the
    # correction would go untested
    lam, vl, vr = eig_c0
    rng = np.random.default_rng(21)
    U = vr[:, :6] + 1e-3 * rng.standard_normal((A.shape[0], 6))
    Ut = vl[:, :6] + 1e-3 * rng.standard_normal((A.shape[0], 6))
    bl = o.make_blocks(A, At, U, Ut, secant_max=np.inf)
    assert bl.k == 6
    n = A.shape[0]
    b = seq.rhs[1]
    bt = np.ones(n)
    rtol = 1e-8
    x, xt, info = o.rbicg(A, At, bl, b, rtol=rtol)
    assert info.status == o.OK
    Ad = A.toarray()
    kappa = np.linalg.cond(Ad)
    xd = np.linalg.solve(Ad, b)
    xtd = np.linalg.solve(Ad.T, bt)
    assert _rel(x, xd) < kappa * rtol * 10
    assert _rel(xt, xtd) < kappa * rtol * 10
    assert np.linalg.norm(bt - At @ xt) <= 10 * rtol * np.linalg.norm(bt)
    assert info.rel_res_dual <= 10 * rtol


def test_rbicg_stops_on_both_residuals(c0):
    """The stopping rule of RBiCG in Section 3 asks for both residuals; stopping on the
    primary one alone (an option) leaves the dual residual above the tolerance."""
    seq, A, At = c0
    n = A.shape[0]
    b = seq.rhs[1]
    rng = np.random.default_rng(3)
    bt = rng.standard_normal(n) * np.exp(np.linspace(-3.0, 3.0, n))   # a harder dual system
    _, xt_b, ib = o.rbicg(A, At, o.empty_blocks(n), b, bt=bt, rtol=1e-8, stop="both")
    _, xt_p, ip = o.rbicg(A, At, o.empty_blocks(n), b, bt=bt, rtol=1e-8, stop="primary")
    assert ib.status == o.OK and ip.status == o.OK
    assert ib.rel_res_dual <= 1e-8 * 1.5
    assert ib.rel_res_true <= 1e-8 and ip.rel_res_true <= 1e-8
    assert ip.iters <= ib.iters
    dual_recur = lambda xt: np.linalg.norm(bt - At @ xt) / np.linalg.norm(bt)
    if ip.iters < ib.iters:
        assert dual_recur(xt_p) > 1e-8


def test_rbicg_cycles_cover_all_lanczos_vectors(c0):
    seq, A, At = c0
    got = []
    x, xt, info = o.rbicg(A, At, o.empty_blocks(A.shape[0]), seq.rhs[1], s=10,
                          on_cycle=lambda V, Vt: got.append(V.shape[1]))
    assert sum(got) == info.iters and all(g == 10 for g in got[:-1])


# --------------------------------------------------------------------------- recycle space

def test_make_blocks_biorthogonal_and_secant_cap(c0):
    seq, A, At = c0
    rng = np.random.default_rng(5)
    n = A.shape[0]
    U = rng.standard_normal((n, 4))
    Ut = rng.standard_normal((n, 4))
    bl = o.make_blocks(A, At, U, Ut, secant_max=np.inf)
    assert np.abs(bl.Ct.T @ bl.C - np.eye(4)).max() < 1e-10
    # the pair's secant ||c|| ||ct|| / (ct^T c) is the norm of its rank-one projector
    sec = np.linalg.norm(bl.C, axis=0) * np.linalg.norm(bl.Ct, axis=0)
    proj_norm = [np.linalg.norm(np.outer(bl.C[:, j], bl.Ct[:, j]), 2) for j in range(4)]
    assert np.allclose(sorted(sec), sorted(proj_norm), rtol=1e-10)
    capped = o.make_blocks(A, At, U, Ut, secant_max=np.median(sec))
    assert 0 < capped.k < 4


def test_two_sided_ritz_recovers_planted_pairs(c0, eig_c0):
    """W containing exact right eigenvectors and Wt the matching left ones: exact Ritz values."""
    seq, A, At = c0
    lam, vl, vr = eig_c0
    k = 5
    rng = np.random.default_rng(9)
    # padding vectors drawn from the span of large-|lambda| eigenvectors keep the pencil
    # block-triangular, so the planted eigenvalues are the smallest ones it has
    pad = vr[:, -40:] @ rng.standard_normal((40, 6))
    padt = vl[:, -40:] @ rng.standard_normal((40, 6))
    W = np.hstack([vr[:, :k], pad])
    Wt = np.hstack([vl[:, :k], padt])
    U, Ut, vals, m = o.two_sided_ritz(A, W, Wt, k)
    assert np.allclose(np.sort(vals.real), np.sort(lam[:k].real), rtol=1e-9)
    # the returned spaces are the planted ones, on both sides
    cosines = sla.svdvals(sla.orth(U).T @ sla.orth(vr[:, :k]))
    assert cosines.min() > 1 - 1e-9
    cosines_left = sla.svdvals(sla.orth(Ut).T @ sla.orth(vl[:, :k]))
    assert cosines_left.min() > 1 - 1e-9
    # and vector by vector: the j-th left vector belongs to the j-th value
    for j in range(k):
        i = int(np.argmin(np.abs(lam[:k] - vals[j])))
        c = abs(Ut[:, j] @ vl[:, i]) / (np.linalg.norm(Ut[:, j]) * np.linalg.norm(vl[:, i]))
        assert c > 1 - 1e-9, j
    # a left eigenvector satisfies u^T A = theta u^T
    res = np.linalg.norm(At @ Ut - Ut * vals.real, axis=0) / np.abs(vals)
    assert res.max() < 1e-8


def test_ritz_select_pairs():
    th = np.array([5.0, 1 + 2j, 1 - 2j, 3.0, np.inf])
    # |1 +- 2i| < 3 < 5: the pair takes two slots, the infinite value is never chosen
    assert o.recycle.ritz_select(th, 3) == [(2, True), (3, False)]
    assert o.recycle.ritz_select(th, 4) == [(2, True), (3, False), (0, False)]
    assert o.recycle.ritz_select(th, 9) == [(2, True), (3, False), (0, False)]
    # the k-th slot would split the pair: keep k - 1
    assert o.recycle.ritz_select(np.array([3.0, 4 + 1j, 4 - 1j]), 2) == [(0, False)]


# --------------------------------------------------------------------------- sequence

def test_sequence_2d_converges():
    seq = w.seq_2d()
    res = o.run_sequence(seq, mode="rbicgstab")
    assert all(s == o.OK for s in res.status)
    assert max(res.rel_res_true) <= 1e-8
    assert res.solver == ["rbicg"] * 4
    for idx, x in enumerate(res.x):
        A, _ = seq.matrix(seq.system(idx)[0])
        xd = np.linalg.solve(A.to_scipy().toarray(), seq.rhs[idx])
        assert _rel(x, xd) < 1e-5


def test_harmonic_ritz_recovers_planted_vectors(c0, eig_c0):
    """Exact eigenvectors in W give exact harmonic Ritz pairs (residual orthogonal to A W is zero)."""
    seq, A, At = c0
    lam, vl, vr = eig_c0
    rng = np.random.default_rng(4)
    pad = vr[:, -40:] @ rng.standard_normal((40, 6))
    W = np.hstack([vr[:, :5], pad])
    U, vals = o.harmonic_ritz(A, W, 5)
    assert np.allclose(np.sort(vals.real), np.sort(lam[:5].real), rtol=1e-9)
    cosines = sla.svdvals(sla.orth(U).T @ sla.orth(vr[:, :5]))
    assert cosines.min() > 1 - 1e-9
    # a right eigenvector's harmonic residual is zero: ||A u - theta u|| ~ 0
    res = np.linalg.norm(A @ U - U * vals.real, axis=0) / np.abs(vals)
    assert res.max() < 1e-8


def test_recycle_space_reduces_iterations_3d():
    """Sequence-level property of the update (Section 6.2): RBiCGSTAB with the space
    from one RBiCG solve needs fewer iterations than BiCGSTAB on the other rhs."""
    seq = w.seq_3d(N=16, nshift=1, nrhs=3, k=12)
    res = o.run_sequence(seq, mode="rbicgstab", rtol=1e-8)
    base = o.run_sequence(seq, mode="bicgstab", rtol=1e-8)
    assert all(s == o.OK for s in res.status)
    assert res.k_used[1] >= 8
    assert sum(res.iters[1:]) < sum(base.iters[1:])

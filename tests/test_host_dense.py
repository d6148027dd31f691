"""CPU checks of the library's host-side dense algebra (LU, SVD, pivoted
Cholesky, Hessenberg + Francis QR eigenvalues, recycle-space Ritz step),
built with g++ from the library's own source into a throwaway shim."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as o
import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1406_2831_amd", "csrc")


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("shim") / "libdense_shim.so")
    cmd = [gxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-I", CSRC,
           os.path.join(ROOT, "tests", "dense_shim.cpp"), os.path.join(CSRC, "dense.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    lib = ctypes.CDLL(out)
    P = ctypes.POINTER(ctypes.c_double)
    lib.shim_lu_solve.argtypes = [ctypes.c_int, P, P, ctypes.c_int]
    lib.shim_svd.argtypes = [ctypes.c_int, P, P, P, P]
    lib.shim_eig.argtypes = [ctypes.c_int, P, P, P]
    lib.shim_pivoted_cholesky.argtypes = [ctypes.c_int, P, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_int), P]
    lib.shim_orth_factor.argtypes = [ctypes.c_int, P, ctypes.c_double, P]
    lib.shim_orth_factor_chol.argtypes = [ctypes.c_int, P, ctypes.c_double, P]
    lib.shim_recycle_ritz_orth.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, ctypes.c_int, P, P]
    lib.shim_left_coefficients_early.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_int), P]
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fortran(a):
    return np.asfortranarray(a, dtype=np.float64)


def test_lu_solve(shim):
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 30))
    b = rng.standard_normal(30)
    for trans in (0, 1):
        x = b.copy()
        assert shim.shim_lu_solve(30, _p(_fortran(A).ravel(order="F")), _p(x), trans) == 0
        ref = np.linalg.solve(A.T if trans else A, b)
        assert np.allclose(x, ref, rtol=1e-10, atol=1e-12)


def test_svd(shim):
    rng = np.random.default_rng(2)
    M = rng.standard_normal((12, 12))
    Mf = _fortran(M).ravel(order="F")
    P, s, Q = np.zeros(144), np.zeros(12), np.zeros(144)
    shim.shim_svd(12, _p(Mf), _p(P), _p(s), _p(Q))
    P, Q = P.reshape(12, 12, order="F"), Q.reshape(12, 12, order="F")
    assert np.allclose(s, np.linalg.svd(M, compute_uv=False), rtol=1e-12)
    assert np.allclose(P @ np.diag(s) @ Q.T, M, atol=1e-12)
    assert np.allclose(P.T @ P, np.eye(12), atol=1e-12)


def test_pivoted_cholesky_rank(shim):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((50, 6))
    X = np.hstack([X, X[:, :2] @ rng.standard_normal((2, 3))])   # rank 6, 9 columns
    G = _fortran(X.T @ X).ravel(order="F")
    perm = (ctypes.c_int * 9)()
    R = np.zeros(81)
    r = shim.shim_pivoted_cholesky(9, _p(G), 1e-12, perm, _p(R))
    assert r == 6
    Rm = R[: r * r].reshape(r, r, order="F")
    cols = list(perm)[:r]
    assert np.allclose(Rm.T @ Rm, (X.T @ X)[np.ix_(cols, cols)], rtol=1e-10)


@pytest.mark.parametrize("n,seed", [(5, 0), (40, 1), (120, 2)])
def test_eigenvalues_match_lapack(shim, n, seed):
    rng = np.random.default_rng(seed)
    H = rng.standard_normal((n, n))
    wr, wi = np.zeros(n), np.zeros(n)
    assert shim.shim_eig(n, _p(_fortran(H).ravel(order="F")), _p(wr), _p(wi)) == 0
    got = np.sort_complex(wr + 1j * wi)
    ref = np.sort_complex(np.linalg.eigvals(H))
    assert np.max(np.abs(got - ref)) < 1e-9 * np.abs(ref).max()


def _orth(shim, X, AX=None):
    """The library's orthonormalisation applied the way the API does: shifted
    Cholesky QR (shift 11 (n m + m (m+1)) u m on the column-scaled Gram
    matrix), then an unshifted pass; pivoted truncated Cholesky as fallback."""
    n = X.shape[0]
    for p in range(2):
        m = X.shape[1]
        G = _fortran(X.T @ X).ravel(order="F")
        S = np.zeros(m * m)
        shift = 11.0 * (n * m + m * (m + 1)) * np.finfo(float).eps * m if p == 0 else 0.0
        r = shim.shim_orth_factor_chol(m, _p(G), shift, _p(S))
        if r < 0:
            r = shim.shim_orth_factor(m, _p(G), 1e-12 if p == 0 else 1e-14, _p(S))
        Sm = S[: m * r].reshape(m, r, order="F")
        X = X @ Sm
        if AX is not None:
            AX = AX @ Sm
    return X, AX


def test_orth_factor_orthonormalises(shim):
    rng = np.random.default_rng(7)
    # column norms over ten orders of magnitude, like raw residual vectors
    X = rng.standard_normal((400, 30)) @ np.diag(np.logspace(0, -10, 30))
    S = np.zeros(30 * 30)
    G = _fortran(X.T @ X).ravel(order="F")
    r = shim.shim_orth_factor(30, _p(G), 1e-12, _p(S))   # the pivoted fallback
    Q = X @ S[: 30 * r].reshape(30, r, order="F")
    assert r == 30 and np.abs(Q.T @ Q - np.eye(30)).max() < 1e-8
    Q, _ = _orth(shim, X)
    assert Q.shape[1] == 30
    assert np.abs(Q.T @ Q - np.eye(30)).max() < 1e-12
    assert sla.subspace_angles(Q, X).max() < 1e-8


def test_shifted_cholesky_qr_keeps_ill_conditioned_directions(shim):
    """A Krylov-like basis with cond > 1e10: the shifted pass keeps every
    direction (each column of X lies in range(Q) to rounding) where the
    pivoted truncated factor drops some; a zero column is left out.  Two
    passes leave Q only roughly orthonormal at this conditioning, which the
    Ritz step does not need (its pencils do not depend on the basis)."""
    rng = np.random.default_rng(9)
    n, m = 3000, 60
    d = np.linspace(1.0, 2.0, n)
    X = np.empty((n, m))
    v = rng.standard_normal(n)
    for j in range(m):   # power-like sequence with a little noise: nearly dependent columns
        v = d * v
        v /= np.linalg.norm(v)
        X[:, j] = v + 1e-12 * rng.standard_normal(n)
    X[:, 17] = 0.0
    cond = np.linalg.cond(np.delete(X, 17, axis=1))
    assert cond > 1e10
    Q, _ = _orth(shim, X)
    assert Q.shape[1] == m - 1
    assert np.abs(Q.T @ Q - np.eye(m - 1)).max() < 1e-2
    assert np.linalg.cond(Q) < 1.1
    Qo, _ = np.linalg.qr(Q)
    assert np.linalg.norm(X - Qo @ (Qo.T @ X)) < 1e-12 * np.linalg.norm(X)
    S = np.zeros(m * m)
    G = _fortran(X.T @ X).ravel(order="F")
    assert shim.shim_orth_factor(m, _p(G), 1e-12, _p(S)) < m - 1


def _ritz_inputs(shim):
    """The reduced pencils of one RBiCG cycle of a small convection-diffusion
    system, in the library's orthonormal coordinates."""
    seq = w.seq_3d(N=12, nshift=1, nrhs=1, k=10)
    A, At = (m.to_scipy() for m in seq.matrix(0))
    n = A.shape[0]
    st = {}

    def cyc(V, Vt):
        st["V"], st["Vt"] = V, Vt

    o.rbicg(A, At, o.empty_blocks(n), seq.rhs[0], rtol=1e-10, s=100000, on_cycle=cyc)
    W, Wt = st["V"], st["Vt"]
    scale = np.logspace(0, -9, W.shape[1])
    W, Wt = W * scale, Wt * scale[::-1]
    Q, AQ = _orth(shim, W, A @ W)
    Qt, _ = _orth(shim, Wt)
    F = _fortran(Qt.T @ Q).ravel(order="F")
    G = _fortran(Qt.T @ AQ).ravel(order="F")
    F2 = _fortran(Q.T @ AQ).ravel(order="F")
    G2 = _fortran(AQ.T @ AQ).ravel(order="F")
    return Q.shape[1], Qt.shape[1], F, G, F2, G2


def test_left_coefficients_formed_early_match(shim):
    """The left space's transform is launched before the harmonic pencil is done,
    with as many columns as the two-sided pencil gave: its leading columns must be
    exactly the combined result's (unit columns, built column by column)."""
    r, rt, F, G, F2, G2 = _ritz_inputs(shim)
    for k in (4, 10):
        kl = ctypes.c_int(0)
        diff = np.zeros(1)
        kout = shim.shim_left_coefficients_early(r, rt, _p(F), _p(G), _p(G2), _p(F2), k,
                                                 ctypes.byref(kl), _p(diff))
        assert 0 < kout <= kl.value
        assert diff[0] == 0.0


def test_recycle_ritz_vs_oracle(shim):
    """Orthonormalise + reduced Ritz (the library's path) reproduces the oracle's space."""
    seq = w.seq_3d(N=12, nshift=1, nrhs=1, k=10)
    A, At = (m.to_scipy() for m in seq.matrix(0))
    n = A.shape[0]
    st = {}

    def cyc(V, Vt):
        st["V"], st["Vt"] = V, Vt

    o.rbicg(A, At, o.empty_blocks(n), seq.rhs[0], rtol=1e-10, s=100000, on_cycle=cyc)
    W, Wt = st["V"], st["Vt"]
    # the library stores raw residuals: rescale the columns like them
    scale = np.logspace(0, -9, W.shape[1])
    W, Wt = W * scale, Wt * scale[::-1]
    k = 10
    Q, AQ = _orth(shim, W, A @ W)
    Qt, _ = _orth(shim, Wt)
    r, rt = Q.shape[1], Qt.shape[1]
    F = _fortran(Qt.T @ Q).ravel(order="F")
    G = _fortran(Qt.T @ AQ).ravel(order="F")
    F2 = _fortran(Q.T @ AQ).ravel(order="F")
    G2 = _fortran(AQ.T @ AQ).ravel(order="F")
    Y, Yt = np.zeros(r * k), np.zeros(rt * k)
    kout = shim.shim_recycle_ritz_orth(r, rt, _p(F), _p(G), _p(G2), _p(F2), k, _p(Y), _p(Yt))
    assert kout > 0
    U = Q @ Y[: r * kout].reshape(r, kout, order="F")
    Ut = Qt @ Yt[: rt * kout].reshape(rt, kout, order="F")
    Uo, Uto, _ = o.recycle_space(A, W, Wt, k)
    assert kout == Uo.shape[1]
    assert np.allclose(np.linalg.norm(U, axis=0), 1.0, rtol=1e-10)
    # same subspaces, away from a possible near-tie at the k boundary: the leading half
    h = kout // 2
    assert sla.subspace_angles(U[:, :h], Uo).max() < 1e-6
    assert sla.subspace_angles(Ut[:, :h], Uto).max() < 1e-6

"""Pins of the oracle's adjoint (dL/db, dL/dsigma, dL/dK of L = c^T A(sigma)^-1 b).

The gradient formulas are checked against central finite differences of
dense LU solves (nothing of the oracle's Krylov code is involved); the
adjoint Krylov solve against a dense solve of A^T lambda = c; the swapped
recycle blocks against the transpose of A's oblique projector.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as o
import workloads as w


@pytest.fixture(scope="module")
def prob():
    seq = w.seq_2d()
    sigma = float(seq.sigmas[2])
    K = seq.K
    rng = np.random.default_rng(7)
    c = rng.standard_normal(seq.n)
    return seq, K, sigma, c


def _dense(K, mdiag, sigma, kval=None):
    A = K.to_scipy().toarray() if kval is None else \
        o_csr(K, kval).toarray()
    return A + sigma * np.diag(mdiag)


def o_csr(K, kval):
    import scipy.sparse as sp
    return sp.csr_matrix((kval, K.colidx, K.rowptr), shape=(K.n, K.n))


def _loss(K, mdiag, sigma, kval, b, c):
    return float(c @ np.linalg.solve(_dense(K, mdiag, sigma, kval), b))


def test_gradient_formulas_match_central_differences(prob):
    seq, K, sigma, c = prob
    b, m = seq.rhs[0], seq.mdiag
    A = _dense(K, m, sigma)
    x = np.linalg.solve(A, b)
    lam = np.linalg.solve(A.T, c)
    g_b, g_sig, g_val = o.gradients(K.rowptr, K.colidx, m, x, lam)
    rng = np.random.default_rng(11)
    h = 1e-6
    for _ in range(3):
        db = rng.standard_normal(seq.n)
        dk = rng.standard_normal(K.nnz) * np.abs(K.val)
        ds = rng.standard_normal() * sigma
        lp = _loss(K, m, sigma + h * ds, K.val + h * dk, b + h * db, c)
        lm = _loss(K, m, sigma - h * ds, K.val - h * dk, b - h * db, c)
        fd = (lp - lm) / (2 * h)
        an = g_b @ db + g_sig * ds + g_val @ dk
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9, (fd, an)
    # each part separately (a sign or a transposed index fails one of these)
    lp = _loss(K, m, sigma * (1 + h), K.val, b, c)
    lm = _loss(K, m, sigma * (1 - h), K.val, b, c)
    assert abs((lp - lm) / (2 * h * sigma) - g_sig) <= 1e-6 * abs(g_sig)
    e = int(np.nonzero(K.colidx != np.repeat(np.arange(K.n), np.diff(K.rowptr)))[0][5])
    dk = np.zeros(K.nnz)
    dk[e] = 1.0
    hk = h * abs(K.val[e])
    lp = _loss(K, m, sigma, K.val + hk * dk, b, c)
    lm = _loss(K, m, sigma, K.val - hk * dk, b, c)
    assert abs((lp - lm) / (2 * hk) - g_val[e]) <= 1e-5 * abs(g_val[e])
    assert np.array_equal(g_b, lam)


def test_adjoint_solve_matches_dense(prob):
    seq, K, sigma, c = prob
    A, At = seq.matrix(2)
    As, Ats = A.to_scipy(), At.to_scipy()
    lam_d = np.linalg.solve(As.toarray().T, c)
    kappa = np.linalg.cond(As.toarray())
    # with an exact eigenvector space and with a random one
    ev, vl, vr = sla.eig(As.toarray(), left=True, right=True)
    order = np.argsort(np.abs(ev))
    rng = np.random.default_rng(3)
    for U, Ut in ((vr[:, order[:8]].real, vl[:, order[:8]].real),
                  (rng.standard_normal((seq.n, 6)), rng.standard_normal((seq.n, 6)))):
        lam, info = o.adjoint_solve(As, Ats, U, Ut, c, rtol=1e-12)
        assert info.status == o.OK
        assert np.linalg.norm(lam - lam_d) / np.linalg.norm(lam_d) < 10 * kappa * 1e-12


def test_swapped_blocks_give_the_transposed_projector(prob):
    """The blocks of A^T built from (Ut, U) are A's blocks with roles exchanged:
    C' Chat'^T = (C Chat^T)^T, i.e. Chat' spans Ccheck's role (eq. (CcheckChat))."""
    seq, K, sigma, c = prob
    A, At = seq.matrix(2)
    As, Ats = A.to_scipy(), At.to_scipy()
    rng = np.random.default_rng(5)
    U, Ut = rng.standard_normal((seq.n, 6)), rng.standard_normal((seq.n, 6))
    bl = o.make_blocks(As, Ats, U, Ut, secant_max=np.inf)
    tb = o.transposed_blocks(As, Ats, U, Ut, secant_max=np.inf)
    P = bl.C @ bl.Chat.T
    Pt = tb.C @ tb.Chat.T
    assert np.abs(Pt - P.T).max() < 1e-10 * np.abs(P).max()
    # and the x-correction operators U Chat^T: U' Chat'^T = Ut Ccheck^T
    assert np.abs(tb.U @ tb.Chat.T - bl.Ut @ bl.Ccheck.T).max() < 1e-10 * np.abs(bl.Ut @ bl.Ccheck.T).max()

"""Recycle blocks and recycle-space selection (oracle, FP64) -- TEST INFRASTRUCTURE ONLY.

``make_blocks`` establishes what RBiCG and RBiCGSTAB assume of their recycle
space (Sections 3 and 4): given ``U`` and ``Ut``, form ``C = A U``, ``Ct = A^T Ut``,
make ``C`` and ``Ct`` bi-orthogonal with a positive diagonal ``D_c = Ct^T C``
(Section 3, the paragraph introducing ``U``, ``Ut``, ``C``, ``Ct``), and form
``Chat = Ct D_c^{-1}`` and ``Ccheck = C D_c^{-1}`` (eq. CcheckChat).

Readings where the paper defers to other work:

* bi-orthogonalisation (the paper points to its thesis reference): an SVD
  ``Ct^T C = P S Q^T`` followed by ``U <- U Q S^-1/2``, ``C <- C Q S^-1/2``,
  ``Ut <- Ut P S^-1/2``, ``Ct <- Ct P S^-1/2`` gives ``D_c = I``; a pair j is
  discarded (k shrinks) when ``s_j <= drop * s_max`` or when its secant
  ``||C q_j|| ||Ct p_j|| / s_j`` (the norm of that pair's rank-one oblique
  projector) exceeds ``secant_max``: strongly oblique pairs make the
  projected operator ``(I - C Chat^T) A`` ill-conditioned;
* ``D_c^{-1}``: computed as a full k-by-k LU solve with ``D_c = Ct^T C``
  (identical in exact arithmetic, exact ``Chat^T C = I`` in floating point);
* the selection of U, Ut (deferred to the RBiCG reference), see
  ``recycle_space``: right vectors are harmonic Ritz vectors of A on W (the
  k smallest-magnitude harmonic Ritz values), left vectors are the left
  vectors of the two-sided (Petrov-Galerkin) Rayleigh-Ritz projection on
  (Wt, W) for its k smallest-magnitude Ritz values.  On the convection-
  diffusion operators two-sided right vectors carry large high-frequency
  components (relative residuals ~1e2), which makes the C/Ct pairs nearly
  orthogonal; harmonic right vectors do not.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla


@dataclass
class Blocks:
    """U, Ut (n x k), C = A U, Ct = A^T Ut, Chat = Ct D_c^-1, Ccheck = C D_c^-1."""
    U: np.ndarray
    Ut: np.ndarray
    C: np.ndarray
    Ct: np.ndarray
    Chat: np.ndarray
    Ccheck: np.ndarray
    matvecs_A: int = 0
    matvecs_At: int = 0

    @property
    def k(self) -> int:
        return int(self.U.shape[1])


def empty_blocks(n: int) -> Blocks:
    """No recycle space (k = 0): the first system of a sequence has none (Section 3)."""
    z = np.zeros((n, 0))
    return Blocks(z, z.copy(), z.copy(), z.copy(), z.copy(), z.copy())


def make_blocks(A, At, U: np.ndarray, Ut: np.ndarray, drop: float = 1e-12,
                secant_max: float = 1e2) -> Blocks:
    """C, Ct, Chat, Ccheck for (U, Ut) with the bi-orthogonalisation reading described above."""
    n = A.shape[0]
    if U.shape[1] == 0:
        return empty_blocks(n)
    if U.shape != Ut.shape:
        raise ValueError("U and Ut must have the same shape")
    k0 = U.shape[1]
    C = A @ U                      # C = A U
    Ct = At @ Ut                   # Ct = A^* Ut
    M = Ct.T @ C
    P, sig, Qh = np.linalg.svd(M)  # M = P diag(sig) Q^T
    secant = np.linalg.norm(C @ Qh.T, axis=0) * np.linalg.norm(Ct @ P, axis=0) / sig
    keep = (sig > drop * sig[0]) & (secant <= secant_max)
    if not np.any(keep):
        return empty_blocks(n)
    scale = 1.0 / np.sqrt(sig[keep])
    Qk = Qh.T[:, keep] * scale
    Pk = P[:, keep] * scale
    U, C = U @ Qk, C @ Qk
    Ut, Ct = Ut @ Pk, Ct @ Pk
    Dc = Ct.T @ C                  # D_c = Ct^* C  (= I up to rounding)
    lu = sla.lu_factor(Dc)
    Chat = sla.lu_solve(lu, Ct.T).T            # Chat = Ct D_c^{-T}  (Ct D_c^{-1} when diagonal)
    Ccheck = sla.lu_solve(lu, C.T, trans=1).T  # Ccheck = C D_c^{-1}
    return Blocks(U, Ut, C, Ct, Chat, Ccheck, matvecs_A=k0, matvecs_At=k0)


def _orth(W: np.ndarray) -> np.ndarray:
    Q, R = np.linalg.qr(W)
    d = np.abs(np.diag(R))
    keep = d > 1e-12 * max(d.max(), 1e-300)
    return Q[:, keep]


def ritz_select(theta: np.ndarray, k: int, pair_tol: float = 1e-10):
    """Indices (and pair flags) of the k finite Ritz values of smallest magnitude.

    Ordered by (|theta|, Re theta, Im theta).  A complex-conjugate pair occupies
    two slots ([Re y, Im y]); if the k-th slot would split a pair, only k-1
    vectors are kept.
    """
    fin = np.nonzero(np.isfinite(theta))[0]
    order = sorted(fin, key=lambda i: (abs(theta[i]), theta[i].real, theta[i].imag))
    picks = []
    used = set()
    slots = 0
    for i in order:
        if slots >= k:
            break
        if i in used:
            continue
        is_complex = abs(theta[i].imag) > pair_tol * max(abs(theta[i]), 1e-300)
        if is_complex:
            if slots + 2 > k:
                break
            # the conjugate partner, nearest conj(theta) among unused
            cands = [j for j in fin if j != i and j not in used]
            j = min(cands, key=lambda j: abs(theta[j] - np.conj(theta[i])))
            used.update((i, j))
            picks.append((i, True))
            slots += 2
        else:
            used.add(i)
            picks.append((i, False))
            slots += 1
    return picks


def _real_basis(Y: np.ndarray, theta: np.ndarray, picks):
    cols, vals = [], []
    for i, cplx in picks:
        if cplx:
            cols += [Y[:, i].real, Y[:, i].imag]
            vals += [theta[i], np.conj(theta[i])]
        else:
            cols.append(Y[:, i].real)
            vals.append(theta[i])
    return cols, vals


def harmonic_ritz(A, W: np.ndarray, k: int, Q=None):
    """Harmonic Ritz vectors of A on range(W) for the k smallest-magnitude harmonic Ritz values.

    With Q an orthonormal basis of W: solve (AQ)^T (AQ) y = theta (AQ)^T Q y,
    i.e. the residual A Q y - theta Q y is orthogonal to A Q.  Returns
    ``(U, theta)`` with unit-norm columns.
    """
    Q = _orth(W) if Q is None else Q
    AQ = A @ Q
    theta, Y = sla.eig(AQ.T @ AQ, AQ.T @ Q)
    cols, vals = _real_basis(Y, theta, ritz_select(theta, k))
    if not cols:
        return np.zeros((W.shape[0], 0)), np.zeros(0, dtype=complex)
    U = Q @ np.array(cols).T
    return U / np.linalg.norm(U, axis=0), np.array(vals)


def recycle_space(A, W: np.ndarray, Wt: np.ndarray, k: int):
    """The recycle-space update: harmonic right vectors, two-sided left vectors.

    Returns ``(U, Ut, number of products with A)``.
    """
    Q = _orth(W)
    U, _ = harmonic_ritz(A, W, k, Q=Q)
    _, Ut, _, m = two_sided_ritz(A, W, Wt, k, Q=Q)
    kk = min(U.shape[1], Ut.shape[1])   # conjugate pairs can make the two counts differ by one
    return U[:, :kk], Ut[:, :kk], m


def two_sided_ritz(A, W: np.ndarray, Wt: np.ndarray, k: int, Q=None):
    """Approximate right/left invariant subspaces for the k smallest-|theta| Ritz values.

    Reading of the paper's deferred selection rule (Sections 5 and 6.2 ask
    for approximate left and right invariant subspaces of smallest-magnitude
    eigenvalues): orthonormalise ``W`` and ``Wt``, form ``G = Wt^T A W`` and
    ``F = Wt^T W``, solve ``G y = theta F y`` and ``G^T yt = theta F^T yt``,
    and return ``U = W Y``, ``Ut = Wt Yt`` (columns scaled to unit norm) and
    the selected Ritz values.  ``A W`` is formed with explicit products.
    """
    Q = _orth(W) if Q is None else Q
    Qt = _orth(Wt)
    m = min(Q.shape[1], Qt.shape[1])
    Q, Qt = Q[:, :m], Qt[:, :m]
    AQ = A @ Q
    G = Qt.T @ AQ
    F = Qt.T @ Q
    theta, yl, yr = sla.eig(G, F, left=True, right=True)
    picks = ritz_select(theta, k)
    Y, Yt, vals = [], [], []
    for i, cplx in picks:
        if cplx:
            Y += [yr[:, i].real, yr[:, i].imag]
            Yt += [yl[:, i].real, yl[:, i].imag]
            vals += [theta[i], np.conj(theta[i])]
        else:
            Y.append(yr[:, i].real)
            Yt.append(yl[:, i].real)
            vals.append(theta[i])
    if not Y:
        z = np.zeros((W.shape[0], 0))
        return z, z.copy(), np.zeros(0, dtype=complex), Q.shape[1]
    U = Q @ np.array(Y).T
    Ut = Qt @ np.array(Yt).T
    U /= np.linalg.norm(U, axis=0)
    Ut /= np.linalg.norm(Ut, axis=0)
    return U, Ut, np.array(vals), Q.shape[1]

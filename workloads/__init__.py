"""Seeded synthetic inputs for the shifted convection-diffusion sequences.

This module builds the *inputs* of the problem family only: sparse matrices
``K`` (finite-difference convection-diffusion operators), the diagonal mass
matrix ``M``, the shifts ``sigma``, right-hand sides and shadow vectors.  It
holds none of the solver's arithmetic, so both the CPU oracle and the GPU
path can consume it without sharing any solver code.

The sequence it describes is the paper's problem statement (Section 1,
equation (1.1)): matrices ``A(i) = K + sigma_i M`` that change slowly along
the sequence, each with several right-hand sides ``b(i, j)``; the PMOR
family of Section 6.1 (``A0 + sigma A1 + delta A2`` with small perturbation
terms) is the model for the ``K + sigma M`` form.

Operator: ``K = -Laplace_h + Pe * (v . grad_h)`` on the unit square / cube
with homogeneous Dirichlet boundary, the interior points ordered
lexicographically with x fastest, ``h = 1/(N+1)`` per axis, diffusion scaled
by ``1/h^2`` and first-order upwind convection per axis sign.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence as Seq, Tuple

import numpy as np
import scipy.sparse as sp

SEED_ROOT = 1406
STREAMS = {"M": 0, "b": 1, "shadow": 2, "c": 3, "v": 4, "dirs": 5, "U": 6}


def generator(cfg: int, system: int, stream: str) -> np.random.Generator:
    """PCG64 generator for (config, system, stream); every input is drawn from one."""
    return np.random.default_rng(
        np.random.SeedSequence([SEED_ROOT, int(cfg), int(system), STREAMS[stream]]))


@dataclass
class Csr:
    """CSR matrix with int32 indices and float64 values (sorted column indices)."""
    n: int
    rowptr: np.ndarray
    colidx: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.colidx.shape[0])

    @staticmethod
    def from_scipy(m) -> "Csr":
        m = sp.csr_matrix(m)
        m.sort_indices()
        return Csr(int(m.shape[0]), m.indptr.astype(np.int32),
                   m.indices.astype(np.int32), m.data.astype(np.float64))

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.colidx, self.rowptr), shape=(self.n, self.n))

    def transpose(self) -> "Csr":
        # coo -> csr keeps explicit zeros, so the transpose has the same structure
        coo = self.to_scipy().tocoo()
        t = sp.coo_matrix((coo.data, (coo.col, coo.row)), shape=(self.n, self.n)).tocsr()
        return Csr.from_scipy(t)

    def diag_positions(self) -> np.ndarray:
        """Index into ``val`` of each row's diagonal entry (every row must have one)."""
        pos = np.full(self.n, -1, dtype=np.int64)
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        hit = np.nonzero(self.colidx == rows)[0]
        pos[rows[hit]] = hit
        if np.any(pos < 0):
            raise ValueError("matrix has rows without a stored diagonal")
        return pos


def _axis_1d(N: int, c: float, h: float) -> sp.csr_matrix:
    """1D factor ``h^-2 tridiag(-1, 2, -1) + (c/h) * upwind`` for one axis."""
    main = np.full(N, 2.0 / h**2)
    lower = np.full(N - 1, -1.0 / h**2)
    upper = np.full(N - 1, -1.0 / h**2)
    if c >= 0.0:   # c u_x ~ c (u_i - u_{i-1}) / h
        main += c / h
        lower += -c / h
    else:          # c u_x ~ c (u_{i+1} - u_i) / h
        main += -c / h
        upper += c / h
    return sp.diags([lower, main, upper], [-1, 0, 1], shape=(N, N), format="coo")


def _coo_sum(terms) -> sp.csr_matrix:
    """Sum COO matrices keeping every structural entry (no zero pruning)."""
    rows = np.concatenate([t.row for t in terms])
    cols = np.concatenate([t.col for t in terms])
    data = np.concatenate([t.data for t in terms])
    shape = terms[0].shape
    m = sp.coo_matrix((data, (rows, cols)), shape=shape).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return m


def _kron(*factors) -> sp.coo_matrix:
    out = factors[0]
    for f in factors[1:]:
        out = sp.kron(out, f, format="coo")
    return sp.coo_matrix(out)


def convdiff(dims: Seq[int], vel: Seq[float], pe: float) -> Csr:
    """5-point (2D) or 7-point (3D) upwind convection-diffusion operator.

    ``dims`` lists the interior points per axis, x first; the lexicographic
    index is ``x + Nx*(y + Ny*z)`` (x fastest).
    """
    d = len(dims)
    if d not in (2, 3) or len(vel) != d:
        raise ValueError("dims/vel must both have 2 or 3 entries")
    eyes = [sp.identity(N, format="coo") for N in dims]
    terms = []
    for a in range(d):
        N = dims[a]
        h = 1.0 / (N + 1)
        fac = [eyes[b] for b in range(d)]
        fac[a] = _axis_1d(N, pe * vel[a], h)
        # Kronecker order: slowest axis first
        terms.append(_kron(*reversed(fac)))
    return Csr.from_scipy(_coo_sum(terms))


def convdiff27(N: int, vel: Seq[float], pe: float) -> Csr:
    """27-point operator ``Kz(x)M(x)M + M(x)Ky(x)M + M(x)M(x)Kx`` with ``M = tridiag(1,4,1)/6``."""
    h = 1.0 / (N + 1)
    m1 = sp.diags([np.full(N - 1, 1 / 6), np.full(N, 4 / 6), np.full(N - 1, 1 / 6)],
                  [-1, 0, 1], shape=(N, N), format="coo")
    kx, ky, kz = (_axis_1d(N, pe * v, h) for v in vel)
    terms = [_kron(kz, m1, m1), _kron(m1, ky, m1), _kron(m1, m1, kx)]
    return Csr.from_scipy(_coo_sum(terms))


def shifted(K: Csr, mdiag: np.ndarray, sigma: float) -> Csr:
    """``K + sigma * diag(mdiag)`` on the structure of ``K`` (diagonal must be stored)."""
    val = K.val.copy()
    pos = K.diag_positions()
    val[pos] += sigma * mdiag
    return Csr(K.n, K.rowptr, K.colidx, val)


def log_shifts(count: int, lo: float = 1e-2, hi: float = 1e1) -> np.ndarray:
    if count == 1:
        return np.array([lo])
    return lo * (hi / lo) ** (np.arange(count) / (count - 1))


@dataclass
class ShiftedSequence:
    """The systems ``(K + sigma_i M) x = b(i, j)`` in shift-major order."""
    cfg: int
    K: Csr
    Kt: Csr
    mdiag: np.ndarray
    sigmas: np.ndarray
    nrhs: int
    k: int
    name: str = ""
    rhs: List[np.ndarray] = field(default_factory=list)
    shadows: List[np.ndarray] = field(default_factory=list)

    @property
    def n(self) -> int:
        return self.K.n

    @property
    def num_systems(self) -> int:
        return len(self.sigmas) * self.nrhs

    def system(self, idx: int) -> Tuple[int, int]:
        """(shift index, rhs index) of system ``idx``."""
        return idx // self.nrhs, idx % self.nrhs

    def matrix(self, shift_idx: int) -> Tuple[Csr, Csr]:
        s = float(self.sigmas[shift_idx])
        return shifted(self.K, self.mdiag, s), shifted(self.Kt, self.mdiag, s)


def make_sequence(cfg: int, K: Csr, nshift: int, nrhs: int, k: int, name: str = "",
                  sigmas=None) -> ShiftedSequence:
    n = K.n
    mdiag = generator(cfg, 0, "M").uniform(0.5, 1.5, size=n)
    sig = log_shifts(nshift) if sigmas is None else np.asarray(sigmas, dtype=np.float64)
    seq = ShiftedSequence(cfg, K, K.transpose(), mdiag, sig, nrhs, k, name)
    for idx in range(len(sig) * nrhs):
        seq.rhs.append(generator(cfg, idx, "b").standard_normal(n))
        seq.shadows.append(generator(cfg, idx, "shadow").standard_normal(n))
    return seq


# ---------------------------------------------------------------------------
# The named workloads.  ``N`` may be overridden to build a smaller instance of
# the same family (tests); the defaults are the full sizes.
# ---------------------------------------------------------------------------

VEL2 = (1.0, 0.5)
VEL3 = (1.0, 0.5, 0.25)
PECLET = 10.0


def seq_2d(N: int = 32, nshift: int = 4, nrhs: int = 1, k: int = 8) -> ShiftedSequence:
    """2D 5-point convection-diffusion, N x N grid, v=(1, 0.5), Pe=10 (n=1024 at N=32)."""
    K = convdiff((N, N), VEL2, PECLET)
    return make_sequence(0, K, nshift, nrhs, k, f"2d5pt-{N}")


def seq_3d(N: int = 64, nshift: int = 5, nrhs: int = 4, k: int = 20) -> ShiftedSequence:
    """3D 7-point convection-diffusion, N^3 grid, v=(1, .5, .25), Pe=10 (n=262144 at N=64)."""
    K = convdiff((N, N, N), VEL3, PECLET)
    return make_sequence(1, K, nshift, nrhs, k, f"3d7pt-{N}")


def seq_3d27(N: int = 160, nshift: int = 10, nrhs: int = 5, k: int = 30) -> ShiftedSequence:
    """3D 27-point nonsymmetric stencil on N^3 (n=4,096,000 at N=160)."""
    K = convdiff27(N, VEL3, PECLET)
    return make_sequence(4, K, nshift, nrhs, k, f"3d27pt-{N}")


def adjoint_problem(N: int = 128, sigma: float = 1.0, ndirs: int = 16):
    """3D 7-point grid with one shift; returns (sequence, loss vector c, FD directions)."""
    K = convdiff((N, N, N), VEL3, PECLET)
    seq = make_sequence(3, K, 1, 1, 20, f"adjoint-{N}", sigmas=[sigma])
    c = generator(3, 0, "c").standard_normal(K.n)
    dirs = generator(3, 0, "dirs").standard_normal((ndirs, K.n))
    return seq, c, dirs


def batched_dims(count: int = 32, n_lo: float = 40e3, n_hi: float = 500e3) -> List[Tuple[int, int, int]]:
    """Uneven 3D grid shapes (m+8, m, m-6) with n spread log-uniformly over [n_lo, n_hi]."""
    out = []
    for j in range(count):
        nt = n_lo * (n_hi / n_lo) ** (j / (count - 1))
        m = int(round(nt ** (1.0 / 3.0)))
        out.append((m + 8, m, m - 6))
    return out


def batched_systems(count: int = 32, scale: float = 1.0):
    """Batch of shifted 3D systems of uneven size; velocities U[-1,1]^3, shifts log-spaced.

    Returns a list of (A, At, b, shadow) with ``A = K_j + sigma_j M_j``.
    ``scale`` shrinks every grid (tests).
    """
    dims = batched_dims(count)
    sig = log_shifts(count)
    out = []
    for j, (nx, ny, nz) in enumerate(dims):
        if scale != 1.0:
            nx, ny, nz = (max(3, int(round(d * scale))) for d in (nx, ny, nz))
        vel = tuple(generator(2, j, "v").uniform(-1.0, 1.0, size=3))
        K = convdiff((nx, ny, nz), vel, PECLET)
        mdiag = generator(2, j, "M").uniform(0.5, 1.5, size=K.n)
        A = shifted(K, mdiag, float(sig[j]))
        At = A.transpose()
        b = generator(2, j, "b").standard_normal(K.n)
        sh = generator(2, j, "shadow").standard_normal(K.n)
        out.append((A, At, b, sh))
    return out


def separable_eigenpairs(dims: Seq[int], vel: Seq[float], pe: float, k: int):
    """The k smallest eigenvalues of ``convdiff(dims, vel, pe)`` with their right
    and left eigenvectors, in closed form (an exact recycle space to install).

    The operator is a Kronecker sum of 1D tridiagonal Toeplitz factors
    ``tridiag(a, b, c)`` (sub-, main, super-diagonal), whose eigenpairs are
    ``b + 2 sgn(a) sqrt(a c) cos(j pi / (N+1))`` with right vectors
    ``(a/c)^(i/2) sin(i j pi / (N+1))`` and left vectors
    ``(c/a)^(i/2) sin(i j pi / (N+1))`` (i, j = 1..N); the 3D (2D) pairs are
    sums of values and Kronecker products of vectors.  Returns
    ``(lam (k,), U (n, k), Ut (n, k))`` with unit-norm columns, ordered by
    eigenvalue.
    """
    d = len(dims)
    facs = []
    for a in range(d):
        N = dims[a]
        h = 1.0 / (N + 1)
        c = pe * vel[a]
        lo, mid, up = -1.0 / h**2, 2.0 / h**2, -1.0 / h**2
        if c >= 0.0:
            mid += c / h
            lo += -c / h
        else:
            mid += -c / h
            up += c / h
        j = np.arange(1, N + 1)
        i = np.arange(1, N + 1)
        lam = mid + 2.0 * np.sign(lo) * np.sqrt(lo * up) * np.cos(j * np.pi / (N + 1))
        s = np.sin(np.outer(i, j) * np.pi / (N + 1))
        # weights (a/c)^(i/2) formed in logs: they span many orders of magnitude
        logw = 0.5 * i * np.log(lo / up)
        right = s * np.exp(logw - logw.max())[:, None]
        left = s * np.exp(-logw - (-logw).max())[:, None]
        facs.append((lam, right, left))
    # candidate modes: every axis index up to k (enough for the k smallest sums)
    grids = np.meshgrid(*[np.arange(min(k, dims[a])) for a in range(d)], indexing="ij")
    modes = np.stack([g.ravel() for g in grids], axis=1)
    vals = sum(facs[a][0][modes[:, a]] for a in range(d))
    order = np.argsort(vals, kind="stable")[:k]
    n = int(np.prod(dims))
    U = np.empty((n, k))
    Ut = np.empty((n, k))
    for col, m in enumerate(order):
        r = np.ones(1)
        l = np.ones(1)
        for a in reversed(range(d)):   # Kronecker order: slowest axis (z) first
            r = np.kron(r, facs[a][1][:, modes[m, a]])
            l = np.kron(l, facs[a][2][:, modes[m, a]])
        U[:, col] = r / np.linalg.norm(r)
        Ut[:, col] = l / np.linalg.norm(l)
    return vals[order], U, Ut

"""Seeded synthetic inputs: SPD matrices in CSR form and right-hand sides.

This module only builds inputs.  It holds none of the method's arithmetic
(no ordering, no factorization, no iteration), so both the CPU oracle and the
HIP path can draw their inputs from it.

The paper measures on SuiteSparse and FEM matrices that are not available
here (Section 5.1, Table "matInfo").  These generators stand in for them with
matrices of the same class: sparse, symmetric positive definite M-matrices
from 2D/3D discretizations and an unstructured graph Laplacian.

Every matrix is returned as a :class:`CSR` with 0-based int64 row pointers,
int32 column indices sorted ascending inside each row, float64 values and
both triangles stored.  Values are exactly symmetric: a_ij and a_ji are the
same double.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass(frozen=True)
class CSR:
    n: int
    rowptr: np.ndarray  # int64 [n+1]
    col: np.ndarray     # int32 [nnz]
    val: np.ndarray     # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


def _from_coo(n: int, rows, cols, vals) -> CSR:
    m = sp.coo_matrix((np.asarray(vals, np.float64),
                       (np.asarray(rows, np.int64), np.asarray(cols, np.int64))),
                      shape=(n, n)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return CSR(n, m.indptr.astype(np.int64), m.indices.astype(np.int32),
               m.data.astype(np.float64))


def from_scipy(m) -> CSR:
    m = sp.csr_matrix(m)
    m.sum_duplicates()
    m.sort_indices()
    return CSR(m.shape[0], m.indptr.astype(np.int64), m.indices.astype(np.int32),
               m.data.astype(np.float64))


# --------------------------------------------------------------------------
# structured grids
# --------------------------------------------------------------------------

def grid2d_5pt(nx: int, ny: int | None = None) -> CSR:
    """2D 5-point Laplacian, Dirichlet boundary eliminated: 4 on the diagonal,
    -1 to each of the (up to) four neighbours.  Unknown (x, y) has index
    ``nx*y + x`` (x fastest)."""
    ny = nx if ny is None else ny
    n = nx * ny
    idx = np.arange(n, dtype=np.int64)
    x, y = idx % nx, idx // nx
    rows, cols, vals = [idx], [idx], [np.full(n, 4.0)]
    for ok, nb in ((x > 0, idx - 1), (x < nx - 1, idx + 1),
                   (y > 0, idx - nx), (y < ny - 1, idx + nx)):
        rows.append(idx[ok]); cols.append(nb[ok]); vals.append(np.full(ok.sum(), -1.0))
    return _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def path_1d(n: int) -> CSR:
    """1D Laplacian (tridiagonal 2, -1) on a path of n unknowns."""
    idx = np.arange(n, dtype=np.int64)
    rows = np.concatenate([idx, idx[1:], idx[:-1]])
    cols = np.concatenate([idx, idx[:-1], idx[1:]])
    vals = np.concatenate([np.full(n, 2.0), np.full(2 * (n - 1), -1.0)])
    return _from_coo(n, rows, cols, vals)


def face_coefficients(N: int, sigma: float, seed: int):
    """Lognormal face coefficients kappa = exp(sigma * N(0,1)) of an N^3 cell
    grid, drawn in the fixed order x-faces (N, N, N+1), y-faces (N, N+1, N),
    z-faces (N+1, N, N) from ``numpy.random.default_rng(seed)``.  Arrays are
    indexed [z, y, x]; face index f lies between cells f-1 and f."""
    rng = np.random.default_rng(seed)
    kx = np.exp(sigma * rng.standard_normal((N, N, N + 1)))
    ky = np.exp(sigma * rng.standard_normal((N, N + 1, N)))
    kz = np.exp(sigma * rng.standard_normal((N + 1, N, N)))
    return kx, ky, kz


def diffusion3d(N: int, sigma: float = 1.0, seed: int = 2, *, kappa=None) -> CSR:
    """Cell-centred finite-volume 7-point diffusion on an N^3 grid.

    Interior face f between cells i and j gives a_ij = a_ji = -kappa_f.  The
    diagonal is the sum of the six face coefficients of the cell; boundary
    faces are Dirichlet, so they add to the diagonal only.  Cell (x, y, z) has
    index ``x + N*y + N*N*z``.  ``sigma = 0`` (or unit ``kappa``) gives the
    7-point Poisson matrix with 6 on the diagonal and -1 off it.
    """
    if kappa is None:
        kx, ky, kz = face_coefficients(N, sigma, seed)
    else:
        kx, ky, kz = kappa
    n = N ** 3
    idx = np.arange(n, dtype=np.int64).reshape(N, N, N)  # [z, y, x]
    diag = (kx[:, :, :-1] + kx[:, :, 1:]) + (ky[:, :-1, :] + ky[:, 1:, :]) \
        + (kz[:-1, :, :] + kz[1:, :, :])
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [diag.ravel()]
    # x-faces 1..N-1 couple cells (x-1, x)
    a, b, k = idx[:, :, :-1], idx[:, :, 1:], kx[:, :, 1:-1]
    # y-faces 1..N-1 couple (y-1, y), z-faces 1..N-1 couple (z-1, z)
    pairs = [(a, b, k),
             (idx[:, :-1, :], idx[:, 1:, :], ky[:, 1:-1, :]),
             (idx[:-1, :, :], idx[1:, :, :], kz[1:-1, :, :])]
    for a, b, k in pairs:
        a, b, k = a.ravel(), b.ravel(), -k.ravel()
        rows += [a, b]; cols += [b, a]; vals += [k, k]
    return _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def poisson3d(N: int) -> CSR:
    """7-point Poisson on N^3 (6 on the diagonal, -1 off it, Dirichlet)."""
    ones = (np.ones((N, N, N + 1)), np.ones((N, N + 1, N)), np.ones((N + 1, N, N)))
    return diffusion3d(N, kappa=ones)


# --------------------------------------------------------------------------
# unstructured: symmetric k-nearest-neighbour graph Laplacian
# --------------------------------------------------------------------------

def knn_laplacian(npts: int, k: int = 13, seed_points: int = 4, seed_perm: int | None = 5,
                  shift: float = 1e-3, points=None) -> CSR:
    """Graph Laplacian of the union-symmetrized k-NN graph of ``npts`` points
    uniform in the unit cube, with edge weights 1/distance, plus ``shift`` on
    the diagonal; the numbering is shuffled with a seeded permutation
    (``seed_perm=None``: the points' own order).

    A = diag(sum_j w_ij) - W + shift*I.  It is a symmetric M-matrix and
    strictly diagonally dominant, hence SPD.
    """
    from scipy.spatial import cKDTree
    if points is None:
        points = np.random.default_rng(seed_points).random((npts, 3))
    tree = cKDTree(points)
    _, nbr = tree.query(points, k=k + 1, workers=-1)
    src = np.repeat(np.arange(npts, dtype=np.int64), k)
    dst = nbr[:, 1:].ravel().astype(np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    key = np.unique(lo * npts + hi)                     # union symmetrization
    lo, hi = key // npts, key % npts
    d = points[lo] - points[hi]
    w = 1.0 / np.sqrt((d * d).sum(axis=1))              # one value per edge
    deg = np.zeros(npts)
    np.add.at(deg, lo, w)
    np.add.at(deg, hi, w)
    perm = (np.arange(npts) if seed_perm is None
            else np.random.default_rng(seed_perm).permutation(npts))  # old -> new
    rows = np.concatenate([perm[lo], perm[hi], perm])
    cols = np.concatenate([perm[hi], perm[lo], perm])
    vals = np.concatenate([-w, -w, deg + shift])
    return _from_coo(npts, rows, cols, vals)


# --------------------------------------------------------------------------
# small test graphs
# --------------------------------------------------------------------------

def random_spd(n: int, density: float, seed: int) -> CSR:
    """Random symmetric pattern with negative off-diagonals and a dominant
    diagonal (a symmetric M-matrix, hence SPD)."""
    rng = np.random.default_rng(seed)
    m = sp.random(n, n, density=density, random_state=rng, format="coo")
    lo, hi = np.minimum(m.row, m.col), np.maximum(m.row, m.col)
    keep = lo != hi
    key = np.unique(lo[keep].astype(np.int64) * n + hi[keep])
    lo, hi = key // n, key % n
    w = rng.uniform(0.1, 1.0, size=len(key))
    deg = np.zeros(n)
    np.add.at(deg, lo, w)
    np.add.at(deg, hi, w)
    diag = deg + rng.uniform(0.05, 0.5, size=n)
    rows = np.concatenate([lo, hi, np.arange(n)])
    cols = np.concatenate([hi, lo, np.arange(n)])
    vals = np.concatenate([-w, -w, diag])
    return _from_coo(n, rows, cols, vals)


def tree_spd(n: int, seed: int) -> CSR:
    """SPD matrix on a random tree (no cycles, so IC(0) has no fill)."""
    rng = np.random.default_rng(seed)
    parent = np.array([rng.integers(0, i) for i in range(1, n)], dtype=np.int64)
    child = np.arange(1, n, dtype=np.int64)
    w = rng.uniform(0.2, 1.0, size=n - 1)
    deg = np.zeros(n)
    np.add.at(deg, parent, w)
    np.add.at(deg, child, w)
    diag = deg + rng.uniform(0.1, 1.0, size=n)
    rows = np.concatenate([parent, child, np.arange(n)])
    cols = np.concatenate([child, parent, np.arange(n)])
    vals = np.concatenate([-w, -w, diag])
    return _from_coo(n, rows, cols, vals)


# --------------------------------------------------------------------------
# right-hand sides
# --------------------------------------------------------------------------

def uniform_rhs(n: int, seed: int, k: int | None = None) -> np.ndarray:
    """b ~ U[-1, 1] from ``default_rng(seed)``; shape (n,) or (k, n)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=n if k is None else (k, n))


def row_sums(A: CSR) -> np.ndarray:
    """b = A * ones, so that the exact solution is x = 1."""
    return np.add.reduceat(A.val, A.rowptr[:-1]) if A.n else np.zeros(0)


# body diagonals of the unit cube, each as (start point, direction)
_DIAGONALS = (((0., 0., 0.), (1., 1., 1.)), ((1., 0., 0.), (-1., 1., 1.)),
              ((0., 1., 0.), (1., -1., 1.)), ((0., 0., 1.), (1., 1., -1.)))


def sample_sources(count: int, seed: int) -> np.ndarray:
    """Source parameters theta, shape (count, 12): four positions s_q in
    [0.15, 0.85] along the cube's body diagonals, four widths in
    [0.03, 0.15] and four amplitudes in [-1, 1]."""
    rng = np.random.default_rng(seed)
    s = rng.uniform(0.15, 0.85, size=(count, 4))
    w = rng.uniform(0.03, 0.15, size=(count, 4))
    a = rng.uniform(-1.0, 1.0, size=(count, 4))
    return np.concatenate([s, w, a], axis=1)


def gaussian_sources_rhs(N: int, theta: np.ndarray) -> np.ndarray:
    """b at the N^3 cell centres (index x + N*y + N*N*z) for one parameter
    vector theta = (s_0..s_3, width_0..width_3, amp_0..amp_3)."""
    c = (np.arange(N) + 0.5) / N
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    b = np.zeros((N, N, N))
    for q in range(4):
        o, d = _DIAGONALS[q]
        cq = np.array(o) + theta[q] * np.array(d)
        r2 = (x - cq[0]) ** 2 + (y - cq[1]) ** 2 + (z - cq[2]) ** 2
        b += theta[8 + q] * np.exp(-r2 / (2.0 * theta[4 + q] ** 2))
    return b.ravel()


def batch_sizes(count: int = 128, seed: int = 7, lo: int = 16, hi: int = 64) -> np.ndarray:
    """Edge lengths N_s ~ U{lo..hi} of a batch of Poisson systems."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=count)


def block_diag(mats) -> tuple[CSR, np.ndarray]:
    """One block-diagonal CSR holding independent systems one after another,
    and sys_ptr (system s owns rows sys_ptr[s] .. sys_ptr[s + 1] - 1)."""
    sizes = np.array([m.n for m in mats], np.int64)
    sys_ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    rp = [np.zeros(1, np.int64)]
    at = 0
    for m in mats:
        rp.append(np.asarray(m.rowptr[1:], np.int64) + at)
        at += int(m.rowptr[-1])
    col = np.concatenate([np.asarray(m.col, np.int64) + o for m, o in zip(mats, sys_ptr[:-1])])
    val = np.concatenate([np.asarray(m.val, np.float64) for m in mats])
    return CSR(int(sys_ptr[-1]), np.concatenate(rp), col.astype(np.int32), val), sys_ptr


def poisson_batch(count: int = 128, seed: int = 7, lo: int = 16, hi: int = 64):
    """The uneven batch: Poisson systems on N_s^3 grids, N_s ~ U{lo..hi}."""
    return block_diag([poisson3d(int(N)) for N in batch_sizes(count, seed, lo, hi)])

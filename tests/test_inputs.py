"""The synthetic inputs have the structure the workloads call for."""
import numpy as np
import pytest

from paper_1908_00741_amd import inputs


def _symmetric_exact(A):
    S = A.to_scipy()
    D = (S - S.T).tocoo()
    return D.nnz == 0 or np.all(D.data == 0.0)


def test_grid2d_counts():
    A = inputs.grid2d_5pt(64)
    assert A.n == 4096
    # 5-point: n diagonal entries + 2 * (2 * 64 * 63) couplings
    assert A.nnz == 4096 + 4 * 64 * 63
    assert _symmetric_exact(A)
    assert np.allclose(inputs.row_sums(A), (A.to_scipy() @ np.ones(A.n)))


def test_diffusion3d_counts_and_symmetry():
    N = 12
    A = inputs.diffusion3d(N, 1.0, 2)
    assert A.n == N ** 3
    assert A.nnz == N ** 3 + 6 * N * N * (N - 1)
    assert _symmetric_exact(A)
    S = A.to_scipy()
    off = S - __import__("scipy.sparse", fromlist=["diags"]).diags(S.diagonal())
    # irreducibly diagonally dominant: equality inside, strict where a
    # Dirichlet face adds to the diagonal only
    rowsum = np.abs(off).sum(axis=1).A1
    assert np.all(S.diagonal() >= rowsum * (1 - 1e-14))
    assert np.all(S.diagonal()[0] > rowsum[0])


def test_diffusion3d_full_size_nnz_closed_form():
    # 128^3: n + 6 N^2 (N-1) = 14,581,760 nonzeros
    N = 128
    assert N ** 3 + 6 * N * N * (N - 1) == 14_581_760


def test_poisson3d_values():
    A = inputs.poisson3d(5)
    S = A.to_scipy()
    assert np.all(S.diagonal() == 6.0)
    assert set(np.unique(A.val)) == {-1.0, 6.0}


def test_knn_laplacian_small():
    A = inputs.knn_laplacian(2000, k=13, seed_points=4, seed_perm=5)
    assert _symmetric_exact(A)
    S = A.to_scipy()
    assert np.allclose(S @ np.ones(A.n), 1e-3)       # Laplacian rows sum to the shift
    deg = np.diff(A.rowptr) - 1
    assert deg.min() >= 13 and 14 <= deg.mean() + 1 <= 20


def test_sources_rhs_shape():
    th = inputs.sample_sources(3, 11)
    assert th.shape == (3, 12)
    assert np.all((th[:, :4] >= 0.15) & (th[:, :4] <= 0.85))
    b = inputs.gaussian_sources_rhs(16, th[0])
    assert b.shape == (16 ** 3,) and np.isfinite(b).all()


@pytest.mark.parametrize("seed", [0, 1])
def test_random_spd_is_m_matrix(seed):
    A = inputs.random_spd(200, 0.03, seed)
    S = A.to_scipy()
    assert _symmetric_exact(A)
    assert np.all(np.linalg.eigvalsh(S.toarray()) > 0)

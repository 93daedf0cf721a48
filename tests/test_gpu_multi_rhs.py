"""GPU parity for several right-hand sides at once (vectors [n][K]).

Bars:
- ic0_apply and hbmc_spmv with K right-hand sides, for every right-hand-side
  tile: each column against the oracle's single-vector result, with the
  single-vector bars (apply FP64: 1e-13 in norm and 1e-12 per entry of
  max|z_ref|; FP32: 1e-5 of max|z_ref|; SpMV: 1e-14 relative);
- iccg_solve with K right-hand sides: each column takes the iteration count
  of its single-vector solve and agrees with it to 1e-12 relative (FP64:
  the column's arithmetic is the single-vector arithmetic up to the order
  of the partial sums); a zero column returns x = 0 after 0 iterations;
  batches of systems with several right-hand sides report system-major.
"""
import numpy as np
import pytest

from paper_1908_00741_amd import hbmc, inputs

pytestmark = pytest.mark.gpu
TILES = [4, 8, 16]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


CASES = [
    ("diff3d_20_bs8_w64", lambda: inputs.diffusion3d(20, 1.0, 2), 8, 64),
    ("grid_ragged_bs4_w8", lambda: inputs.grid2d_5pt(37, 11), 4, 8),
    ("knn_3000_bs4_w16", lambda: inputs.knn_laplacian(3000, 13, 6, 7, shift=1e-3), 4, 16),
    ("random_bs2_w32", lambda: inputs.random_spd(999, 0.006, 8), 2, 32),
    ("random_bs16_w4", lambda: inputs.random_spd(1200, 0.004, 9), 16, 4),
]


@pytest.mark.parametrize("K", [2, 5, 32])
@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("name,make,bs,w", CASES, ids=[c[0] for c in CASES])
def test_apply_multi_rhs(torch, orc, name, make, bs, w, tile, K):
    print(f"multi-rhs apply {name} tile {tile} K {K}", flush=True)
    A = make()
    s = orc.system(A, bs, w)
    o = hbmc.hbmc_order(A, bs, w)
    f = hbmc.ic0_factor(o, A).set_rhs_tile(tile).upload()
    rng = np.random.default_rng(3 + K)
    R = rng.uniform(-1, 1, (s.ordr.n_pad, K))
    dummy = np.setdiff1d(np.arange(s.ordr.n_pad), s.ordr.perm)
    R[dummy] = 0.0
    Z = hbmc.ic0_apply(f, _dev(torch, R.ravel()), nrhs=K).cpu().numpy().reshape(-1, K)
    for q in range(K):
        zref = orc.apply(s.Ab, s.d, s.fac, R[:, q])
        assert np.linalg.norm(Z[:, q] - zref) <= 1e-13 * np.linalg.norm(zref), q
        assert np.abs(Z[:, q] - zref).max() <= 1e-12 * np.abs(zref).max(), q
    assert np.all(Z[dummy] == 0.0)


@pytest.mark.parametrize("tile", [4, 16])
def test_apply_multi_rhs_f32(torch, orc, tile):
    print(f"multi-rhs apply f32 tile {tile}", flush=True)
    A = inputs.diffusion3d(16, 1.0, 5)
    s = orc.system(A, 8, 64)
    f = hbmc.ic0_factor(hbmc.hbmc_order(A, 8, 64), A, hbmc.HBMC_F32).set_rhs_tile(tile).upload()
    K = 9
    R = np.random.default_rng(4).uniform(-1, 1, (s.ordr.n_pad, K))
    R[np.setdiff1d(np.arange(s.ordr.n_pad), s.ordr.perm)] = 0.0
    Z = hbmc.ic0_apply(f, _dev(torch, R.ravel()), nrhs=K).cpu().numpy().reshape(-1, K)
    for q in range(K):
        zref = orc.apply(s.Ab, s.d, s.fac, R[:, q], "f32")
        assert np.abs(Z[:, q] - zref).max() <= 1e-5 * np.abs(zref).max(), q


@pytest.mark.parametrize("K", [1, 3, 12])
def test_spmv_multi_rhs(torch, orc, K):
    A = inputs.knn_laplacian(2000, 13, 4, 5)
    s = orc.system(A, 4, 16)
    m = hbmc.hbmc_matrix_create(hbmc.hbmc_order(A, 4, 16), A).upload()
    X = np.random.default_rng(6).uniform(-1, 1, (s.ordr.n_pad, K))
    Y = hbmc.hbmc_spmv(m, _dev(torch, X.ravel()), nrhs=K).cpu().numpy().reshape(-1, K)
    for q in range(K):
        yref = orc.spmv(s.Ab, X[:, q])
        assert np.abs(Y[:, q] - yref).max() <= 1e-14 * np.abs(s.Ab.val).max() * np.abs(X).max() * 16


def _solve_cols(torch, sv, B, **kw):
    n, K = B.shape
    x, st = sv.solve(_dev(torch, B.ravel()), nrhs=K, **kw)
    return x.cpu().numpy().reshape(n, K), st


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("use_graph", [True, False], ids=["graph", "eager"])
def test_solve_multi_rhs_equals_single(torch, tile, use_graph):
    print(f"multi-rhs solve tile {tile} graph {use_graph}", flush=True)
    A = inputs.diffusion3d(18, 1.0, 4)
    K = 6
    B = np.stack([inputs.uniform_rhs(A.n, 70 + q) for q in range(K)], axis=1)
    B[:, 3] = 0.0                       # one zero column
    B[:, 5] = inputs.row_sums(A)        # b = A 1
    sv = hbmc.Solver.setup(A, 8, 64)
    sv.factor.set_rhs_tile(tile)
    X, sts = _solve_cols(torch, sv, B, tol=1e-9, use_graph=use_graph, check_every=4)
    assert len(sts) == K
    for q in range(K):
        if q == 3:
            assert sts[q].iters == 0 and np.all(X[:, q] == 0.0)
            continue
        x1, st1 = sv.solve(_dev(torch, B[:, q]), tol=1e-9)
        x1 = x1.cpu().numpy()
        assert sts[q].status == hbmc.HBMC_OK and sts[q].iters == st1.iters, q
        assert np.linalg.norm(X[:, q] - x1) <= 1e-12 * np.linalg.norm(x1), q
    assert np.abs(X[:, 5] - 1.0).max() < 1e-6


def test_batch_with_multi_rhs(torch):
    """Two systems, three right-hand sides each: stats are system-major and
    every (system, column) equals its own single solve."""
    print("batch x multi-rhs", flush=True)
    mats = [inputs.poisson3d(9), inputs.diffusion3d(11, 1.0, 6)]
    A, sys_ptr = inputs.block_diag(mats)
    K = 3
    B = np.random.default_rng(8).uniform(-1, 1, (A.n, K))
    sv = hbmc.Solver.setup(A, 8, 64, sys_ptr=sys_ptr)
    X, sts = _solve_cols(torch, sv, B, tol=1e-9)
    assert len(sts) == 2 * K
    for s, M in enumerate(mats):
        one = hbmc.Solver.setup(M, 8, 64)
        for q in range(K):
            x1, st1 = one.solve(_dev(torch, B[sys_ptr[s]: sys_ptr[s + 1], q]), tol=1e-9)
            x1 = x1.cpu().numpy()
            st = sts[s * K + q]
            assert st.iters == st1.iters, (s, q)
            assert np.linalg.norm(X[sys_ptr[s]: sys_ptr[s + 1], q] - x1) <= 1e-12 * np.linalg.norm(x1)



@pytest.mark.parametrize("K", [16, 32, 40, 64])
def test_solve_many_rhs_vector_tiles(torch, K):
    """K from 16 to 64 right-hand sides: the vector kernels cover whole rows
    per wavefront (16, 32, 64 per wavefront; 40 leaves lanes idle); every
    column equals its single-vector solve."""
    print(f"many-rhs solve K {K}", flush=True)
    A = inputs.diffusion3d(10, 1.0, 8)
    B = np.stack([inputs.uniform_rhs(A.n, 900 + q) for q in range(K)], axis=1)
    sv = hbmc.Solver.setup(A, 4, 16)
    X, sts = _solve_cols(torch, sv, B, tol=1e-9)
    for q in range(0, K, 7):
        x1, st1 = sv.solve(_dev(torch, B[:, q]), tol=1e-9)
        x1 = x1.cpu().numpy()
        assert sts[q].iters == st1.iters, q
        assert np.linalg.norm(X[:, q] - x1) <= 1e-12 * np.linalg.norm(x1), q
    assert all(st.status == hbmc.HBMC_OK and st.true_rel_res < 1e-8 for st in sts)

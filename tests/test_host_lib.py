"""Host side of the library against the oracle (no GPU needed).

- the C ABI loads and exports every function include/hbmc.h declares;
- hbmc_order is bit-exact with the oracle's ordering (perm, color starts,
  color count, n_pad) on every workload shape and on ragged/random graphs;
- the IC(0) factor agrees with the oracle's to 1e-14 (FP64);
- error paths return the documented status codes.
"""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1908_00741_amd import hbmc, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_mlp_symbol():
    from paper_1908_00741_amd import mlp
    header = open(os.path.join(ROOT, "include", "hbmc_mlp.h")).read()
    header = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    declared = set(re.findall(r"\b(mlp_[a-z0-9_]+)\s*\(", header))
    assert declared == set(mlp.SYMBOLS)
    L = mlp.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_mlp_gemm_rejects_short_leading_dimensions():
    """Argument errors come back before any launch: host buffers stand in
    for the operands and are never read."""
    import ctypes as C
    from paper_1908_00741_amd import mlp
    L = mlp.lib()
    buf = (C.c_float * 64)()
    p = C.cast(buf, C.c_void_p)
    M, N, K = 8, 16, 4
    # (layout, lda, ldb, ldc): each one short of its row width by one
    for layout, lda, ldb, ldc in [(mlp.MLP_NN, K - 1, N, N), (mlp.MLP_NN, K, N - 1, N), (mlp.MLP_NN, K, N, N - 1),
                                  (mlp.MLP_TN, M - 1, N, N), (mlp.MLP_NT, K, K - 1, N), (7, K, N, N)]:
        code = L.mlp_gemm(mlp.MLP_BF16, layout, M, N, K, p, lda, p, ldb, p, ldc, 1, None)
        assert code == hbmc.HBMC_EINVAL, (layout, lda, ldb, ldc)


def test_mlp_train_step_rejects_bad_arguments():
    """Argument errors of the fused training step come back before any
    launch (host buffers stand in for device arrays and are never read)."""
    import ctypes as C
    from paper_1908_00741_amd import mlp
    L = mlp.lib()
    buf = (C.c_float * 64)()
    p = C.cast(buf, C.c_void_p)
    six = (C.c_void_p * 6)(*([p.value] * 6))
    holed = (C.c_void_p * 6)(*([p.value] * 3 + [None] + [p.value] * 2))

    def call(w=six, m=six, v=six, g=six, wc=six, step=1, dtype=mlp.MLP_BF16, M=4, work_bytes=1 << 40):
        return L.mlp_train_step(dtype, M, 12, 256, 64, p, p, w, m, v, g, wc, 1e-3, 0.9, 0.999, 1e-8, step, p, p,
                                work_bytes, None)
    assert call(step=0) == hbmc.HBMC_EINVAL
    assert call(m=holed) == hbmc.HBMC_EINVAL
    assert call(wc=(C.c_void_p * 6)(*([p.value] * 4 + [None, p.value]))) == hbmc.HBMC_EINVAL   # W3 copy missing
    assert call(dtype=7) == hbmc.HBMC_EINVAL
    assert call(M=0) == hbmc.HBMC_EINVAL
    assert call(work_bytes=16) == hbmc.HBMC_EINVAL
    assert call(w=None) == hbmc.HBMC_EINVAL


def test_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "hbmc.h")).read()
    header = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    declared = set(re.findall(r"\b([a-z0-9_]+)\s*\(", header)) - {"defined"}
    declared = {d for d in declared if d.startswith(("hbmc_", "ic0_", "iccg_", "ssor_"))}
    assert declared == set(hbmc.SYMBOLS)
    L = hbmc.lib()
    for name in declared:
        assert hasattr(L, name), name


CASES = [
    ("c1_grid64", lambda: inputs.grid2d_5pt(64), 4, 8),
    ("grid_ragged", lambda: inputs.grid2d_5pt(37, 11), 4, 8),
    ("diff3d_20", lambda: inputs.diffusion3d(20, 1.0, 2), 8, 64),
    ("diff3d_13_bs4", lambda: inputs.diffusion3d(13, 0.5, 3), 4, 16),
    ("knn_5000", lambda: inputs.knn_laplacian(5000, 13, 4, 5), 8, 64),
    ("random", lambda: inputs.random_spd(777, 0.01, 6), 5, 4),
    ("random_bs1", lambda: inputs.random_spd(300, 0.02, 7), 1, 64),
    ("random_bs32", lambda: inputs.random_spd(1000, 0.005, 8), 32, 2),
    ("path", lambda: inputs.path_1d(101), 4, 8),
    ("single", lambda: inputs.path_1d(1), 8, 64),
]


@pytest.mark.parametrize("name,make,bs,w", CASES, ids=[c[0] for c in CASES])
def test_order_bit_exact(orc, name, make, bs, w):
    A = make()
    o = hbmc.hbmc_order(A, bs, w)
    ref = orc.order(A, bs, w)
    perm, cs = o.perm()
    assert o.n_colors == ref.ncolors
    assert o.n_pad == ref.n_pad
    assert o.n_blocks == ref.nblocks
    assert np.array_equal(cs, ref.color_start)
    assert np.array_equal(perm, ref.perm)


@pytest.mark.parametrize("name,make,bs,w", CASES, ids=[c[0] for c in CASES])
def test_rcm_order_bit_exact(orc, name, make, bs, w):
    """The reverse Cuthill-McKee numbering and the ordering of the renumbered
    system (hbmc_rcm, hbmc_order_rcm) against the oracle's: same numbering,
    same permutation in the input's numbering, same color starts."""
    A = make()
    assert np.array_equal(hbmc.hbmc_rcm(A), orc.rcm(A))
    o = hbmc.hbmc_order(A, bs, w, rcm=True)
    ref = orc.order_rcm(A, bs, w)
    perm, cs = o.perm()
    assert (o.n_colors, o.n_pad, o.n_blocks) == (ref.ncolors, ref.n_pad, ref.nblocks)
    assert np.array_equal(cs, ref.color_start) and np.array_equal(perm, ref.perm)


def test_rcm_order_bit_exact_knn_100k(orc):
    """The unstructured workload at 100,000 points (bs 2, w 32): the
    renumbered ordering bit-exact, with fewer colors than the shuffled
    numbering's and the factor built on it against the oracle's."""
    A = inputs.knn_laplacian(100_000, 13, 4, 5, shift=1e-3)
    o = hbmc.hbmc_order(A, 2, 32, rcm=True)
    ref = orc.order_rcm(A, 2, 32)
    perm, cs = o.perm()
    assert np.array_equal(perm, ref.perm) and np.array_equal(cs, ref.color_start)
    assert o.n_colors <= hbmc.hbmc_order(A, 2, 32).n_colors
    d, rp, ci, v = hbmc.ic0_factor(o, A).export()
    Ab = orc.permute(A, ref.perm, ref.n_pad)
    dref, fac = orc.ic0(Ab)
    Lref = sp.tril(sp.csr_matrix((fac, Ab.col, Ab.rowptr), shape=(Ab.n, Ab.n)), k=-1).tocsr()
    Lref.sort_indices()
    assert np.array_equal(rp, Lref.indptr) and np.array_equal(ci, Lref.indices)
    assert np.allclose(v, Lref.data, rtol=1e-14, atol=0) and np.allclose(d, dref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("N,sigma,seed", [(128, 1.0, 2), (96, 0.5, 10)])
def test_order_bit_exact_full_size_grids(orc, N, sigma, seed):
    """The 128^3 (sigma 1) and 96^3 (sigma 0.5) diffusion workloads at full size."""
    A = inputs.diffusion3d(N, sigma, seed)
    o = hbmc.hbmc_order(A, 8, 64)
    ref = orc.order(A, 8, 64)
    perm, cs = o.perm()
    assert np.array_equal(perm, ref.perm) and np.array_equal(cs, ref.color_start)


def test_order_bit_exact_full_size_knn(orc):
    """The 1M-point 13-NN Laplacian in its timed configuration (bs 2, w 32):
    ordering bit-exact, and the factor (IC(0) with off-diagonal updates on
    this graph) against the oracle's."""
    A = inputs.knn_laplacian(1_000_000, 13, 4, 5, shift=1e-3)
    o = hbmc.hbmc_order(A, 2, 32)
    ref = orc.order(A, 2, 32)
    perm, cs = o.perm()
    assert o.n_colors == ref.ncolors and o.n_pad == ref.n_pad
    assert np.array_equal(perm, ref.perm) and np.array_equal(cs, ref.color_start)
    d, rp, ci, v = hbmc.ic0_factor(o, A).export()
    Ab = orc.permute(A, ref.perm, ref.n_pad)
    dref, fac = orc.ic0(Ab)
    Lref = sp.tril(sp.csr_matrix((fac, Ab.col, Ab.rowptr), shape=(Ab.n, Ab.n)), k=-1).tocsr()
    Lref.sort_indices()
    assert np.array_equal(rp, Lref.indptr) and np.array_equal(ci, Lref.indices)
    assert np.allclose(v, Lref.data, rtol=1e-14, atol=0)
    assert np.allclose(d, dref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("name,make,bs,w", CASES[:8], ids=[c[0] for c in CASES[:8]])
def test_factor_matches_oracle(orc, name, make, bs, w):
    A = make()
    o = hbmc.hbmc_order(A, bs, w)
    f = hbmc.ic0_factor(o, A)
    d, rp, ci, v = f.export()
    s = orc.system(A, bs, w)
    Ab = sp.csr_matrix((s.fac, s.Ab.col, s.Ab.rowptr), shape=(s.Ab.n, s.Ab.n))
    Lref = sp.tril(Ab, k=-1).tocsr()
    Lref.sort_indices()
    assert np.array_equal(rp, Lref.indptr) and np.array_equal(ci, Lref.indices)
    assert np.allclose(v, Lref.data, rtol=1e-14, atol=0)
    assert np.allclose(d, s.d, rtol=1e-14, atol=0)


def test_factor_shift(orc):
    A = inputs.random_spd(200, 0.03, 3)
    o = hbmc.hbmc_order(A, 4, 8)
    d, *_ = hbmc.ic0_factor(o, A, shift=0.3).export()
    s = orc.system(A, 4, 8, shift=0.3)
    assert np.allclose(d, s.d, rtol=1e-14, atol=0)


@pytest.mark.parametrize("omega", [1.0, 1.3])
@pytest.mark.parametrize("name,make,bs,w", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_ssor_factor_matches_oracle(orc, name, make, bs, w, omega):
    """The SSOR splitting is bit-exact: L is Abar's strict lower part and
    d = abar_ii / omega, one rounding each on both sides."""
    A = make()
    f = hbmc.ssor_factor(hbmc.hbmc_order(A, bs, w), A, omega=omega)
    d, rp, ci, v = f.export()
    s = orc.system(A, bs, w)
    dref, fac = orc.core.ssor_split(s.Ab, omega)
    L = sp.tril(sp.csr_matrix((fac, s.Ab.col, s.Ab.rowptr), shape=(s.Ab.n, s.Ab.n)), k=-1).tocsr()
    L.sort_indices()
    assert np.array_equal(rp, L.indptr) and np.array_equal(ci, L.indices)
    assert np.array_equal(v, L.data) and np.array_equal(d, dref)


def test_revalue_create():
    """Pattern data for device refactorization: host-only construction and
    its CSR checks."""
    A = inputs.diffusion3d(10, 1.0, 2)
    o = hbmc.hbmc_order(A, 8, 16)
    rv = hbmc.Revalue(o, A)
    assert rv.nnz == int(A.rowptr[-1])
    col = A.col.copy()
    col[[0, 1]] = col[[1, 0]]
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.Revalue(o, inputs.CSR(A.n, A.rowptr, col, A.val))
    assert e.value.code == hbmc.HBMC_EINVAL


def test_ssor_factor_errors():
    A = inputs.grid2d_5pt(6)
    o = hbmc.hbmc_order(A, 4, 8)
    for bad in (0.0, 2.0, -0.5, float("nan")):
        with pytest.raises(hbmc.HbmcError) as e:
            hbmc.ssor_factor(o, A, omega=bad)
        assert e.value.code == hbmc.HBMC_EINVAL
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.ssor_factor(o, _bad(A, p0=-1.0))    # negative diagonal
    assert e.value.code == hbmc.HBMC_EDIAG


@pytest.mark.parametrize("name,make,bs,w", [
    ("diff3d_40_bs8_w64", lambda: inputs.diffusion3d(40, 1.0, 2), 8, 64),
    ("knn_40000_bs4_w16", lambda: inputs.knn_laplacian(40000, 13, 4, 5), 4, 16),
    ("random_bs2_w32", lambda: inputs.random_spd(30000, 0.0002, 8), 2, 32),
    ("grid_ragged_bs4_w8", lambda: inputs.grid2d_5pt(301, 257), 4, 8),
])
def test_setup_independent_of_threads(name, make, bs, w):
    """The parallel setup (chunks joined in order, colors in turn) gives the
    same device images, bit for bit, for any number of threads; the kNN case
    has off-diagonal IC(0) updates inside level-1 blocks and across colors."""
    A = make()
    images = []
    try:
        for t in (1, 3, 8):
            hbmc.set_num_threads(t)
            o = hbmc.hbmc_order(A, bs, w)
            images.append((hbmc.ic0_factor(o, A).image(), hbmc.ssor_factor(o, A, omega=1.3).image(),
                            hbmc.hbmc_matrix_create(o, A).image(), o.perm()[0]))
    finally:
        hbmc.set_num_threads(0)
    for other in images[1:]:
        for a, b in zip(images[0], other):
            assert np.array_equal(a, b)


def test_setup_threads_batch():
    mats = [inputs.poisson3d(n) for n in (9, 14, 11)]
    A, sys_ptr = inputs.block_diag(mats)
    images = []
    try:
        for t in (1, 5):
            hbmc.set_num_threads(t)
            o = hbmc.hbmc_order_batch(A, sys_ptr, 4, 16)
            images.append((hbmc.ic0_factor(o, A).image(), hbmc.hbmc_matrix_create(o, A).image()))
    finally:
        hbmc.set_num_threads(0)
    assert all(np.array_equal(a, b) for a, b in zip(*images))
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.set_num_threads(-1)
    assert e.value.code == hbmc.HBMC_EINVAL


def _bad(A, **kw):
    v = A.val.copy()
    for k, x in kw.items():
        v[int(k[1:])] = x
    return inputs.CSR(A.n, A.rowptr, A.col, v)


def test_errors():
    A = inputs.grid2d_5pt(6)
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.hbmc_order(A, 0, 8)
    assert e.value.code == hbmc.HBMC_EINVAL
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.hbmc_order(A, 4, 3)          # w must divide 64
    assert e.value.code == hbmc.HBMC_EINVAL
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.hbmc_order(A, 33, 8)
    assert e.value.code == hbmc.HBMC_EINVAL
    o = hbmc.hbmc_order(A, 4, 8)
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.ic0_factor(o, _bad(A, p1=-0.25))   # value asymmetry
    assert e.value.code == hbmc.HBMC_ENOTSYM
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.ic0_factor(o, _bad(A, p0=-1.0))    # negative diagonal
    assert e.value.code == hbmc.HBMC_EDIAG
    # pattern asymmetry: drop one off-diagonal entry
    S = A.to_scipy().tolil()
    S[0, 1] = 0
    S = S.tocsr(); S.eliminate_zeros()
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.hbmc_order(inputs.from_scipy(S), 4, 8)
    assert e.value.code == hbmc.HBMC_ENOTSYM
    # missing diagonal
    S = A.to_scipy().tolil()
    S[3, 3] = 0
    S = S.tocsr(); S.eliminate_zeros()
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.hbmc_order(inputs.from_scipy(S), 4, 8)
    assert e.value.code == hbmc.HBMC_EDIAG
    # unsorted columns
    col = A.col.copy()
    col[[0, 1]] = col[[1, 0]]
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.hbmc_order(inputs.CSR(A.n, A.rowptr, col, A.val), 4, 8)
    assert e.value.code == hbmc.HBMC_EINVAL


def test_breakdown():
    A = inputs.from_scipy(sp.csr_matrix(np.array([[1.0, 2.0], [2.0, 1.0]])))
    o = hbmc.hbmc_order(A, 1, 1)
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.ic0_factor(o, A)
    assert e.value.code == hbmc.HBMC_EBREAKDOWN


def test_rhs_tile_errors():
    A = inputs.grid2d_5pt(8)
    f = hbmc.ic0_factor(hbmc.hbmc_order(A, 4, 8), A)
    for ok in (0, 4, 8, 16):
        f.set_rhs_tile(ok)
    for bad in (1, 2, 3, 32, -1):
        with pytest.raises(hbmc.HbmcError) as e:
            f.set_rhs_tile(bad)
        assert e.value.code == hbmc.HBMC_EINVAL


def test_one_launch_settings_and_workspace_size():
    """The synchronization and wait-limit settings take their documented
    values only; ic0_apply_ws's workspace is the 256-byte error-word head
    plus one FP64 value per padded row."""
    A = inputs.knn_laplacian(3000, 13, 4, 5)
    o = hbmc.hbmc_order(A, 2, 32)
    f = hbmc.ic0_factor(o, A)
    assert f.apply_ws_bytes() == 256 + 8 * o.n_pad
    for ok in (hbmc.HBMC_SYNC_AUTO, hbmc.HBMC_SYNC_LAUNCH):
        f.set_sync(ok)
    for ok in (0, 1, 50_000, 60_000_000):
        f.set_wait_limit(ok)
    for bad, setter in ((2, f.set_sync), (-1, f.set_sync), (-1, f.set_wait_limit),
                        (60_000_001, f.set_wait_limit)):
        with pytest.raises(hbmc.HbmcError) as e:
            setter(bad)
        assert e.value.code == hbmc.HBMC_EINVAL


@pytest.mark.parametrize("name,make,bs,w,rcm", [
    ("knn_20000_bs2_w32", lambda: inputs.knn_laplacian(20000, 13, 4, 5, shift=1e-3), 2, 32, False),
    ("knn_20000_bs2_w32_rcm", lambda: inputs.knn_laplacian(20000, 13, 4, 5, shift=1e-3), 2, 32, True),
    ("knn_3000_bs4_w8", lambda: inputs.knn_laplacian(3000, 13, 6, 7), 4, 8, False),
    ("grid_ragged_bs4_w8", lambda: inputs.grid2d_5pt(37, 11), 4, 8, False),
    ("random_bs1_w64", lambda: inputs.random_spd(1500, 0.004, 7), 1, 64, False),
], ids=lambda v: v if isinstance(v, str) else "")
def test_one_launch_waits_only_on_earlier_phases(name, make, bs, w, rcm):
    """What makes the one-launch substitution's waits end: in the factor the
    library builds, every coupling of a row to another level-1 block belongs
    to an earlier color (the forward sweep waits on its y) -- so, U being
    L's transpose, the backward sweep waits only on later colors' z -- and
    couplings inside a color stay inside one level-1 block, where the chain
    computes them without a wait.  The phase order (forward colors up, then
    backward colors down) therefore puts every awaited value in an earlier
    phase."""
    A = make()
    o = hbmc.hbmc_order(A, bs, w, rcm=rcm)
    _, cs = o.perm()
    _, rp, ci, _ = hbmc.ic0_factor(o, A).export()
    rows = np.repeat(np.arange(o.n_pad), np.diff(rp))
    color = np.searchsorted(cs, np.arange(o.n_pad), side="right") - 1
    local = np.arange(o.n_pad) - cs[color]
    block = (color.astype(np.int64) << 40) | ((local // (bs * w)) << 16) | (local % w)   # level-1 block id
    ci = ci.astype(np.int64)
    assert np.all(ci < rows)                                   # strictly lower
    earlier = color[ci] < color[rows]
    same_block = block[ci] == block[rows]
    assert np.all(earlier | same_block), name
    assert np.all(color[ci] <= color[rows])
    step = (local // w) % bs                                   # in-block: an earlier step of the chain
    assert np.all(step[ci][same_block] < step[rows][same_block])

"""iccg_solve_noalloc (the solve whose workspace is the library's static
device array) against iccg_solve with a caller-allocated workspace, through
the C ABI.

The two run the same kernels in the same order on the same inputs, so the
solutions and statistics must be the same bits.  Two calls in a row, the
second on a smaller system (the scratch keeps the first call's contents;
the solve must clear what starts at zero), then a graph Laplacian whose
substitution runs its color phases in one launch (its forward values and
empty markers live in the scratch too), then the first system again.
Argument errors (workspace larger than the scratch, graph replay, residual
history) come back before any device work.
"""
import numpy as np
import pytest

from paper_1908_00741_amd import hbmc, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


def _pair(torch, solver, b, nrhs, tol, maxit):
    """(x, stats) of iccg_solve (eager launches, caller workspace) and of
    iccg_solve_noalloc on the same right-hand sides, both from x0 = 0."""
    f, m = solver.factor, solver.matrix
    x_ref, st_ref = hbmc.iccg_solve(f, m, b, None, tol=tol, maxit=maxit, nrhs=nrhs, use_graph=False)
    x = torch.full_like(b, float("nan"))         # ignored: x0_zero
    st = hbmc.iccg_solve_noalloc(f, m, b, x, tol=tol, maxit=maxit, nrhs=nrhs, x0_zero=True)
    torch.cuda.synchronize()
    return x_ref.cpu().numpy(), st_ref, x.cpu().numpy(), st


def _same(x_ref, st_ref, x, st):
    assert np.array_equal(x, x_ref), np.abs(x - x_ref).max()
    st_ref = st_ref if isinstance(st_ref, list) else [st_ref]
    st = st if isinstance(st, list) else [st]
    for a, c in zip(st_ref, st):
        assert (a.iters, a.status) == (c.iters, c.status)
        assert a.rel_res == c.rel_res and a.true_rel_res == c.true_rel_res


def test_noalloc_matches_iccg_solve_twice(torch):
    big = inputs.diffusion3d(40, 1.0, 2)              # 64,000 unknowns, bs 8, w 64
    small = inputs.grid2d_5pt(64)                     # 4,096 unknowns, bs 4, w 8
    s_big = hbmc.Solver.setup(big, 8, 64)
    s_small = hbmc.Solver.setup(small, 4, 8)
    b_big = _dev(torch, inputs.uniform_rhs(big.n, 3))
    rng = np.random.default_rng(5)
    b_small = _dev(torch, rng.uniform(-1, 1, (small.n, 3)).reshape(-1))
    print("case noalloc diffusion40 nrhs 1", flush=True)
    x_ref, st_ref, x, st = _pair(torch, s_big, b_big, 1, 1e-7, 10000)
    assert st.status == hbmc.HBMC_OK and st.true_rel_res < 1.5e-7
    _same(x_ref, st_ref, x, st)
    print("case noalloc grid64 nrhs 3", flush=True)
    x_ref, st_ref, x, st = _pair(torch, s_small, b_small, 3, 1e-7, 10000)
    assert all(s.status == hbmc.HBMC_OK for s in st)
    _same(x_ref, st_ref, x, st)
    print("case noalloc knn20000 nrhs 1 (row kernel, color phases in one launch)", flush=True)
    knn = inputs.knn_laplacian(20000, 13, 4, 5, shift=1e-3)   # bs 2, w 32: row kernel, one launch
    s_knn = hbmc.Solver.setup(knn, 2, 32)
    x_ref, st_ref, x, st = _pair(torch, s_knn, _dev(torch, inputs.uniform_rhs(knn.n, 6)), 1, 1e-7, 10000)
    assert st.status == hbmc.HBMC_OK and st.true_rel_res < 1.5e-7
    _same(x_ref, st_ref, x, st)
    print("case noalloc diffusion40 again, maxit 7", flush=True)
    x_ref, st_ref, x, st = _pair(torch, s_big, b_big, 1, 1e-7, 7)
    assert st.status == hbmc.HBMC_ENOCONV and st.iters == 7
    _same(x_ref, st_ref, x, st)


def test_noalloc_rejects_before_device_work(torch):
    A = inputs.diffusion3d(48, 1.0, 2)                # 110,592 unknowns
    s = hbmc.Solver.setup(A, 8, 64)
    nrhs = 12                                         # 7 vectors of [n][12] FP64: 74 MB > 64 MiB
    b = torch.zeros(A.n * nrhs, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.iccg_solve_noalloc(s.factor, s.matrix, b, x, nrhs=nrhs)
    assert e.value.code == hbmc.HBMC_EINVAL and "scratch" in str(e.value)
    L = hbmc.lib()
    import ctypes as C
    b1 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    for opts in (hbmc.SolveOpts(1, 0, 1, 0), hbmc.SolveOpts(1, 0, 0, 1)):
        st = (hbmc.SolveStats * 1)()
        code = L.iccg_solve_noalloc(s.factor.handle, s.matrix.handle, C.c_void_p(b1.data_ptr()),
                                    C.c_void_p(x.data_ptr()), 1, 1e-7, 100, C.byref(opts), st, None)
        assert code == hbmc.HBMC_EINVAL

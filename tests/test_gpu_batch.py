"""GPU parity for batches of independent systems (hbmc_order_batch).

Bars:
- ic0_apply on a batch, FP64: as for one system (1e-13 in norm, 1e-12 per
  entry against the oracle's substitution on the permuted batch); FP32:
  1e-5 of max|z_ref| against the oracle's FP32 substitution;
- iccg_solve on a batch, FP64: every system takes the iteration count it
  takes when solved alone with the same kernel, and its solution agrees
  with the one-by-one solution to 1e-12 relative (with w = 64 the
  reductions see the same partial sums in the same order);
- the same with the FP32 preconditioner: +-1 iteration and 1e-9 relative.
  The batch may run another register/LDS variant of the substitution than
  the system alone (the variant follows the largest number of couplings per
  step over all systems), which rounds the FP32 products in another order;
  the FP64 CG then follows a different FP32 rounding of the same
  preconditioner, and its iterates differ at about the FP32 rounding of
  M^-1 r times the reduction CG makes per iteration, well below 1e-9;
- against the oracle's FP64 PCG of each system alone: 1e-10 relative and the
  oracle's iteration count +-1;
- systems with b = 0 return x = 0 after 0 iterations while the others
  converge; a maxit that stops some systems stops only those.
"""
import numpy as np
import pytest

from paper_1908_00741_amd import hbmc, inputs

pytestmark = pytest.mark.gpu

KERNELS = [hbmc.HBMC_KERNEL_SWEEP, hbmc.HBMC_KERNEL_ROWS]
KIDS = ["sweep", "rows"]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


def _mats():
    return [inputs.diffusion3d(14, 1.0, 2), inputs.poisson3d(9), inputs.grid2d_5pt(40, 23),
            inputs.knn_laplacian(2500, 13, 4, 5, shift=1e-3), inputs.diffusion3d(6, 0.5, 3),
            inputs.path_1d(7), inputs.poisson3d(17)]


def _rhs(mats, seed):
    return [inputs.uniform_rhs(M.n, seed + s) for s, M in enumerate(mats)]


@pytest.mark.parametrize("kernel", KERNELS, ids=KIDS)
@pytest.mark.parametrize("precision", [hbmc.HBMC_F64, hbmc.HBMC_F32], ids=["f64", "f32"])
@pytest.mark.parametrize("bs,w", [(8, 64), (4, 16)])
def test_batch_apply(torch, orc, bs, w, precision, kernel):
    print(f"batch apply bs {bs} w {w} precision {precision} kernel {kernel}", flush=True)
    mats = _mats()
    A, sys_ptr = inputs.block_diag(mats)
    ref = orc.order_batch(mats, bs, w)
    Ab = orc.permute(A, ref.perm, ref.n_pad)
    d, fac = orc.ic0(Ab)
    o = hbmc.hbmc_order_batch(A, sys_ptr, bs, w)
    f = hbmc.ic0_factor(o, A, precision).set_kernel(kernel).upload()
    r = np.random.default_rng(9).uniform(-1, 1, ref.n_pad)
    dummy = np.setdiff1d(np.arange(ref.n_pad), ref.perm)
    r[dummy] = 0.0
    z = hbmc.ic0_apply(f, _dev(torch, r)).cpu().numpy()
    if precision == hbmc.HBMC_F64:
        zref = orc.apply(Ab, d, fac, r)
        assert np.linalg.norm(z - zref) <= 1e-13 * np.linalg.norm(zref)
        assert np.abs(z - zref).max() <= 1e-12 * np.abs(zref).max()
    else:
        zref = orc.apply(Ab, d, fac, r, "f32")
        assert np.abs(z - zref).max() <= 1e-5 * np.abs(zref).max()
    assert np.all(z[dummy] == 0.0)


def _solve_batch(torch, mats, rhs, bs, w, precision, kernel, **kw):
    A, sys_ptr = inputs.block_diag(mats)
    sv = hbmc.Solver.setup(A, bs, w, precision, kernel=kernel, sys_ptr=sys_ptr)
    x, st = sv.solve(_dev(torch, np.concatenate(rhs)), **kw)
    x = x.cpu().numpy()
    return [x[sys_ptr[s]: sys_ptr[s + 1]] for s in range(len(mats))], st


def _solve_alone(torch, M, b, bs, w, precision, kernel, **kw):
    sv = hbmc.Solver.setup(M, bs, w, precision, kernel=kernel)
    x, st = sv.solve(_dev(torch, b), **kw)
    return x.cpu().numpy(), st


@pytest.mark.parametrize("kernel", KERNELS, ids=KIDS)
@pytest.mark.parametrize("precision", [hbmc.HBMC_F64, hbmc.HBMC_F32], ids=["f64", "f32"])
def test_batch_solve_equals_one_by_one(torch, kernel, precision):
    print(f"batch solve kernel {kernel} precision {precision}", flush=True)
    mats = _mats()
    rhs = _rhs(mats, 30)
    xs, sts = _solve_batch(torch, mats, rhs, 8, 64, precision, kernel, tol=1e-8)
    assert len(sts) == len(mats)
    for s, M in enumerate(mats):
        x1, st1 = _solve_alone(torch, M, rhs[s], 8, 64, precision, kernel, tol=1e-8)
        assert sts[s].status == hbmc.HBMC_OK and st1.status == hbmc.HBMC_OK
        if precision == hbmc.HBMC_F64:
            assert sts[s].iters == st1.iters, s
            assert np.linalg.norm(xs[s] - x1) <= 1e-12 * np.linalg.norm(x1), s
        else:
            assert abs(sts[s].iters - st1.iters) <= 1, s
            assert np.linalg.norm(xs[s] - x1) <= 1e-9 * np.linalg.norm(x1), s
        assert sts[s].true_rel_res < 1e-7


def test_batch_solve_matches_oracle(torch, orc):
    print("batch solve vs oracle bs 4 w 16", flush=True)
    mats = _mats()
    rhs = _rhs(mats, 40)
    xs, sts = _solve_batch(torch, mats, rhs, 4, 16, hbmc.HBMC_F64, hbmc.HBMC_KERNEL_AUTO, tol=1e-9)
    for s, M in enumerate(mats):
        res = orc.system(M, 4, 16).solve(rhs[s], tol=1e-9)
        assert abs(sts[s].iters - res.iters) <= 1, s
        assert np.linalg.norm(xs[s] - res.x) <= 1e-10 * np.linalg.norm(res.x), s


@pytest.mark.parametrize("use_graph", [True, False], ids=["graph", "eager"])
def test_batch_zero_rhs_and_maxit(torch, use_graph):
    print(f"batch zero rhs / maxit graph={use_graph}", flush=True)
    mats = _mats()
    rhs = _rhs(mats, 50)
    rhs[2] = np.zeros(mats[2].n)
    xs, sts = _solve_batch(torch, mats, rhs, 8, 64, hbmc.HBMC_F64, hbmc.HBMC_KERNEL_AUTO,
                           tol=1e-8, use_graph=use_graph, check_every=4)
    assert sts[2].iters == 0 and sts[2].status == hbmc.HBMC_OK and np.all(xs[2] == 0.0)
    iters = [st.iters for st in sts]
    for s in range(len(mats)):
        if s != 2:
            assert sts[s].status == hbmc.HBMC_OK and sts[s].true_rel_res < 1e-7
    # a maxit between the smallest and largest counts stops only the slow systems
    cap = sorted(i for i in iters if i > 0)[len(mats) // 2]
    xs2, sts2 = _solve_batch(torch, mats, rhs, 8, 64, hbmc.HBMC_F64, hbmc.HBMC_KERNEL_AUTO,
                             tol=1e-8, maxit=cap, use_graph=use_graph, check_every=4)
    for s in range(len(mats)):
        if iters[s] <= cap:
            assert sts2[s].iters == iters[s] and sts2[s].status == hbmc.HBMC_OK, s
            assert np.array_equal(xs2[s], xs[s]), s
        else:
            assert sts2[s].iters == cap and sts2[s].status == hbmc.HBMC_ENOCONV, s


def test_batch_graph_equals_eager(torch):
    print("batch graph vs eager", flush=True)
    mats = _mats()
    rhs = _rhs(mats, 60)
    xg, sg = _solve_batch(torch, mats, rhs, 8, 64, hbmc.HBMC_F64, hbmc.HBMC_KERNEL_AUTO,
                          tol=1e-8, use_graph=True, check_every=6)
    xe, se = _solve_batch(torch, mats, rhs, 8, 64, hbmc.HBMC_F64, hbmc.HBMC_KERNEL_AUTO,
                          tol=1e-8, use_graph=False, check_every=1)
    for s in range(len(mats)):
        assert sg[s].iters == se[s].iters
        assert np.array_equal(xg[s], xe[s])

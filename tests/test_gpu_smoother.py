"""GPU parity of the SOR / Gauss-Seidel smoother and SSOR-preconditioned CG
(the GS and SOR steps of Section 2 on the HBMC substitution kernels),
through the C ABI, against the oracle's literal sweeps.

Bars:
- ic0_apply with the SSOR splitting: as for IC(0), ||z - z_ref|| / ||z_ref||
  <= 1e-13 (only the summation order differs);
- hbmc_smooth: the library takes each step in correction form
  x + c M^-1 (b - A x), the oracle sweeps one unknown at a time; the two are
  the same map up to rounding, and with contraction factors below 1 the
  rounding differences stay at a few ulps of the iterates per step:
  ||x - x_ref|| / ||x_ref|| <= 1e-12 after a few steps;
- SSOR-PCG at a fixed iteration count: 1e-10 as for IC(0)-PCG; converged
  counts within one of the oracle's;
- several right-hand sides: each column agrees with its single-vector
  smoothing to 1e-12 (the substitution may sum in another order).
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


def _host(t):
    return t.cpu().numpy()


CASES = [
    ("c1_grid64_bs4_w8", lambda: inputs.grid2d_5pt(64), 4, 8),
    ("grid_ragged_bs4_w8", lambda: inputs.grid2d_5pt(37, 11), 4, 8),
    ("diff3d_20_bs8_w64", lambda: inputs.diffusion3d(20, 1.0, 2), 8, 64),
    ("knn_3000_bs4_w8", lambda: inputs.knn_laplacian(3000, 13, 6, 7), 4, 8),
    ("random_bs1_w64_mc", lambda: inputs.random_spd(1500, 0.004, 7), 1, 64),
    ("random_bs16_w4", lambda: inputs.random_spd(2000, 0.003, 9), 16, 4),
    ("random_bs32_w2", lambda: inputs.random_spd(1200, 0.004, 10), 32, 2),
    ("random_w1_bmc", lambda: inputs.random_spd(700, 0.008, 11), 8, 1),
    ("path_short", lambda: inputs.path_1d(5), 4, 8),
]


def _setup(orc, A, bs, w, omega, precision=hbmc.HBMC_F64):
    s = orc.system(A, bs, w)
    o = hbmc.hbmc_order(A, bs, w)
    f = hbmc.ssor_factor(o, A, precision, omega).upload()
    m = hbmc.hbmc_matrix_create(o, A).upload()
    dummy = np.setdiff1d(np.arange(s.ordr.n_pad), s.ordr.perm)
    return s, f, m, dummy


def _vectors(s, dummy, seed):
    rng = np.random.default_rng(seed)
    b = rng.uniform(-1, 1, s.ordr.n_pad)
    x0 = rng.uniform(-1, 1, s.ordr.n_pad)
    b[dummy] = 0.0
    x0[dummy] = 0.0
    return b, x0


@pytest.mark.parametrize("omega", [1.0, 1.5])
@pytest.mark.parametrize("name,make,bs,w", CASES, ids=[c[0] for c in CASES])
def test_ssor_apply(torch, orc, name, make, bs, w, omega):
    print(f"case ssor_apply {name} omega {omega}", flush=True)
    A = make()
    s, f, m, dummy = _setup(orc, A, bs, w, omega)
    r, _ = _vectors(s, dummy, 1)
    z = _host(hbmc.ic0_apply(f, _dev(torch, r)))
    d, fac = orc.core.ssor_split(s.Ab, omega)
    zref = orc.core.apply(s.Ab, d, fac, r)
    assert np.linalg.norm(z - zref) <= 1e-13 * np.linalg.norm(zref)
    assert np.all(z[dummy] == 0.0)


@pytest.mark.parametrize("omega", [1.0, 1.5])
@pytest.mark.parametrize("name,make,bs,w", CASES, ids=[c[0] for c in CASES])
def test_smooth_symmetric(torch, orc, name, make, bs, w, omega):
    print(f"case smooth_sym {name} omega {omega}", flush=True)
    A = make()
    s, f, m, dummy = _setup(orc, A, bs, w, omega)
    b, x0 = _vectors(s, dummy, 2)
    x = _dev(torch, x0)
    hbmc.hbmc_smooth(f, m, _dev(torch, b), x, sweeps=3)
    x = _host(x)
    ref = orc.core.sor_sweeps(s.Ab, b, x0, omega, 3, symmetric=True)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.all(x[dummy] == 0.0)


@pytest.mark.parametrize("omega", [1.0, 1.3])
@pytest.mark.parametrize("name,make,bs,w", CASES, ids=[c[0] for c in CASES])
def test_smooth_forward(torch, orc, name, make, bs, w, omega):
    print(f"case smooth_fwd {name} omega {omega}", flush=True)
    A = make()
    s, f, m, dummy = _setup(orc, A, bs, w, omega)
    b, x0 = _vectors(s, dummy, 3)
    x = _dev(torch, x0)
    hbmc.hbmc_smooth(f, m, _dev(torch, b), x, sweeps=4, mode=hbmc.HBMC_SMOOTH_FORWARD)
    x = _host(x)
    ref = orc.core.sor_sweeps(s.Ab, b, x0, omega, 4, symmetric=False)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_ic0_smoother(torch, orc):
    """With an IC(0) factor a step is x + M_IC^-1 (b - A x)."""
    A = inputs.diffusion3d(16, 1.0, 4)
    s = orc.system(A, 8, 16)
    o = hbmc.hbmc_order(A, 8, 16)
    f = hbmc.ic0_factor(o, A).upload()
    m = hbmc.hbmc_matrix_create(o, A).upload()
    dummy = np.setdiff1d(np.arange(s.ordr.n_pad), s.ordr.perm)
    b, x0 = _vectors(s, dummy, 4)
    x = _dev(torch, x0)
    hbmc.hbmc_smooth(f, m, _dev(torch, b), x, sweeps=2)
    ref = x0.copy()
    for _ in range(2):
        ref = ref + orc.core.apply(s.Ab, s.d, s.fac, b - orc.core.spmv(s.Ab, ref))
    assert np.linalg.norm(_host(x) - ref) <= 1e-12 * np.linalg.norm(ref)


def test_smooth_edge_cases(torch, orc):
    A = inputs.grid2d_5pt(30, 17)
    s, f, m, dummy = _setup(orc, A, 4, 8, 1.2)
    b, x0 = _vectors(s, dummy, 5)
    x = _dev(torch, x0)
    hbmc.hbmc_smooth(f, m, _dev(torch, b), x, sweeps=0)
    assert np.array_equal(_host(x), x0)                         # no step: x unchanged
    z = torch.zeros(s.ordr.n_pad, dtype=torch.float64, device="cuda")
    hbmc.hbmc_smooth(f, m, torch.zeros_like(z), z, sweeps=3)
    assert not torch.any(z != 0)                                # b = 0, x = 0 stays 0
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.hbmc_smooth(f, m, x, x, sweeps=1)                   # x aliases b
    assert e.value.code == hbmc.HBMC_EINVAL
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.hbmc_smooth(f, m, _dev(torch, b), x, sweeps=1, mode=7)
    assert e.value.code == hbmc.HBMC_EINVAL
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.hbmc_smooth(f, m, _dev(torch, b), x, sweeps=-1)
    assert e.value.code == hbmc.HBMC_EINVAL
    work = hbmc.smooth_workspace(f, 1)
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.hbmc_smooth(f, m, _dev(torch, b), x, sweeps=1, work=work[: work.numel() // 2])
    assert e.value.code == hbmc.HBMC_EINVAL


def test_smooth_fp32(torch, orc):
    """FP32 splitting: the substitutions round to FP32; one step moves x by
    a correction of the size of the residual, so x stays within 1e-5 of the
    FP64 sweeps relative to max |x|."""
    A = inputs.diffusion3d(20, 1.0, 2)
    s, f, m, dummy = _setup(orc, A, 8, 64, 1.0, hbmc.HBMC_F32)
    b, x0 = _vectors(s, dummy, 6)
    x = _dev(torch, x0)
    hbmc.hbmc_smooth(f, m, _dev(torch, b), x, sweeps=2)
    ref = orc.core.sor_sweeps(s.Ab, b, x0, 1.0, 2, symmetric=True)
    assert np.max(np.abs(_host(x) - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("mode", [hbmc.HBMC_SMOOTH_SYMMETRIC, hbmc.HBMC_SMOOTH_FORWARD])
def test_smooth_multi_rhs(torch, orc, mode):
    A = inputs.diffusion3d(18, 1.0, 3)
    s, f, m, dummy = _setup(orc, A, 8, 32, 1.1)
    K = 6
    rng = np.random.default_rng(7)
    B = rng.uniform(-1, 1, (s.ordr.n_pad, K))
    X0 = rng.uniform(-1, 1, (s.ordr.n_pad, K))
    B[dummy] = 0.0
    X0[dummy] = 0.0
    X = _dev(torch, X0.ravel())
    hbmc.hbmc_smooth(f, m, _dev(torch, B.ravel()), X, sweeps=2, mode=mode, nrhs=K)
    X = _host(X).reshape(-1, K)
    for q in range(K):
        x = _dev(torch, X0[:, q])
        hbmc.hbmc_smooth(f, m, _dev(torch, B[:, q]), x, sweeps=2, mode=mode)
        xq = _host(x)
        assert np.linalg.norm(X[:, q] - xq) <= 1e-12 * np.linalg.norm(xq), q
        ref = orc.core.sor_sweeps(s.Ab, B[:, q], X0[:, q], 1.1, 2, symmetric=mode == hbmc.HBMC_SMOOTH_SYMMETRIC)
        assert np.linalg.norm(xq - ref) <= 1e-12 * np.linalg.norm(ref), q


def test_smooth_full_size_128(torch, orc):
    """128^3, bs 8, w 64: two symmetric Gauss-Seidel steps against the
    oracle's sweeps over all 2,097,152 unknowns."""
    print("case smooth_full_128", flush=True)
    A = inputs.diffusion3d(128, 1.0, 2)
    s, f, m, dummy = _setup(orc, A, 8, 64, 1.0)
    b, x0 = _vectors(s, dummy, 8)
    x = _dev(torch, x0)
    hbmc.hbmc_smooth(f, m, _dev(torch, b), x, sweeps=2)
    ref = orc.core.sor_sweeps(s.Ab, b, x0, 1.0, 2, symmetric=True)
    assert np.linalg.norm(_host(x) - ref) <= 1e-12 * np.linalg.norm(ref)


SOLVE_CASES = [
    ("diff3d_24_bs8_w16", lambda: inputs.diffusion3d(24, 1.0, 3), 8, 16),
    ("knn_3000_bs4_w8", lambda: inputs.knn_laplacian(3000, 13, 6, 7), 4, 8),
    ("random_bs1_w64_mc", lambda: inputs.random_spd(1500, 0.004, 7), 1, 64),
]


@pytest.mark.parametrize("omega", [1.0, 1.6])
@pytest.mark.parametrize("name,make,bs,w", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_ssor_pcg(torch, orc, name, make, bs, w, omega):
    print(f"case ssor_pcg {name} omega {omega}", flush=True)
    A = make()
    b = inputs.uniform_rhs(A.n, 11)
    s = orc.system(A, bs, w)
    d, fac = orc.core.ssor_split(s.Ab, omega)
    solver = hbmc.Solver.setup(A, bs, w, omega=omega)
    K = 12
    ref = orc.core.pcg(s.Ab, d, fac, s.to_hbmc(b), tol=0.0, maxit=K)
    x, st = solver.solve(_dev(torch, b), tol=0.0, maxit=K)
    assert st.iters == K
    xr = s.from_hbmc(ref.x)
    assert np.linalg.norm(_host(x) - xr) <= 1e-10 * np.linalg.norm(xr)
    ref = orc.core.pcg(s.Ab, d, fac, s.to_hbmc(b), tol=1e-7)
    x, st = solver.solve(_dev(torch, b), tol=1e-7)
    assert st.status == hbmc.HBMC_OK and abs(st.iters - ref.iters) <= 1
    assert st.true_rel_res < 1.5e-7

"""GPU: the row kernel's color phases in one launch (each tile waits for the
values of other colors it reads) against one launch per color phase.

Both forms run the same arithmetic in the same order on every row, so the
bar is bit-identical results: ic0_apply_ws against ic0_apply (whose parity
with the oracle the parity tests establish), and the CG solve with the
factor's synchronization set to automatic against the same solve with one
launch per color (iteration counts, stopping residuals and x all equal).
Every case also checks that no wait ran past its time limit (the
workspace's error word is 0).  Covered: FP64 and FP32 factors; bs 1, 2, 4
(bs 8 and above fall back to launches and must be unchanged); grids (strided
slots) and graphs (flat form with row splitting, packed slots); a ragged
last tile; the pattern renumbered by reverse Cuthill-McKee (five
workgroups per CU instead of four); the 1M-point 13-NN Laplacian at full
size; repeated calls on one workspace; the captured CG graph replayed.
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


def _rhs(torch, o, seed):
    """r uniform in [-1, 1] in HBMC order, 0 on the dummy rows."""
    r = np.random.default_rng(seed).uniform(-1, 1, o.n_pad)
    r[np.setdiff1d(np.arange(o.n_pad), o.perm()[0])] = 0.0
    return torch.from_numpy(r).cuda()


CASES = [
    ("grid64_bs4_w8", lambda: inputs.grid2d_5pt(64), 4, 8, False),
    ("grid_ragged_bs4_w8", lambda: inputs.grid2d_5pt(37, 11), 4, 8, False),
    ("diff3d_20_bs8_w16", lambda: inputs.diffusion3d(20, 1.0, 2), 8, 16, False),
    ("knn_20000_bs2_w32", lambda: inputs.knn_laplacian(20000, 13, 4, 5, shift=1e-3), 2, 32, False),
    ("knn_20000_bs2_w32_rcm", lambda: inputs.knn_laplacian(20000, 13, 4, 5, shift=1e-3), 2, 32, True),
    ("knn_6000_bs8_w64", lambda: inputs.knn_laplacian(6000, 13, 4, 5), 8, 64, False),
    ("random_bs1_w64", lambda: inputs.random_spd(1500, 0.004, 7), 1, 64, False),
    ("random_bs16_w4", lambda: inputs.random_spd(2000, 0.003, 9), 16, 4, False),
    ("random_bs32_w2", lambda: inputs.random_spd(1200, 0.004, 10), 32, 2, False),
    ("path_short", lambda: inputs.path_1d(5), 4, 8, False),
]


@pytest.mark.parametrize("precision", [hbmc.HBMC_F64, hbmc.HBMC_F32], ids=["f64", "f32"])
@pytest.mark.parametrize("name,make,bs,w,rcm", CASES, ids=[c[0] for c in CASES])
def test_apply_one_launch_matches_launches(torch, name, make, bs, w, rcm, precision):
    print(f"case {name} precision {precision}", flush=True)
    A = make()
    o = hbmc.hbmc_order(A, bs, w, rcm=rcm)
    f = hbmc.ic0_factor(o, A, precision).set_kernel(hbmc.HBMC_KERNEL_ROWS).upload()
    ws = hbmc.apply_workspace(f)
    for seed in (1, 2):   # two calls on one workspace
        r = _rhs(torch, o, seed)
        z_ref = hbmc.ic0_apply(f, r)
        z = hbmc.ic0_apply_ws(f, r, ws=ws)
        torch.cuda.synchronize()
        assert hbmc.apply_ws_error(ws) == 0
        assert torch.equal(z, z_ref), (name, seed, (z - z_ref).abs().max().item())


@pytest.mark.parametrize("rcm", [False, True], ids=["shuffled", "rcm"])
@pytest.mark.parametrize("precision", [hbmc.HBMC_F64, hbmc.HBMC_F32], ids=["f64", "f32"])
def test_apply_one_launch_knn1m(torch, precision, rcm):
    """The timed unstructured configuration at full size: 1M-point 13-NN
    Laplacian, bs 2, w 32, automatic kernel choice (rows)."""
    print(f"case knn1m precision {precision} rcm {rcm}", flush=True)
    A = inputs.knn_laplacian(1_000_000, 13, 4, 5, shift=1e-3)
    o = hbmc.hbmc_order(A, 2, 32, rcm=rcm)
    f = hbmc.ic0_factor(o, A, precision).upload()
    ws = hbmc.apply_workspace(f)
    r = _rhs(torch, o, 42)
    z_ref = hbmc.ic0_apply(f, r)
    z = hbmc.ic0_apply_ws(f, r, ws=ws)
    torch.cuda.synchronize()
    assert hbmc.apply_ws_error(ws) == 0
    assert torch.equal(z, z_ref), (z - z_ref).abs().max().item()


def _solve_pair(torch, A, bs, w, rcm=False, precision=hbmc.HBMC_F64, **kw):
    o = hbmc.hbmc_order(A, bs, w, rcm=rcm)
    f = hbmc.ic0_factor(o, A, precision).set_kernel(hbmc.HBMC_KERNEL_ROWS).upload()
    solver = hbmc.Solver(o, f, hbmc.hbmc_matrix_create(o, A).upload())
    b = torch.from_numpy(inputs.uniform_rhs(A.n, 6)).cuda()
    x1, st1 = solver.solve(b, tol=1e-7, **kw)
    f.set_sync(hbmc.HBMC_SYNC_LAUNCH)
    x0, st0 = solver.solve(b, tol=1e-7, **kw)
    torch.cuda.synchronize()
    return (x1, st1), (x0, st0)


SOLVES = [
    ("knn_20000_bs2_w32", lambda: inputs.knn_laplacian(20000, 13, 4, 5, shift=1e-3), 2, 32, False),
    ("knn_20000_bs2_w32_rcm", lambda: inputs.knn_laplacian(20000, 13, 4, 5, shift=1e-3), 2, 32, True),
    ("grid64_bs4_w8", lambda: inputs.grid2d_5pt(64), 4, 8, False),
    ("diff3d_20_bs8_w16", lambda: inputs.diffusion3d(20, 1.0, 2), 8, 16, False),
]


@pytest.mark.parametrize("precision", [hbmc.HBMC_F64, hbmc.HBMC_F32], ids=["f64", "f32"])
@pytest.mark.parametrize("name,make,bs,w,rcm", SOLVES, ids=[c[0] for c in SOLVES])
def test_solve_one_launch_matches_launches(torch, name, make, bs, w, rcm, precision):
    """ICCG to 1e-7: the one-launch substitution inside CG (forward values in
    the old direction's storage, marked empty by the direction update or,
    after the product that forms the direction itself, by a kernel of its
    own) against one launch per color."""
    print(f"case solve {name} precision {precision}", flush=True)
    (x1, st1), (x0, st0) = _solve_pair(torch, make(), bs, w, rcm, precision)
    assert st1.status == st0.status == hbmc.HBMC_OK
    assert st1.iters == st0.iters and st1.rel_res == st0.rel_res
    assert torch.equal(x1, x0), (x1 - x0).abs().max().item()


@pytest.mark.parametrize("name,make,bs,w", [
    ("knn_20000_bs2_w32", lambda: inputs.knn_laplacian(20000, 13, 4, 5, shift=1e-3), 2, 32),
    ("grid64_bs4_w8", lambda: inputs.grid2d_5pt(64), 4, 8),
], ids=["knn_20000", "grid64"])
def test_solve_one_launch_graph_replay(torch, name, make, bs, w):
    """The captured CG graph (pairs of iterations, no-op iterations past the
    stop) with the one-launch substitution, replayed with several check
    intervals, against eager launches with one launch per color.  On the
    grid the product forms p itself and the α finalizer marks the step's
    vectors empty, except past the stop, where the old direction may be the
    last step's."""
    print(f"case graph {name}", flush=True)
    A = make()
    o = hbmc.hbmc_order(A, bs, w)
    f = hbmc.ic0_factor(o, A).set_kernel(hbmc.HBMC_KERNEL_ROWS).upload()
    solver = hbmc.Solver(o, f, hbmc.hbmc_matrix_create(o, A).upload())
    b = torch.from_numpy(inputs.uniform_rhs(A.n, 3)).cuda()
    f.set_sync(hbmc.HBMC_SYNC_LAUNCH)
    x_e, st_e = solver.solve(b, use_graph=False, check_every=1)
    f.set_sync(hbmc.HBMC_SYNC_AUTO)
    for check in (16, 5, 16, 1):
        x_g, st_g = solver.solve(b, use_graph=True, check_every=check)
        torch.cuda.synchronize()
        _ = (x_g * 2).sum().item()          # eager work between replays
        assert st_g.iters == st_e.iters and st_g.status == hbmc.HBMC_OK
        assert torch.equal(x_g, x_e)


def test_wait_limit_reports_time_out(torch):
    """The failure path, forced from the host: with a 1 us limit the waits of
    the one-launch form run out long before the values they wait for are
    stored (all 27 phases of the 100k-point graph are resident at once), so
    ic0_apply_ws must set its error word and leave NaN in z, and the solve
    must report the time-out; back at the default limit both give the same
    bits as one launch per phase again (the next call clears the word)."""
    A = inputs.knn_laplacian(100_000, 13, 4, 5, shift=1e-3)
    o = hbmc.hbmc_order(A, 2, 32)
    f = hbmc.ic0_factor(o, A).set_kernel(hbmc.HBMC_KERNEL_ROWS).upload()
    solver = hbmc.Solver(o, f, hbmc.hbmc_matrix_create(o, A).upload())
    b = torch.from_numpy(inputs.uniform_rhs(A.n, 6)).cuda()
    ws = hbmc.apply_workspace(f)
    r = _rhs(torch, o, 3)
    z_ref = hbmc.ic0_apply(f, r)
    f.set_wait_limit(1)
    z = hbmc.ic0_apply_ws(f, r, ws=ws)
    torch.cuda.synchronize()
    assert hbmc.apply_ws_error(ws) != 0
    assert torch.isnan(z).any()
    with pytest.raises(hbmc.HbmcError, match="timed out"):
        solver.solve(b, tol=1e-7)
    f.set_wait_limit(0)
    z = hbmc.ic0_apply_ws(f, r, ws=ws)
    torch.cuda.synchronize()
    assert hbmc.apply_ws_error(ws) == 0 and torch.equal(z, z_ref)
    x, st = solver.solve(b, tol=1e-7)
    f.set_sync(hbmc.HBMC_SYNC_LAUNCH)
    x0, st0 = solver.solve(b, tol=1e-7)
    assert st.status == hbmc.HBMC_OK and st.iters == st0.iters and torch.equal(x, x0)

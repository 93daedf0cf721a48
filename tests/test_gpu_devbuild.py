"""The factor and the matrix built on the device (hbmc_device_build) from a
CSR in device memory.

- the device images are the host build's (ic0_factor / hbmc_matrix_create
  + upload) byte for byte: structure (strided slots, indexed slots or the
  flat form, in-block slots, tables, padding) and values (the device IC(0)
  runs the host's arithmetic in the host's order); grids (slots), graphs
  (flat form), ragged and padded orderings, FP64 and FP32, the 128^3
  benchmark workload;
- the device-built IC(0) factor against the oracle's directly: the lower
  pattern exactly, L and d to 1e-14 (Section 2, eq. "ILU"; only the
  summation order of the independent rows could differ, and it does not);
- the handles work in ic0_apply and iccg_solve like uploaded ones (same
  bits as the host-built handles);
- input errors come back as status codes before any layout is built.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1908_00741_amd import hbmc, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


CASES = [
    ("c1_grid64_bs4_w8", lambda: inputs.grid2d_5pt(64), 4, 8),
    ("grid_ragged_bs4_w8", lambda: inputs.grid2d_5pt(37, 11), 4, 8),
    ("diff3d_20_bs8_w64", lambda: inputs.diffusion3d(20, 1.0, 2), 8, 64),
    ("diff3d_24_bs8_w16", lambda: inputs.diffusion3d(24, 1.0, 3), 8, 16),
    ("knn_6000_bs8_w64", lambda: inputs.knn_laplacian(6000, 13, 4, 5), 8, 64),
    ("knn_5000_bs2_w32", lambda: inputs.knn_laplacian(5000, 13, 4, 5, shift=1e-3), 2, 32),
    ("random_bs1_w64_mc", lambda: inputs.random_spd(1500, 0.004, 7), 1, 64),
    ("random_bs16_w4", lambda: inputs.random_spd(2000, 0.003, 9), 16, 4),
    ("random_w1_bmc", lambda: inputs.random_spd(700, 0.008, 11), 8, 1),
    ("path_short", lambda: inputs.path_1d(5), 4, 8),
]


def _host_images(A, o, precision):
    f = hbmc.ic0_factor(o, A, precision)
    m = hbmc.hbmc_matrix_create(o, A)
    return f, f.image(), m, m.image()


@pytest.mark.parametrize("precision", [hbmc.HBMC_F64, hbmc.HBMC_F32], ids=["f64", "f32"])
@pytest.mark.parametrize("name,make,bs,w", CASES, ids=[c[0] for c in CASES])
def test_device_images_equal_host(torch, name, make, bs, w, precision):
    print(f"case devbuild {name} precision {precision}", flush=True)
    A = make()
    o = hbmc.hbmc_order(A, bs, w)
    fh, fimg, mh, mimg = _host_images(A, o, precision)
    b = hbmc.device_build(o, A, precision)
    fd = b.factor.dev[: b.factor.device_bytes()].cpu().numpy()
    md = b.matrix.dev[: b.matrix.device_bytes()].cpu().numpy()
    assert fd.size == fimg.size and md.size == mimg.size
    assert np.array_equal(fd, fimg), np.flatnonzero(fd != fimg)[:8]
    assert np.array_equal(md, mimg), np.flatnonzero(md != mimg)[:8]


@pytest.mark.parametrize("name,make,bs,w", CASES[:8], ids=[c[0] for c in CASES[:8]])
def test_device_factor_matches_oracle(torch, orc, name, make, bs, w):
    print(f"case devbuild_oracle {name}", flush=True)
    A = make()
    o = hbmc.hbmc_order(A, bs, w)
    b = hbmc.device_build(o, A)
    d, rp, ci, v = b.factor.export()
    s = orc.system(A, bs, w)
    Ab = sp.csr_matrix((s.fac, s.Ab.col, s.Ab.rowptr), shape=(s.Ab.n, s.Ab.n))
    Lref = sp.tril(Ab, k=-1).tocsr()
    Lref.sort_indices()
    assert np.array_equal(rp, Lref.indptr) and np.array_equal(ci, Lref.indices)
    assert np.allclose(v, Lref.data, rtol=1e-14, atol=0)
    assert np.allclose(d, s.d, rtol=1e-14, atol=0)


def test_device_built_handles_solve(torch, orc):
    """ic0_apply and iccg_solve on device-built handles: the bits of the
    host-built ones, and the oracle's iteration count."""
    A = inputs.knn_laplacian(8000, 13, 4, 5, shift=1e-3)
    o = hbmc.hbmc_order(A, 2, 32)
    b = hbmc.device_build(o, A)
    fh = hbmc.ic0_factor(o, A).upload()
    mh = hbmc.hbmc_matrix_create(o, A).upload()
    r = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, o.n_pad)).cuda()
    za = hbmc.ic0_apply(b.factor, r).cpu().numpy()
    zb = hbmc.ic0_apply(fh, r).cpu().numpy()
    assert np.array_equal(za, zb)
    rhs = inputs.uniform_rhs(A.n, 6)
    bd = torch.from_numpy(rhs).cuda()
    xa, sa = hbmc.iccg_solve(b.factor, b.matrix, bd, tol=1e-7)
    xb, sb = hbmc.iccg_solve(fh, mh, bd, tol=1e-7)
    assert np.array_equal(xa.cpu().numpy(), xb.cpu().numpy()) and sa.iters == sb.iters
    assert abs(sa.iters - orc.system(A, 2, 32).solve(rhs, tol=1e-7).iters) <= 1


def test_device_build_full_size_128(torch):
    """The benchmark workload (128^3, bs 8, w 64): images equal to the host
    build's; the two setups timed (printed)."""
    import time
    print("case devbuild_128", flush=True)
    A = inputs.diffusion3d(128, 1.0, 2)
    t0 = time.perf_counter()
    o = hbmc.hbmc_order(A, 8, 64)
    t1 = time.perf_counter()
    b = hbmc.device_build(o, A)
    t2 = time.perf_counter()
    fh, fimg, mh, mimg = _host_images(A, o, hbmc.HBMC_F64)
    t3 = time.perf_counter()
    print(f"order {t1 - t0:.3f} s, device build {t2 - t1:.3f} s ({b.seconds}), host build {t3 - t2:.3f} s",
          flush=True)
    assert np.array_equal(b.factor.dev[: fimg.size].cpu().numpy(), fimg)
    assert np.array_equal(b.matrix.dev[: mimg.size].cpu().numpy(), mimg)


def test_device_build_rejects_bad_input(torch):
    A = inputs.random_spd(300, 0.02, 5)
    o = hbmc.hbmc_order(A, 4, 8)
    rp, ci, v = (np.asarray(A.rowptr, np.int64), np.asarray(A.col, np.int32), np.asarray(A.val, np.float64))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    # one off-diagonal value changed: not symmetric
    v2 = v.copy()
    i = int(np.flatnonzero(ci != np.repeat(np.arange(A.n), np.diff(rp)))[0])
    v2[i] *= 1.5
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.device_build(o, csr_dev=(dev(rp), dev(ci), dev(v2)))
    assert e.value.code == hbmc.HBMC_ENOTSYM
    # a non-positive diagonal
    v3 = v.copy()
    v3[rp[0] + int(np.flatnonzero(ci[rp[0]:rp[1]] == 0)[0])] = -1.0
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.device_build(o, csr_dev=(dev(rp), dev(ci), dev(v3)))
    assert e.value.code == hbmc.HBMC_EDIAG
    # nnz that does not match rowptr
    with pytest.raises(hbmc.HbmcError) as e:
        hbmc.device_build(o, csr_dev=(dev(rp), dev(ci[:-1]), dev(v[:-1])))
    assert e.value.code == hbmc.HBMC_EINVAL

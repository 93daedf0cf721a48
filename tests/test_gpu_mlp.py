"""GPU checks of the warm-start network's kernels (include/hbmc_mlp.h).

Bars:
- products C = A B in all three layouts, with and without a split over K:
  inputs that bfloat16 holds exactly, so BF16 products are exact and only
  the FP32 accumulation rounds: |C - C_ref| <= 1e-5 * (|A| |B|)_ij; FP32
  inputs: the same bound;
- loss and gradients of the network against the FP64 oracle on the same
  weights: FP32 mode 1e-5 relative (norm of each parameter's gradient);
  BF16 mode 1e-2 against the oracle that rounds weights, inputs,
  activations, targets and backward signals to bfloat16 where the kernels
  store them, and 5e-2 against the all-FP64 oracle (bfloat16 storage of the
  activations alone moves the first layer's gradient by about 2 % on this
  case, ReLU gates near zero flipping);
- one Adam step against the published update: 1e-6 relative;
- the Gaussian-source right-hand side against the input generator: 1e-12.
"""
import ctypes as C

import numpy as np
import pytest

from paper_1908_00741_amd import inputs
from paper_1908_00741_amd import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _bf16_exact(rng, shape):
    """Values with at most 8 significant bits, held exactly in bfloat16."""
    return (rng.integers(-128, 128, shape) / 64.0).astype(np.float32)


def _to_dtype(torch, a, dtype):
    t = torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    if dtype == mlp.MLP_F32:
        return t
    out = torch.empty(a.shape, dtype=torch.int16, device="cuda")
    mlp.cast(dtype, t, out)
    return out


@pytest.mark.parametrize("dtype", [mlp.MLP_BF16, mlp.MLP_F32], ids=["bf16", "f32"])
@pytest.mark.parametrize("layout", [mlp.MLP_NN, mlp.MLP_TN, mlp.MLP_NT], ids=["NN", "TN", "NT"])
@pytest.mark.parametrize("M,N,K,split,pad", [(70, 130, 45, 1, 0), (64, 64, 32, 1, 0), (64, 64, 64, 1, 0),
                                             (5, 300, 1000, 3, 0), (128, 33, 12, 1, 0), (128, 192, 256, 3, 0),
                                             (192, 128, 128, 1, 8), (128, 64, 64, 1, 3),
                                             (128, 128, 448, 2, 0), (64, 128, 640, 1, 0), (64, 64, 1280, 3, 8)])
def test_gemm(torch, dtype, layout, M, N, K, split, pad):
    """Whole 64 x 64 tiles with K a multiple of 64 (the K slice) and rows
    16-byte aligned take the BF16 kernel's 16-byte staging (with a split
    over K whose last range is empty, and with rows padded by pad
    elements); a pad of 3 breaks the alignment and K = 32 a whole slice, so
    those take the element-wise staging.  K ranges of 4, 3, 7 and 10 slices
    cover the loads that run four slices ahead (fewer slices than that,
    a number that is not a multiple of it, a last range cut short)."""
    print(f"gemm dtype {dtype} layout {layout} {M}x{N}x{K} split {split} pad {pad}", flush=True)
    rng = np.random.default_rng(M + N + K)
    A = _bf16_exact(rng, (M, K))
    B = _bf16_exact(rng, (K, N))
    As = A.T.copy() if layout == mlp.MLP_TN else A
    Bs = B.T.copy() if layout == mlp.MLP_NT else B
    if pad:
        As = np.pad(As, ((0, 0), (0, pad)), constant_values=1e30)
        Bs = np.pad(Bs, ((0, 0), (0, pad)), constant_values=1e30)
    lda = As.shape[1]
    ldb = Bs.shape[1]
    Cd = torch.zeros((split, M, N), dtype=torch.float32, device="cuda")
    mlp.gemm(dtype, layout, M, N, K, _to_dtype(torch, As, dtype), lda, _to_dtype(torch, Bs, dtype), ldb, Cd, N, split)
    Cg = Cd.cpu().numpy().astype(np.float64).sum(axis=0)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    bound = np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64)
    assert np.all(np.abs(Cg - ref) <= 1e-5 * bound + 1e-30)


@pytest.mark.parametrize("dtype", [mlp.MLP_BF16, mlp.MLP_F32], ids=["bf16", "f32"])
@pytest.mark.parametrize("M,N,K", [(1, 1000, 256), (3, 1024, 256), (4, 4104, 12), (5, 1000, 256), (70, 333, 45)])
def test_linear_fwd(torch, dtype, M, N, K):
    """Bias and ReLU epilogue, on both product paths (few rows: the
    matrix-vector kernel; more: the tiled MFMA kernel)."""
    rng = np.random.default_rng(M * 7 + N)
    X = _bf16_exact(rng, (M, K))
    W = _bf16_exact(rng, (K, N))
    b = (rng.integers(-64, 64, N) / 32.0).astype(np.float32)
    for relu in (0, 1):
        Y = torch.empty((M, N), dtype=torch.int16 if dtype == mlp.MLP_BF16 else torch.float32, device="cuda")
        Yf = torch.empty((M, N), dtype=torch.float32, device="cuda")
        Xd, Wd, bd = _to_dtype(torch, X, dtype), _to_dtype(torch, W, dtype), torch.from_numpy(b).cuda()
        mlp._ck("mlp_linear_fwd", mlp.lib().mlp_linear_fwd(dtype, M, N, K, mlp._p(Xd), mlp._p(Wd), mlp._p(bd), relu,
                                                           mlp._p(Y), mlp._p(Yf), mlp._s()))
        torch.cuda.synchronize()
        ref = X.astype(np.float64) @ W.astype(np.float64) + b
        if relu:
            ref = np.maximum(ref, 0.0)
        bound = np.abs(X).astype(np.float64) @ np.abs(W).astype(np.float64) + np.abs(b)
        assert np.all(np.abs(Yf.cpu().numpy() - ref) <= 1e-5 * bound + 1e-30)


@pytest.mark.parametrize("dtype", [mlp.MLP_BF16, mlp.MLP_F32], ids=["bf16", "f32"])
@pytest.mark.parametrize("M,N,K", [(70, 333, 45), (128, 192, 128), (64, 64, 64), (256, 320, 256), (192, 128, 192),
                                   (320, 128, 64)])
def test_linear_fwd_mse(torch, dtype, M, N, K):
    """Output layer with the loss: dY = scale (X W + b - T) in the compute
    type, the loss partial of each 64 x 64 output tile and the bias-gradient
    partial of each 64-row tile, against FP64 on inputs that bfloat16 holds
    exactly (whole BF16 tiles take the 16-byte epilogue of the tiled
    kernel; one to five row tiles)."""
    print(f"linear_fwd_mse dtype {dtype} {M}x{N}x{K}", flush=True)
    rng = np.random.default_rng(M + 3 * N + 7 * K)
    X = _bf16_exact(rng, (M, K))
    W = _bf16_exact(rng, (K, N))
    T = _bf16_exact(rng, (M, N))
    b = (rng.integers(-64, 64, N) / 32.0).astype(np.float32)
    scale = 2.0 / (M * N)
    nl, nr = C.c_int64(0), C.c_int64(0)
    mlp._ck("mlp_mse_parts", mlp.lib().mlp_mse_parts(M, N, C.byref(nl), C.byref(nr)))
    Mt, Nt = (M + 63) // 64, (N + 63) // 64
    assert (nl.value, nr.value) == (Mt * Nt, Mt)
    dY = torch.empty((M, N), dtype=torch.int16 if dtype == mlp.MLP_BF16 else torch.float32, device="cuda")
    loss = torch.empty(nl.value, dtype=torch.float32, device="cuda")
    dbias = torch.empty((nr.value, N), dtype=torch.float32, device="cuda")
    Xd, Wd, Td = _to_dtype(torch, X, dtype), _to_dtype(torch, W, dtype), _to_dtype(torch, T, dtype)
    bd = torch.from_numpy(b).cuda()
    mlp._ck("mlp_linear_fwd_mse", mlp.lib().mlp_linear_fwd_mse(dtype, M, N, K, mlp._p(Xd), mlp._p(Wd), mlp._p(bd),
                                                               mlp._p(Td), scale, mlp._p(dY), mlp._p(loss),
                                                               mlp._p(dbias), mlp._s()))
    torch.cuda.synchronize()
    y = X.astype(np.float64) @ W.astype(np.float64) + b
    bound = np.abs(X).astype(np.float64) @ np.abs(W).astype(np.float64) + np.abs(b)
    d = y - T
    g = scale * d
    if dtype == mlp.MLP_BF16:
        got = (dY.cpu().numpy().astype(np.int32) & 0xFFFF).astype(np.uint32) << 16
        got = got.view(np.float32).astype(np.float64)
        assert np.all(np.abs(got - g) <= 2.0 ** -8 * np.abs(g) + scale * 1e-5 * bound + 1e-30)
    else:
        assert np.all(np.abs(dY.cpu().numpy() - g) <= scale * 1e-5 * bound + 1e-30)
    lp = loss.cpu().numpy().astype(np.float64).reshape(Mt, Nt)
    dp = dbias.cpu().numpy().astype(np.float64)
    for mt in range(Mt):
        rows = slice(64 * mt, min(M, 64 * mt + 64))
        ref_db = g[rows].sum(axis=0)
        tol_db = scale * (np.abs(d[rows]).sum(axis=0) * 1e-5 + 1e-5 * bound[rows].sum(axis=0))
        assert np.all(np.abs(dp[mt] - ref_db) <= tol_db + 1e-30), mt
        for nt in range(Nt):
            cols = slice(64 * nt, min(N, 64 * nt + 64))
            ref_l = (d[rows, cols] ** 2).sum()
            assert abs(lp[mt, nt] - ref_l) <= 1e-5 * ref_l + 2e-5 * (np.abs(d[rows, cols]) * bound[rows, cols]).sum()


def _net(rng, dims):
    ps = []
    for k in range(3):
        b = 1.0 / np.sqrt(dims[k])
        ps += [rng.uniform(-b, b, (dims[k], dims[k + 1])).astype(np.float32),
               rng.uniform(-b, b, dims[k + 1]).astype(np.float32)]
    return ps


@pytest.mark.parametrize("M,n", [(40, 777), (128, 768)], ids=["ragged", "whole_tiles"])
@pytest.mark.parametrize("dtype,tol", [(mlp.MLP_F32, 1e-5), (mlp.MLP_BF16, 1e-2)], ids=["f32", "bf16"])
def test_gradients_against_oracle(torch, dtype, tol, M, n):
    """Ragged: every product takes the element-wise staging; whole tiles
    (batch and widths multiples of 64): the hidden and output layers and
    their backward products take the BF16 16-byte staging."""
    from oracle import mlp as omlp
    print(f"mlp gradient check dtype {dtype} batch {M} outputs {n}", flush=True)
    rng = np.random.default_rng(11)
    ps = _net(rng, [12, 256, 256, n])
    theta = rng.uniform(-1, 1, (M, 12)).astype(np.float32)
    target = rng.uniform(-1, 1, (M, n)).astype(np.float32)
    net = mlp.MLP(n, dtype=dtype)
    net.set_weights(ps)
    tgt = _to_dtype(torch, target, dtype)
    loss_parts = net.loss_and_grads(torch.from_numpy(theta).cuda(), tgt)
    torch.cuda.synchronize()
    loss = float(loss_parts.cpu().numpy().astype(np.float64).sum()) / (M * n)
    grads = [g.cpu().numpy().astype(np.float64) for g in net.grad]
    checks = []
    if dtype == mlp.MLP_BF16:
        # weights as the kernels read them (bfloat16), biases FP32
        ref_ps = [omlp.bf16_round(p) if p.ndim == 2 else p.astype(np.float64) for p in ps]
        checks.append((omlp.loss_and_grads(theta, target, ref_ps, store=omlp.bf16_round), tol))
        checks.append((omlp.loss_and_grads(omlp.bf16_round(theta), omlp.bf16_round(target), ref_ps), 5e-2))
    else:
        checks.append((omlp.loss_and_grads(theta, target, [p.astype(np.float64) for p in ps]), tol))
    for (L, gs), bar in checks:
        assert abs(loss - L) <= bar * abs(L)
        for k, (g, gr) in enumerate(zip(grads, gs)):
            assert np.linalg.norm(g - gr) <= bar * np.linalg.norm(gr), (k, bar)


@pytest.mark.parametrize("M,n", [(40, 777), (128, 768)], ids=["ragged", "whole_tiles"])
@pytest.mark.parametrize("dtype", [mlp.MLP_F32, mlp.MLP_BF16], ids=["f32", "bf16"])
def test_train_step_matches_separate_calls(torch, dtype, M, n):
    """mlp_train_step (W3's Adam update inside its weight-gradient product)
    against loss_and_grads + adam_step on the same weights and batches: the
    same bits in every master weight, moment, compute copy and loss, over
    two steps; W3's gradient array is left as it was."""
    print(f"train step dtype {dtype} batch {M} outputs {n}", flush=True)
    rng = np.random.default_rng(5)
    ps = _net(rng, [12, 256, 256, n])
    nets = [mlp.MLP(n, dtype=dtype) for _ in range(2)]
    for net in nets:
        net.set_weights(ps)
    nets[1].grad[4].fill_(12345.0)
    opt = mlp.Adam(lr=3e-3)
    for it in range(2):
        theta = torch.from_numpy(rng.uniform(-1, 1, (M, 12)).astype(np.float32)).cuda()
        tgt = _to_dtype(torch, rng.uniform(-1, 1, (M, n)).astype(np.float32), dtype)
        l0 = nets[0].loss_and_grads(theta, tgt).clone()
        nets[0].adam_step(opt)
        l1 = nets[1].train_step(theta, tgt, opt).clone()
        torch.cuda.synchronize()
        assert torch.equal(l0, l1), it
        for k in range(6):
            for name in ("master", "m", "v", "comp"):
                a, b = getattr(nets[0], name)[k], getattr(nets[1], name)[k]
                assert torch.equal(a, b), (it, k, name)
    assert bool((nets[1].grad[4] == 12345.0).all())


@pytest.mark.parametrize("R,N,pad", [(1, 5, 0), (15, 257, 0), (16, 64, 3), (17, 1, 0), (300, 257, 7)])
def test_sum_rows_in_order(torch, R, N, pad):
    """Column sums in FP32, rows added in order: the same bits as a
    sequential FP32 sum on the host (rows loaded sixteen at a time)."""
    rng = np.random.default_rng(R * 31 + N)
    src = rng.standard_normal((R, N + pad)).astype(np.float32)
    out = torch.empty(N, dtype=torch.float32, device="cuda")
    mlp.sum_rows(R, N, torch.from_numpy(src).cuda(), N + pad, out)
    ref = np.zeros(N, dtype=np.float32)
    for i in range(R):
        ref = (ref + src[i, :N]).astype(np.float32)
    assert np.array_equal(out.cpu().numpy(), ref)


def test_time_steps_mode(torch):
    """The step-timing mode of the warm-start CLI runs the fused step on a
    small network and reports its time."""
    from paper_1908_00741_amd import warmstart
    r = warmstart.time_steps(16, 3, batch=64)
    assert r["network"] == "12-256-256-4096" and r["batch"] == 64 and r["steps"] == 3
    assert r["ms_per_step"] > 0.0


def test_adam_step(torch):
    from oracle import mlp as omlp
    rng = np.random.default_rng(5)
    n = 10007
    w, m, v, g = [rng.uniform(-1, 1, n).astype(np.float32) for _ in range(4)]
    v = np.abs(v)
    dev = [torch.from_numpy(a.copy()).cuda() for a in (w, m, v, g)]
    wc = torch.empty(n, dtype=torch.int16, device="cuda")
    for step in (1, 7):
        lib = mlp.lib()
        mlp._ck("mlp_adam", lib.mlp_adam(mlp.MLP_BF16, n, mlp._p(dev[0]), mlp._p(dev[1]), mlp._p(dev[2]),
                                         mlp._p(dev[3]), mlp._p(wc), 1e-3, 0.9, 0.999, 1e-8, step, mlp._s()))
        w, m, v = omlp.adam(w.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                            g.astype(np.float64), step)
        for t, r in zip(dev[:3], (w, m, v)):
            assert np.allclose(t.cpu().numpy(), r, rtol=1e-6, atol=1e-7)
        w, m, v = [t.cpu().numpy() for t in dev[:3]]
    # the compute copy is the rounded master copy
    wc32 = (wc.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16).view(np.float32)
    assert np.array_equal(wc32.astype(np.float64), omlp.bf16_round(dev[0].cpu().numpy()))


def test_gaussian_rhs(torch):
    N = 20
    theta = inputs.sample_sources(3, 12)
    for th in theta:
        b = torch.empty(N ** 3, dtype=torch.float64, device="cuda")
        mlp.gaussian_rhs(N, th, b)
        ref = inputs.gaussian_sources_rhs(N, th)
        assert np.abs(b.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


def test_combine(torch):
    rng = np.random.default_rng(9)
    G = rng.uniform(-1, 1, (10, 333)).astype(np.float32)
    Gd = torch.from_numpy(G).cuda()
    idx = rng.integers(0, 10, (7, 4))
    amp = rng.uniform(-1, 1, (7, 4)).astype(np.float32)
    out = torch.empty((7, 333), dtype=torch.float32, device="cuda")
    mlp.combine(mlp.MLP_F32, Gd, idx, amp, 0.5, out)
    ref = 0.5 * np.einsum("mq,mqi->mi", amp.astype(np.float64), G[idx].astype(np.float64))
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-6
    with pytest.raises(ValueError):
        mlp.combine(mlp.MLP_F32, Gd, idx + 10, amp, 1.0, out)


def test_warm_start_gain(torch):
    """A network trained on combinations of 2000 single-source solutions of
    a 16^3 problem family gives CG start vectors that save iterations on 24
    unseen source configurations at the same stopping test, and makes none of
    them take more than one extra iteration."""
    from paper_1908_00741_amd import warmstart
    print("warm start gain 16^3", flush=True)
    ws = warmstart.WarmStart(N=16, sigma=0.5, seed=10, device="cuda", tol=1e-8)
    G, S, W, gen = ws.generate_single(500)
    tr = ws.train_combined(G, S, W, steps=3000, batch=128, lr=1e-3, log_every=1000)
    assert tr["curve"][-1][1] < 0.5 * tr["curve"][0][1]
    test = inputs.sample_sources(24, 12)
    rows = []
    for th in test:
        _, s0 = ws.solve(th)
        _, s1 = ws.solve(th, ws.predict(th))
        rows.append((s0.iters, s1.iters, s0.true_rel_res, s1.true_rel_res))
    r = np.array(rows)
    print("iterations x0=0", r[:, 0].mean(), "warm", r[:, 1].mean(), flush=True)
    assert r[:, 2].max() < 1e-7 and r[:, 3].max() < 1e-7
    assert r[:, 1].mean() <= r[:, 0].mean() - 0.5
    assert np.all(r[:, 1] <= r[:, 0] + 1)

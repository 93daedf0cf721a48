"""Learned warm start for ICCG (not part of the paper's method).

A family of problems shares the matrix -- 3D diffusion on N^3 cells with
fixed lognormal coefficients -- and varies the right-hand side: four
Gaussian sources with 12 parameters theta (positions along the cube's body
diagonals, widths, amplitudes).  A network x0 = s * MLP(theta) is trained on
solutions that the solver itself produced, then gives CG its start vector;
CG still stops on its own residual test ||b - A x|| / ||b|| < tol, so the
accuracy is that of the plain solver.  The solver scales the network's x0
by c = (b, x0) / (x0, A x0), the multiple of x0 closest to the solution in
the A-norm (the norm CG minimizes), so the start is never worse than x = 0
in that norm; when (b, x0) <= 0 the scale is 0 and the solve starts from
x = 0, the fallback.  (The test ||b - A x0|| >= ||b|| would reject nearly
every guess of the network: its bfloat16 storage adds high-frequency error
that raises the residual above ||b|| while the A-norm error, and the
iteration count, still improve.)

The right-hand sides, the solves, the network's products, loss and Adam
steps all run in the library's kernels (hbmc.h, hbmc_mlp.h).

Command line (one GPU): ``python -m paper_1908_00741_amd.warmstart --N 96
--train 4000 --test 200`` prints one JSON line with the training curve and
the iterations and times with and without the warm start.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import hbmc, inputs, mlp


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ranges of the source parameters (positions, widths, amplitudes); the
# network sees each parameter mapped affinely onto [-1, 1]
_LO = np.array([0.15] * 4 + [0.03] * 4 + [-1.0] * 4)
_HI = np.array([0.85] * 4 + [0.15] * 4 + [1.0] * 4)


def features(theta) -> np.ndarray:
    t = np.atleast_2d(np.asarray(theta, np.float64))
    return (2.0 * (t - _LO) / (_HI - _LO) - 1.0).astype(np.float32)


class WarmStart:
    def __init__(self, N=96, sigma=0.5, seed=10, bs=8, w=64, dtype=mlp.MLP_BF16, device="cuda", tol=1e-7,
                 net_seed=0):
        import torch
        self.N, self.n, self.tol = N, N ** 3, tol
        self.device = torch.device(device)
        self.A = inputs.diffusion3d(N, sigma, seed)
        self.solver = hbmc.Solver.setup(self.A, bs, w, device=self.device)
        self.work = hbmc.workspace(self.solver.factor, 1, self.device)
        self.net = mlp.MLP(self.n, dtype=dtype, seed=net_seed, device=self.device)
        self.dtype = dtype
        self.scale = 1.0
        self.b = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self.x = torch.empty(self.n, dtype=torch.float64, device=self.device)

    def rhs(self, theta):
        mlp.gaussian_rhs(self.N, theta, self.b)
        return self.b

    def solve(self, theta, x0=None):
        """ICCG for the sources theta from x0 (None: zero).  Returns (x,
        stats); x is the solver's buffer, overwritten by the next call."""
        b = self.rhs(theta)
        if x0 is None:
            x, st = self.solver.solve(b, self.x, tol=self.tol, x0_zero=True, work=self.work)
        else:
            self.x.copy_(x0)
            x, st = self.solver.solve(b, self.x, tol=self.tol, x0_zero=False, work=self.work, x0_scale=True)
        return x, st

    def generate(self, thetas, scale_from=64):
        """Targets: the solutions for thetas, divided by s = the RMS of the
        first scale_from solutions, in the compute type [count][n]."""
        import torch
        count = len(thetas)
        tgt = torch.empty((count, self.n), dtype=mlp._torch_dtype(self.dtype), device=self.device)
        sq, its = 0.0, []
        t0 = time.perf_counter()
        held = []
        for i, th in enumerate(thetas):
            x, st = self.solve(th)
            its.append(st.iters)
            if i < scale_from:
                held.append(x.cpu().numpy())
                if i == min(scale_from, count) - 1:
                    sq = float(np.mean(np.square(np.stack(held))))
                    self.scale = float(np.sqrt(sq)) if sq > 0 else 1.0
                    for k, h in enumerate(held):
                        self.x.copy_(torch.from_numpy(h))
                        mlp.cast_f64(self.dtype, self.x, 1.0 / self.scale, tgt[k])
                    held = None
            else:
                mlp.cast_f64(self.dtype, x, 1.0 / self.scale, tgt[i])
            if (i + 1) % 500 == 0:
                log(f"[warmstart] {i + 1}/{count} solutions, {time.perf_counter() - t0:.1f} s")
        torch.cuda.synchronize()
        return tgt, {"count": count, "seconds": round(time.perf_counter() - t0, 2), "scale": self.scale,
                     "iters_mean": float(np.mean(its))}

    def generate_single(self, per_diagonal, seed=11, scale_from=16):
        """Single-source solutions: for each of the four diagonals,
        per_diagonal sources (position and width uniform in their ranges,
        amplitude 1, the other sources off).  The solution for any theta is
        the amplitude-weighted sum of its four single-source solutions, so
        these solves yield training targets for every combination of them.
        Returns G [4 * per_diagonal][n] (compute type, divided by s), the
        positions and widths [4][per_diagonal], and a summary."""
        import torch
        rng = np.random.default_rng(seed)
        S = rng.uniform(_LO[0], _HI[0], (4, per_diagonal))
        W = rng.uniform(_LO[4], _HI[4], (4, per_diagonal))
        G = torch.empty((4 * per_diagonal, self.n), dtype=mlp._torch_dtype(self.dtype), device=self.device)
        its, held = [], []
        t0 = time.perf_counter()
        for q in range(4):
            for k in range(per_diagonal):
                th = np.array([0.5] * 4 + [0.1] * 4 + [0.0] * 4)
                th[q], th[4 + q], th[8 + q] = S[q, k], W[q, k], 1.0
                x, st = self.solve(th)
                its.append(st.iters)
                if k < scale_from:
                    held.append(x.cpu().numpy())
                mlp.cast_f64(self.dtype, x, 1.0, G[q * per_diagonal + k])
            log(f"[warmstart] diagonal {q}: {per_diagonal} single-source solutions, {time.perf_counter() - t0:.1f} s")
        # E[x^2] of a combination = sum over q of E[a_q^2] E[G_q^2], E[a^2] = 1/3
        self.scale = float(np.sqrt(np.mean(np.square(np.stack(held))) * 4.0 / 3.0))
        # divide the stored solutions by s (in place, in the compute type)
        self._scale_rows(G, 1.0 / self.scale)
        torch.cuda.synchronize()
        return G, S, W, {"solves": 4 * per_diagonal, "seconds": round(time.perf_counter() - t0, 2),
                         "scale": self.scale, "iters_mean": float(np.mean(its))}

    def _scale_rows(self, G, factor):
        """G *= factor through the combination kernel (one source, weight factor)."""
        rows = G.shape[0]
        for a in range(0, rows, 4096):
            e = min(rows, a + 4096)
            idx = np.zeros((e - a, 4), np.int32)
            idx[:, 0] = np.arange(a, e)
            amp = np.zeros((e - a, 4), np.float32)
            amp[:, 0] = 1.0
            mlp.combine(self.dtype, G, idx, amp, factor, G[a:e])

    def train_combined(self, G, S, W, steps=3000, batch=256, lr=1e-3, seed=0, log_every=500):
        """Adam (cosine-decayed rate) on the mean squared error over batches of
        random combinations: per sample, one stored solution per diagonal and
        amplitudes uniform in [-1, 1]; targets formed on the device."""
        import torch
        per = G.shape[0] // 4
        rng = np.random.default_rng(seed)
        T = torch.empty((batch, self.n), dtype=mlp._torch_dtype(self.dtype), device=self.device)
        curve = []
        t0 = time.perf_counter()
        for step in range(1, steps + 1):
            k = rng.integers(0, per, (batch, 4))
            amp = rng.uniform(-1.0, 1.0, (batch, 4))
            th = np.concatenate([S[np.arange(4), k], W[np.arange(4), k], amp], axis=1)
            idx = k + per * np.arange(4)
            mlp.combine(self.dtype, G, idx, amp, 1.0, T)
            rate = lr * 0.5 * (1.0 + np.cos(np.pi * (step - 1) / steps))
            # loss of the weights before this step's update
            parts = self.net.train_step(torch.from_numpy(features(th)).to(self.device), T, mlp.Adam(lr=float(rate)))
            if step % log_every == 0 or step == steps:
                loss = float(parts.cpu().numpy().astype(np.float64).sum()) / (batch * self.n)
                curve.append([step, loss])
                log(f"[warmstart] step {step}: loss {loss:.4e} ({time.perf_counter() - t0:.1f} s)")
        torch.cuda.synchronize()
        return {"steps": steps, "batch": batch, "lr": lr, "schedule": "cosine",
                "seconds": round(time.perf_counter() - t0, 2), "curve": curve}

    def train(self, thetas, targets, epochs=100, batch=256, lr=1e-3, seed=0, log_every=10):
        """Adam on the mean squared error over contiguous batches of the
        (i.i.d.) training set, batch order shuffled each epoch."""
        import torch
        count = len(thetas)
        th = torch.from_numpy(features(thetas)).to(self.device)
        starts = list(range(0, count, batch))
        rng = np.random.default_rng(seed)
        opt = mlp.Adam(lr=lr)
        curve = []
        t0 = time.perf_counter()
        for ep in range(epochs):
            logging = ep % log_every == log_every - 1 or ep == epochs - 1
            total = 0.0
            for k in rng.permutation(len(starts)):
                a = starts[k]
                e = min(count, a + batch)
                parts = self.net.train_step(th[a:e], targets[a:e], opt)
                if logging:   # loss before this batch's update (host sum of the partials)
                    total += float(parts.cpu().numpy().astype(np.float64).sum())
            if logging:
                loss = total / (count * self.n)
                curve.append([ep + 1, loss])
                log(f"[warmstart] epoch {ep + 1}: loss {loss:.4e} ({time.perf_counter() - t0:.1f} s)")
        torch.cuda.synchronize()
        return {"epochs": epochs, "batch": batch, "lr": lr, "seconds": round(time.perf_counter() - t0, 2),
                "curve": curve}

    def predict(self, theta):
        """x0 = s * MLP(theta) in FP64 on the device."""
        import torch
        t = torch.from_numpy(features(theta)).to(self.device)
        y = self.net.forward(t)
        x0 = torch.empty(self.n, dtype=torch.float64, device=self.device)
        mlp.to_f64(y[0], self.scale, x0)
        return x0

    def evaluate(self, thetas):
        """Per test theta: iterations, time and true residual from x0 = 0
        and from the network's x0 (its inference included in the time)."""
        import torch
        rows = []
        for th in thetas:
            self.solve(th)                         # warm the graph caches
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, s0 = self.solve(th)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, s1 = self.solve(th, self.predict(th))
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            rows.append((s0.iters, s1.iters, t1 - t0, t2 - t1, s0.true_rel_res, s1.true_rel_res, s1.x0_scale))
        r = np.array(rows)
        return {"count": len(rows), "iters_x0_zero": float(r[:, 0].mean()), "iters_warm": float(r[:, 1].mean()),
                "x0_scale_mean": round(float(r[:, 6].mean()), 4), "x0_scale_min": round(float(r[:, 6].min()), 4),
                "fallbacks_to_zero": int((r[:, 6] == 0.0).sum()),
                "ms_x0_zero": round(float(r[:, 2].mean()) * 1e3, 3),
                "ms_warm_incl_inference": round(float(r[:, 3].mean()) * 1e3, 3),
                "speedup": round(float(r[:, 2].sum() / r[:, 3].sum()), 3),
                "true_rel_res_max_x0_zero": float(r[:, 4].max()), "true_rel_res_max_warm": float(r[:, 5].max())}


def time_steps(N, steps, batch=256, dtype=mlp.MLP_BF16, device="cuda:0", seed=0):
    """Time of one fused training step (forward, backward, Adam) of the
    12-256-256-N^3 network on a fixed synthetic batch (inputs uniform in
    [-1, 1], targets standard normal), after three untimed steps."""
    import torch
    dev = torch.device(device)
    n = N ** 3
    rng = np.random.default_rng(seed)
    net = mlp.MLP(n, dtype=dtype, seed=seed, device=dev)
    theta = torch.from_numpy(rng.uniform(-1.0, 1.0, (batch, 12)).astype(np.float32)).to(dev)
    tf = torch.from_numpy(rng.standard_normal((batch, n), dtype=np.float32)).to(dev)
    target = torch.empty((batch, n), dtype=mlp._torch_dtype(dtype), device=dev)
    mlp.cast(dtype, tf, target)
    del tf
    opt = mlp.Adam(lr=1e-3)
    for _ in range(3):
        net.train_step(theta, target, opt)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        net.train_step(theta, target, opt)
    e1.record()
    torch.cuda.synchronize()
    return {"network": f"12-256-256-{n}", "dtype": "bf16" if dtype == mlp.MLP_BF16 else "f32", "batch": batch,
            "steps": steps, "ms_per_step": round(e0.elapsed_time(e1) / steps, 4)}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=96)
    ap.add_argument("--train", type=int, default=4000, help="ICCG solves for training data")
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--mode", choices=("combined", "direct"), default="combined",
                    help="combined: single-source solutions combined into targets on the fly; "
                         "direct: one solution per sampled theta")
    ap.add_argument("--steps", type=int, default=100000, help="Adam steps (combined)")
    ap.add_argument("--epochs", type=int, default=100, help="epochs (direct)")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--f32", action="store_true", help="FP32 network (default BF16)")
    ap.add_argument("--time-steps", type=int, default=0,
                    help="only time this many training steps of the N^3 network on a synthetic batch")
    args = ap.parse_args(argv)
    dtype = mlp.MLP_F32 if args.f32 else mlp.MLP_BF16
    if args.time_steps > 0:
        print(json.dumps(time_steps(args.N, args.time_steps, args.batch, dtype)), flush=True)
        return 0
    import torch
    dev = torch.device("cuda:0")
    ws = WarmStart(args.N, dtype=dtype, device=dev)
    test_th = inputs.sample_sources(args.test, 12)
    if args.mode == "combined":
        log(f"[warmstart] {args.N}^3, {args.train} single-source solutions")
        G, S, W, gen = ws.generate_single(args.train // 4)
        log(f"[warmstart] training {args.steps} steps")
        tr = ws.train_combined(G, S, W, args.steps, args.batch, args.lr)
        del G
    else:
        train_th = inputs.sample_sources(args.train, 11)
        log(f"[warmstart] {args.N}^3, generating {args.train} training solutions")
        targets, gen = ws.generate(train_th)
        log(f"[warmstart] training {args.epochs} epochs")
        tr = ws.train(train_th, targets, args.epochs, args.batch, args.lr)
        del targets
    torch.cuda.empty_cache()
    log(f"[warmstart] evaluating on {args.test} test sources")
    ev = ws.evaluate(test_th)
    out = {"workload": f"diffusion3d {args.N}^3 lognormal sigma=0.5 seed 10, b = 4 Gaussian sources "
                       f"(test theta seed 12), HBMC bs=8 w=64, FP64 ICCG tol {ws.tol:g}",
           "network": f"12-256-256-{ws.n} ReLU, {'FP32' if args.f32 else 'BF16'} storage, FP32 accumulation, "
                      f"Adam, MSE on x/s",
           "mode": args.mode, "generate": gen, "train": tr, "evaluate": ev}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

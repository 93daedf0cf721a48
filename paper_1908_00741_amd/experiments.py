"""Measured comparisons of the solver's forms against plain FP64 single-
right-hand-side ICCG on the same GPU, at equal final true residual (every
solve stops at ||r|| / ||b|| < tol and reports ||b - A x|| / ||b||).

- fp32: FP32 factor and substitutions (FP64 CG) against FP64, on the
  unstructured 13-NN Laplacian of 1M points (many small color phases: bound
  by latency) and on the 128^3 diffusion problem (bound by bandwidth);
- batch: 128 Poisson systems of uneven size (16^3 .. 64^3) solved together
  (one set of launches per iteration, per-system stopping tests, FP32
  preconditioner, autotuned bs, w and kernel) against solving them one by
  one in FP64, and the same batch with the FP64 preconditioner (batching
  alone, without the precision change);
- rhs: 32 right-hand sides of the 128^3 lognormal diffusion problem solved
  together (factor read once per apply for all of them, autotuned
  right-hand-side tile, FP32 preconditioner) against 32 FP64 solves;
- graph: the same solve with the iterations replayed as a hipGraph and
  launched one by one;
- smoother: symmetric Gauss-Seidel / SSOR and forward Gauss-Seidel steps
  on the HBMC substitution kernels (time per step, bytes per step), and
  SSOR-preconditioned CG against IC(0)-preconditioned CG;
- refactor: new coefficients of the 128^3 problem (same pattern): the
  factor and matrix rebuilt on the host and uploaded against recomputed on
  the device (ic0_refactor, hbmc_matrix_revalue);
- orderings: multi-color (bs = 1), block multi-color (w = 1: one block per
  lane, rows of a lane 1 apart) and hierarchical block multi-color ordering
  of the same problem, FP64: iterations, time and time per iteration (the
  comparison of Section 5's tables, on one GPU);
- warmstart: the learned warm start on the 96^3 diffusion problem with
  Gaussian sources, trained from scratch on a short schedule (single-source
  ICCG solutions combined into targets, Adam on the device); iterations and
  time to 1e-7 per test source against x0 = 0, the network's inference
  included, the start scaled by the A-norm-optimal factor (0: fallback to
  x0 = 0);
- locality: the 13-NN Laplacian of 1M points (its numbering shuffled) in
  the input's numbering and after the reverse Cuthill-McKee renumbering
  (hbmc_order_rcm, a pre-pass outside the paper): ordering time, colors,
  cold ic0_apply and ICCG to 1e-7 with the FP64 and FP32 preconditioners;
- apply_rate: ic0_apply alone on a named workload, timed with HIP events
  with the caches cold before each call (also the command line used for
  per-workload profiles: ``python -m paper_1908_00741_amd.experiments
  apply knn1m --bs 2 --w 32``; ``solve`` in place of ``apply`` runs ICCG
  to 1e-7 on the workload instead).

Setup (ordering, factorization, upload) is outside every timed region.
"""
from __future__ import annotations

import time

import numpy as np

from . import autotune, hbmc, inputs


def _sync():
    import torch
    torch.cuda.synchronize()


def _timed(fn, reps=3):
    """Median wall time of reps calls (after one untimed call) and the last
    result."""
    out = fn()
    ts = []
    for _ in range(reps):
        _sync()
        t0 = time.perf_counter()
        out = fn()
        _sync()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), out


def _stats(st):
    sts = st if isinstance(st, list) else [st]
    return {"iters_max": max(s.iters for s in sts), "iters_min": min(s.iters for s in sts),
            "true_rel_res_max": max(s.true_rel_res for s in sts),
            "all_converged": all(s.status == hbmc.HBMC_OK for s in sts)}


HBM_PEAK_GBS = 8000.0


def apply_bytes(n: int, nnz_lower: int, s_v: int = 8, s_d: int = 8, s_y: int = 8) -> int:
    """Algorithmic bytes of one ic0_apply: L and U values + int32 indices read
    once, diaginv for the forward and backward sweeps, r read, z written, and
    the intermediate y written and read back."""
    return 2 * nnz_lower * (s_v + 4) + 2 * n * s_d + n * 8 + n * 8 + 2 * n * s_y


class ColdTimer:
    """HIP-event timing of one call on the current stream, with the caches
    put in a known state before each call: "cold" writes 1 GiB (evicting the
    4 MB L2s and the 256 MB MALL) and then reads a different 1 GiB (so the
    MALL holds clean lines and the timed call's misses pay no write-backs);
    "dirty" only writes; "warm" runs back to back."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.flush = torch.empty(1 << 30, dtype=torch.uint8, device=device)
        self.flush2 = torch.zeros(1 << 27, dtype=torch.float64, device=device)
        self.sink = torch.empty((), dtype=torch.float64, device=device)

    def evict(self, i, clean=True):
        self.flush.fill_(i & 255)
        if clean:
            self.torch.sum(self.flush2, dim=0, out=self.sink)

    def times_ms(self, fn, reps, mode="cold"):
        torch = self.torch
        stream = torch.cuda.current_stream()
        ts = []
        for i in range(reps):
            if mode != "warm":
                self.evict(i, mode == "cold")
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return np.array(ts)


WORKLOADS = {
    "grid64": lambda: inputs.grid2d_5pt(64),
    "diffusion128": lambda: inputs.diffusion3d(128, 1.0, 2),
    "diffusion96": lambda: inputs.diffusion3d(96, 0.5, 10),
    "knn1m": lambda: inputs.knn_laplacian(1_000_000, 13, 4, 5, shift=1e-3),
}


def apply_rate(device, A, bs, w, precision=hbmc.HBMC_F64, kernel=hbmc.HBMC_KERNEL_AUTO, reps=50,
               timer=None, order=None, modes=("cold",), log=print, label=""):
    """Median HIP-event time of one preconditioning step on A (random r in
    HBMC order, dummies 0), caches cold before each call, and its
    algorithmic rate.  The step is ic0_apply_ws (the row kernel's phases in
    one launch where that applies, else the same as ic0_apply); the cold
    time of ic0_apply (one launch per color phase) is reported beside it."""
    import torch
    o = order if order is not None else hbmc.hbmc_order(A, bs, w)
    f = hbmc.ic0_factor(o, A, precision).set_kernel(kernel).upload(device)
    perm, _ = o.perm()
    r_np = np.zeros(f.n_pad)
    r_np[perm] = np.random.default_rng(17).uniform(-1, 1, A.n)
    r = torch.from_numpy(r_np).to(device)
    z = torch.empty_like(r)
    ws = hbmc.apply_workspace(f, device)
    for _ in range(5):
        hbmc.ic0_apply_ws(f, r, z, ws)
        hbmc.ic0_apply(f, r, z)
    _sync()
    timer = timer or ColdTimer(device)
    nl = (A.nnz - A.n) // 2
    sv = 8 if precision == hbmc.HBMC_F64 else 4
    B = apply_bytes(f.n_pad, nl, sv, sv, sv)
    out = {"bytes_per_apply": B, "n": A.n, "n_pad": f.n_pad, "nnz_lower": nl, "n_colors": f.n_colors,
           "phases": 2 * f.n_colors - 1, "bs": bs, "w": w,
           "precision": "f64" if precision == hbmc.HBMC_F64 else "f32"}
    t = timer.times_ms(lambda: hbmc.ic0_apply(f, r, z), reps, "cold")
    out["median_us_cold_launches"] = round(float(np.median(t)) * 1e3, 2)
    for mode in modes:
        t = timer.times_ms(lambda: hbmc.ic0_apply_ws(f, r, z, ws), reps, mode)
        us = float(np.median(t)) * 1e3
        g = B / (us * 1e-6) / 1e9
        key = "" if mode == "cold" else "_" + mode
        out["median_us" + ("_cold" if mode == "cold" else key)] = round(us, 2)
        out["gbs" + key] = round(g, 1)
        out["frac" + key] = round(g / HBM_PEAK_GBS, 4)
        log(f"[apply {label}] {mode}: {us:.1f} us, {g:.0f} GB/s algorithmic ({g / HBM_PEAK_GBS:.3f} of peak), "
            f"{f.n_colors} colors (one launch per color: {out['median_us_cold_launches']:.1f} us cold)")
    if hbmc.apply_ws_error(ws):
        raise RuntimeError("a wait inside the one-launch substitution timed out")
    del f, r, z, ws
    return out


def warmstart(device, N=96, per_diagonal=250, steps=20000, test=50, log=print):
    """Learned warm start, trained here on a short schedule: per_diagonal
    single-source solutions per body diagonal, steps Adam steps (batch 256),
    then test sources (seed 12) solved from x0 = 0 and from the network."""
    from . import warmstart as wsm
    t0 = time.perf_counter()
    ws = wsm.WarmStart(N, device=device)
    G, S, W, gen = ws.generate_single(per_diagonal)
    tr = ws.train_combined(G, S, W, steps, 256, 1e-3, log_every=max(1, steps // 4))
    del G
    ev = ws.evaluate(inputs.sample_sources(test, 12))
    out = {"workload": f"diffusion3d {N}^3 lognormal sigma=0.5 seed 10, 4 Gaussian sources, bs 8, w 64, FP64, "
                       f"tol {ws.tol:g}",
           "training_solves": gen["solves"], "training_solve_s": gen["seconds"], "steps": steps,
           "train_s": tr["seconds"], "final_loss": tr["curve"][-1][1] if tr["curve"] else None, **ev,
           "total_s": round(time.perf_counter() - t0, 1)}
    log(f"[ext warmstart] {ev['iters_x0_zero']:.1f} -> {ev['iters_warm']:.1f} iterations, "
        f"{ev['ms_x0_zero']:.2f} -> {ev['ms_warm_incl_inference']:.2f} ms, {ev['speedup']:.3f}x")
    del ws
    return out


def fp32(device, npts=1_000_000, bs=2, w=32, tol=1e-7, log=print):
    """FP32 against FP64 preconditioner on the 13-NN Laplacian (bs 2, w 32:
    the fastest FP64 solve of a sweep over bs in {1, 2, 4, 8}, w and both
    substitution kernels)."""
    import torch
    log(f"[ext fp32] kNN Laplacian {npts} points, bs={bs} w={w}")
    A = inputs.knn_laplacian(npts, 13, 4, 5, shift=1e-3)
    b = torch.from_numpy(inputs.uniform_rhs(A.n, 3)).to(device)
    res = {"workload": f"13-NN Laplacian of {npts} uniform points, 1/dist weights, shift 1e-3, "
                       f"b~U[-1,1], HBMC bs={bs} w={w}, tol {tol:g}"}
    o = hbmc.hbmc_order(A, bs, w)
    m = hbmc.hbmc_matrix_create(o, A).upload(device)
    xs = {}
    for name, prec in (("f64", hbmc.HBMC_F64), ("f32", hbmc.HBMC_F32)):
        sv = hbmc.Solver(o, hbmc.ic0_factor(o, A, prec).upload(device), m)
        t, (x, st) = _timed(lambda: sv.solve(b, tol=tol))
        xs[name] = x.cpu().numpy()
        res[name] = {"ms": round(t * 1e3, 3), **_stats(st)}
        log(f"[ext fp32] {name}: {t * 1e3:.2f} ms, {st.iters} its, true res {st.true_rel_res:.2e}")
    res["speedup"] = round(res["f64"]["ms"] / res["f32"]["ms"], 3)
    res["rel_diff_x_f32_vs_f64"] = float(np.linalg.norm(xs["f32"] - xs["f64"]) / np.linalg.norm(xs["f64"]))
    return res


def locality(device, npts=1_000_000, bs=2, w=32, tol=1e-7, reps=20, log=print):
    """The kNN problem in the input's (shuffled) numbering and renumbered by
    reverse Cuthill-McKee before the ordering: the paper's blocking seeds in
    the input numbering, so its layouts inherit that numbering's locality,
    and the gathers of the substitutions and the SpMV follow it.  Each
    apply and solve is also timed with one launch per color phase."""
    import time
    import torch
    A = inputs.knn_laplacian(npts, 13, 4, 5, shift=1e-3)
    b = torch.from_numpy(inputs.uniform_rhs(A.n, 3)).to(device)
    res = {"workload": f"13-NN Laplacian of {npts} uniform points (numbering shuffled), 1/dist weights, "
                       f"shift 1e-3, b~U[-1,1], HBMC bs={bs} w={w}, tol {tol:g}"}
    for numbering in ("input", "rcm"):
        t0 = time.perf_counter()
        o = hbmc.hbmc_order(A, bs, w, rcm=numbering == "rcm")
        t_order = time.perf_counter() - t0
        m = hbmc.hbmc_matrix_create(o, A).upload(device)
        r = {"order_s": round(t_order, 3), "n_colors": o.n_colors}
        for name, prec in (("f64", hbmc.HBMC_F64), ("f32", hbmc.HBMC_F32)):
            ap = apply_rate(device, A, bs, w, prec, reps=reps, order=o, log=log,
                            label=f"locality {numbering} {name}")
            sv = hbmc.Solver(o, hbmc.ic0_factor(o, A, prec).upload(device), m)
            t, (x, st) = _timed(lambda: sv.solve(b, tol=tol))
            # the same solve with one launch per color phase (same bits)
            sv.factor.set_sync(hbmc.HBMC_SYNC_LAUNCH)
            tl, (xl, stl) = _timed(lambda: sv.solve(b, tol=tol), reps=2)
            if stl.iters != st.iters or not torch.equal(xl, x):
                raise RuntimeError("one launch and a launch per phase gave different solves")
            r[name] = {"apply_us_cold": ap["median_us_cold"], "apply_us_cold_launches": ap["median_us_cold_launches"],
                       "apply_frac": ap["frac"], "solve_ms": round(t * 1e3, 3),
                       "solve_ms_launches": round(tl * 1e3, 3), **_stats(st)}
            log(f"[ext locality] {numbering} {name}: apply {ap['median_us_cold']:.1f} us, solve {t * 1e3:.2f} ms "
                f"(a launch per phase: {ap['median_us_cold_launches']:.1f} us, {tl * 1e3:.2f} ms), "
                f"{st.iters} its, true res {st.true_rel_res:.2e}")
        res[numbering] = r
        del m
        torch.cuda.empty_cache()
    res["speedup_f64"] = round(res["input"]["f64"]["solve_ms"] / res["rcm"]["f64"]["solve_ms"], 3)
    res["speedup_f32_over_input_f64"] = round(res["input"]["f64"]["solve_ms"] / res["rcm"]["f32"]["solve_ms"], 3)
    return res


def fp32_grid(device, N=128, bs=8, w=64, tol=1e-7, log=print):
    """FP32 against FP64 preconditioner on the 128^3 diffusion problem, where
    an iteration is bound by HBM bandwidth (the factor is half the bytes)."""
    import torch
    A = inputs.diffusion3d(N, 1.0, 2)
    b = torch.from_numpy(inputs.uniform_rhs(A.n, 3)).to(device)
    res = {"workload": f"diffusion3d {N}^3 lognormal sigma=1 seed 2, b~U[-1,1] seed 3, HBMC bs={bs} w={w}, "
                       f"tol {tol:g}"}
    o = hbmc.hbmc_order(A, bs, w)
    m = hbmc.hbmc_matrix_create(o, A).upload(device)
    xs = {}
    for name, prec in (("f64", hbmc.HBMC_F64), ("f32", hbmc.HBMC_F32)):
        sv = hbmc.Solver(o, hbmc.ic0_factor(o, A, prec).upload(device), m)
        t, (x, st) = _timed(lambda: sv.solve(b, tol=tol))
        xs[name] = x.cpu().numpy()
        res[name] = {"ms": round(t * 1e3, 3), **_stats(st)}
        log(f"[ext fp32 grid] {name}: {t * 1e3:.2f} ms, {st.iters} its, true res {st.true_rel_res:.2e}")
    res["speedup"] = round(res["f64"]["ms"] / res["f32"]["ms"], 3)
    res["rel_diff_x_f32_vs_f64"] = float(np.linalg.norm(xs["f32"] - xs["f64"]) / np.linalg.norm(xs["f64"]))
    return res


def batch(device, count=128, lo=16, hi=64, seed=7, bs=8, w=64, tol=1e-7, tune=True, log=print):
    """Uneven batch in one set of launches (autotuned bs, w and kernel, FP32
    preconditioner) against one-by-one FP64 solves (bs 8, w 64)."""
    import torch
    sizes = inputs.batch_sizes(count, seed, lo, hi)
    log(f"[ext batch] {count} Poisson systems, N in [{sizes.min()}, {sizes.max()}]")
    mats = [inputs.poisson3d(int(N)) for N in sizes]
    A, sys_ptr = inputs.block_diag(mats)
    rhs = [inputs.uniform_rhs(M.n, 1000 + s) for s, M in enumerate(mats)]
    res = {"workload": f"{count} 7-point Poisson systems, N ~ U{{{lo}..{hi}}} (seed {seed}), "
                       f"n total {A.n}, b~U[-1,1], tol {tol:g}"}
    bb = torch.from_numpy(np.concatenate(rhs)).to(device)
    kernel = hbmc.HBMC_KERNEL_AUTO
    if tune:
        choice = autotune.tune(A, bb, sys_ptr=sys_ptr, precision=hbmc.HBMC_F32, tol=tol, bs_list=(4, 8, 16),
                               w_list=(32, 64), reps=1, device=device, log=log)
        bs, w, kernel = choice.bs, choice.w, choice.kernel
        res["autotune"] = {"bs": bs, "w": w, "kernel": kernel,
                           "trials": [[t.bs, t.w, t.kernel, round(t.seconds * 1e3, 2), t.iters]
                                      for t in choice.trials]}
        del choice
        torch.cuda.empty_cache()
    t0 = time.perf_counter()
    sv = hbmc.Solver.setup(A, bs, w, hbmc.HBMC_F32, device=device, sys_ptr=sys_ptr, kernel=kernel)
    res["setup_s"] = round(time.perf_counter() - t0, 2)
    t, (x, st) = _timed(lambda: sv.solve(bb, tol=tol))
    res["batched_f32"] = {"ms": round(t * 1e3, 3), "bs": bs, "w": w, "kernel": kernel, **_stats(st)}
    log(f"[ext batch] batched FP32 (bs={bs} w={w} kernel={kernel}): {t * 1e3:.2f} ms")
    del sv
    # the same batch and knobs with the FP64 preconditioner: batching alone
    sv = hbmc.Solver.setup(A, bs, w, hbmc.HBMC_F64, device=device, sys_ptr=sys_ptr, kernel=kernel)
    t64, (x, st) = _timed(lambda: sv.solve(bb, tol=tol))
    res["batched_f64"] = {"ms": round(t64 * 1e3, 3), "bs": bs, "w": w, "kernel": kernel, **_stats(st)}
    log(f"[ext batch] batched FP64 (bs={bs} w={w} kernel={kernel}): {t64 * 1e3:.2f} ms")
    del sv
    bs, w = 8, 64
    total, its, worst, conv = 0.0, [], 0.0, True
    for s, M in enumerate(mats):
        one = hbmc.Solver.setup(M, bs, w, hbmc.HBMC_F64, device=device)
        b1 = torch.from_numpy(rhs[s]).to(device)
        t1, (x1, st1) = _timed(lambda: one.solve(b1, tol=tol), reps=1)
        total += t1
        its.append(st1.iters)
        worst = max(worst, st1.true_rel_res)
        conv = conv and st1.status == hbmc.HBMC_OK
    res["one_by_one_f64"] = {"ms": round(total * 1e3, 3), "iters_max": max(its), "iters_min": min(its),
                             "true_rel_res_max": worst, "all_converged": conv}
    res["speedup"] = round(total / t, 3)
    res["speedup_batching_alone_f64"] = round(total / t64, 3)
    res["speedup_f32_over_f64_batched"] = round(t64 / t, 3)
    log(f"[ext batch] one by one FP64: {total * 1e3:.2f} ms, speedup {total / t:.2f} "
        f"(batching alone, FP64: {total / t64:.2f}; FP32 over FP64 batched: {t64 / t:.2f})")
    return res


def rhs(device, N=128, K=32, tol=1e-7, tune=True, log=print):
    """K right-hand sides together against K single FP64 solves."""
    import torch
    log(f"[ext rhs] {N}^3 diffusion, K={K}")
    A = inputs.diffusion3d(N, 1.0, 2)
    B = np.stack([inputs.uniform_rhs(A.n, 500 + q) for q in range(K)], axis=1)
    Bd = torch.from_numpy(np.ascontiguousarray(B).ravel()).to(device)
    res = {"workload": f"diffusion3d {N}^3 lognormal sigma=1 seed 2, {K} right-hand sides "
                       f"b_q~U[-1,1] (seeds 500..), tol {tol:g}"}
    choice = None
    if tune:
        choice = autotune.tune(A, Bd, nrhs=K, precision=hbmc.HBMC_F32, tol=tol, bs_list=(4, 8, 16),
                               w_list=(16, 32, 64), tiles=(4, 8, 16), reps=1, device=device, log=log)
        res["autotune"] = {"bs": choice.bs, "w": choice.w, "rhs_tile": choice.rhs_tile,
                           "trials": [[t.bs, t.w, t.rhs_tile, round(t.seconds * 1e3, 2), t.iters]
                                      for t in choice.trials]}
    bs, w, tile = (choice.bs, choice.w, choice.rhs_tile) if choice else (8, 64, 0)
    sv = hbmc.Solver.setup(A, bs, w, hbmc.HBMC_F32, device=device)
    sv.factor.set_rhs_tile(tile)
    t, (x, st) = _timed(lambda: sv.solve(Bd, nrhs=K, tol=tol), reps=2)
    res["multi_f32"] = {"ms": round(t * 1e3, 3), "bs": bs, "w": w, "rhs_tile": tile, **_stats(st)}
    log(f"[ext rhs] {K} together (FP32 preconditioner, bs={bs} w={w} tile={tile}): {t * 1e3:.2f} ms")
    del sv
    one = hbmc.Solver.setup(A, 8, 64, hbmc.HBMC_F64, device=device)
    cols = [torch.from_numpy(np.ascontiguousarray(B[:, q])).to(device) for q in range(K)]

    def singles():
        return [one.solve(c, tol=tol) for c in cols]
    t1, outs = _timed(singles, reps=1)
    res["singles_f64"] = {"ms": round(t1 * 1e3, 3), "bs": 8, "w": 64, **_stats([o[1] for o in outs])}
    res["speedup"] = round(t1 / t, 3)
    log(f"[ext rhs] {K} single FP64 solves: {t1 * 1e3:.2f} ms, speedup {t1 / t:.2f}")
    return res


def graph(solver, b, tol=1e-7, log=print):
    """The same solve with the iterations as a replayed hipGraph and
    launched one by one."""
    out = {}
    for name, ug in (("graph", True), ("eager", False)):
        t, (x, st) = _timed(lambda: solver.solve(b, tol=tol, use_graph=ug, check_every=16))
        out[name] = {"ms": round(t * 1e3, 3), **_stats(st)}
        log(f"[ext graph] {name}: {t * 1e3:.2f} ms")
    out["speedup"] = round(out["eager"]["ms"] / out["graph"]["ms"], 3)
    return out


def orderings(device, N=128, bs=8, w=64, tol=1e-7, log=print):
    """MC, BMC and HBMC ICCG on the 128^3 diffusion problem.  MC is the
    ordering with blocks of one unknown (more colors, more iterations); BMC
    keeps the blocks but each lane walks its own block, so a warp touches
    rows bs apart; HBMC has BMC's iterations with unit-stride lanes."""
    import torch
    A = inputs.diffusion3d(N, 1.0, 2)
    b = torch.from_numpy(inputs.uniform_rhs(A.n, 3)).to(device)
    res = {"workload": f"diffusion3d {N}^3 lognormal sigma=1 seed 2, b~U[-1,1] seed 3, FP64, tol {tol:g}"}
    for name, obs, ow in (("mc", 1, w), ("bmc", bs, 1), ("hbmc", bs, w)):
        t0 = time.perf_counter()
        sv = hbmc.Solver.setup(A, obs, ow, hbmc.HBMC_F64, device=device)
        setup = time.perf_counter() - t0
        t, (x, st) = _timed(lambda: sv.solve(b, tol=tol))
        res[name] = {"bs": obs, "w": ow, "colors": sv.order.n_colors, "ms": round(t * 1e3, 3),
                     "ms_per_iter": round(t * 1e3 / max(1, st.iters), 4), "setup_s": round(setup, 2),
                     **_stats(st)}
        log(f"[ext orderings] {name} bs={obs} w={ow}: {sv.order.n_colors} colors, "
            f"{st.iters} its, {t * 1e3:.2f} ms ({t * 1e3 / max(1, st.iters):.3f} ms/it)")
        del sv
    res["hbmc_vs_mc"] = round(res["mc"]["ms"] / res["hbmc"]["ms"], 3)
    res["hbmc_vs_bmc"] = round(res["bmc"]["ms"] / res["hbmc"]["ms"], 3)
    return res


def smooth_bytes(n_pad: int, nnz_a: int, nnz_l: int, forward_only: bool = False) -> int:
    """Algorithmic bytes of one FP64 smoothing step x += c M^-1 (b - A x):
    the residual reads A (value and int32 index per entry), x and b and
    writes r; the substitutions read L (value and index per entry, once per
    direction), diaginv per direction, r, and write z (with the intermediate
    y written and read back between the directions); the update reads x, z
    and writes x."""
    resid = nnz_a * 12 + 3 * n_pad * 8
    if forward_only:
        subst = nnz_l * 12 + 3 * n_pad * 8
    else:
        subst = 2 * nnz_l * 12 + 2 * n_pad * 8 + 2 * n_pad * 8 + 2 * n_pad * 8
    return resid + subst + 3 * n_pad * 8


def smoother(device, N=128, bs=8, w=64, steps=20, tol=1e-7, log=print):
    """Smoothing steps and SSOR-PCG on the 128^3 diffusion problem (FP64)."""
    import torch
    A = inputs.diffusion3d(N, 1.0, 2)
    b = inputs.uniform_rhs(A.n, 3)
    res = {"workload": f"diffusion3d {N}^3 lognormal sigma=1 seed 2, b~U[-1,1] seed 3, HBMC bs={bs} w={w}, "
                       f"FP64, {steps} steps timed"}
    o = hbmc.hbmc_order(A, bs, w)
    m = hbmc.hbmc_matrix_create(o, A).upload(device)
    f = hbmc.ssor_factor(o, A, hbmc.HBMC_F64, 1.0).upload(device)
    nnz_l = int(f.export()[1][-1])
    nnz_a = int(A.rowptr[-1])
    bb = hbmc.hbmc_to_hbmc(f, torch.from_numpy(b).to(device))
    work = hbmc.smooth_workspace(f, 1, device)
    stream = torch.cuda.current_stream()
    for name, mode, fo in (("symmetric_gs", hbmc.HBMC_SMOOTH_SYMMETRIC, False),
                           ("forward_gs", hbmc.HBMC_SMOOTH_FORWARD, True)):
        x = torch.zeros_like(bb)
        hbmc.hbmc_smooth(f, m, bb, x, sweeps=2, mode=mode, work=work)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        hbmc.hbmc_smooth(f, m, bb, x, sweeps=steps, mode=mode, work=work)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / steps
        nbytes = smooth_bytes(f.n_pad, nnz_a, nnz_l, fo)
        r = bb - hbmc.hbmc_spmv(m, x)
        res[name] = {"ms_per_step": round(ms, 4), "bytes_per_step": nbytes,
                     "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1),
                     "rel_res_after": float(torch.linalg.norm(r) / torch.linalg.norm(bb))}
        log(f"[ext smoother] {name}: {ms * 1e3:.1f} us/step, {nbytes / 1e6:.1f} MB -> "
            f"{nbytes / (ms * 1e-3) / 1e9:.0f} GB/s")
    bd = torch.from_numpy(b).to(device)
    for name, omega in (("ic0_pcg", None), ("ssor_pcg", 1.0), ("ssor_pcg_1.5", 1.5)):
        sv = hbmc.Solver.setup(A, bs, w, hbmc.HBMC_F64, device=device, omega=omega)
        t, (x, st) = _timed(lambda: sv.solve(bd, tol=tol))
        res[name] = {"ms": round(t * 1e3, 3), **_stats(st)}
        log(f"[ext smoother] {name}: {st.iters} its, {t * 1e3:.2f} ms")
        del sv
    return res


def refactor(device, N=128, bs=8, w=64, reps=3, log=print):
    """New values of the same pattern: host rebuild (ordering kept) against
    the device refactorization; both give the same device images."""
    import torch
    A = inputs.diffusion3d(N, 1.0, 2)
    B = inputs.diffusion3d(N, 1.0, 5)
    o = hbmc.hbmc_order(A, bs, w)
    f = hbmc.ic0_factor(o, A).upload(device)
    m = hbmc.hbmc_matrix_create(o, A).upload(device)
    rv = hbmc.Revalue(o, A).upload(device)
    vb = torch.from_numpy(B.val).to(device)
    res = {"workload": f"diffusion3d {N}^3: coefficients of seed 2 replaced by those of seed 5 (same pattern), "
                       f"HBMC bs={bs} w={w}, FP64"}

    def host():
        fh = hbmc.ic0_factor(o, B).upload(device)
        mh = hbmc.hbmc_matrix_create(o, B).upload(device)
        return fh, mh

    def dev():
        hbmc.ic0_refactor(f, rv, vb)
        hbmc.hbmc_matrix_revalue(m, rv, vb)
        return f, m
    t_host, _ = _timed(host, reps)
    t_dev, _ = _timed(dev, reps)
    res["host_rebuild_ms"] = round(t_host * 1e3, 2)
    res["device_refactor_ms"] = round(t_dev * 1e3, 3)
    res["speedup"] = round(t_host / t_dev, 1)
    log(f"[ext refactor] host rebuild {t_host * 1e3:.1f} ms, device refactor {t_dev * 1e3:.2f} ms")
    return res


def _main():
    import argparse
    import json
    import sys
    import torch
    ap = argparse.ArgumentParser(description="ic0_apply alone on one workload, caches cold before each call")
    ap.add_argument("what", choices=["apply", "solve"],
                    help="apply: ic0_apply timed cold and warm; solve: ICCG to 1e-7 (b ~ U[-1, 1], seed 6)")
    ap.add_argument("--solves", type=int, default=2, help="solve: timed solves after one untimed")
    ap.add_argument("workload", choices=sorted(WORKLOADS))
    ap.add_argument("--bs", type=int, default=8)
    ap.add_argument("--w", type=int, default=64)
    ap.add_argument("--precision", choices=["f64", "f32"], default="f64")
    ap.add_argument("--kernel", choices=["auto", "sweep", "rows"], default="auto")
    ap.add_argument("--rcm", action="store_true", help="order after the reverse Cuthill-McKee renumbering")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--modes", default="cold,warm")
    ap.add_argument("--calibrate", action="store_true",
                    help="first run dst = 2 * src on 256 MiB tensors, a kernel that reads and writes exactly "
                         "256 MiB, for scaling hardware byte counters")
    a = ap.parse_args()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)
    if a.calibrate:
        src = torch.ones(1 << 25, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    A = WORKLOADS[a.workload]()
    prec = hbmc.HBMC_F64 if a.precision == "f64" else hbmc.HBMC_F32
    kern = {"auto": hbmc.HBMC_KERNEL_AUTO, "sweep": hbmc.HBMC_KERNEL_SWEEP, "rows": hbmc.HBMC_KERNEL_ROWS}[a.kernel]
    log = lambda *x: print(*x, file=sys.stderr, flush=True)  # noqa: E731
    if a.what == "solve":
        o = hbmc.hbmc_order(A, a.bs, a.w, rcm=a.rcm)
        solver = hbmc.Solver(o, hbmc.ic0_factor(o, A, prec).set_kernel(kern).upload(dev),
                             hbmc.hbmc_matrix_create(o, A).upload(dev))
        b = torch.from_numpy(inputs.uniform_rhs(A.n, 6)).to(dev)
        work = hbmc.workspace(solver.factor, 1, dev)
        t, (x, st) = _timed(lambda: solver.solve(b, tol=1e-7, work=work), reps=a.solves)
        out = {"workload": a.workload, "bs": a.bs, "w": a.w, "precision": a.precision, "kernel": a.kernel,
               "rcm": a.rcm,
               "ms_to_1e-7": round(t * 1e3, 3), "iterations": st.iters, "true_rel_res": st.true_rel_res,
               "ms_per_iteration": round(t * 1e3 / max(st.iters, 1), 4)}
        log(f"[solve {a.workload}] {out['ms_to_1e-7']} ms, {st.iters} iterations")
        print(json.dumps(out), flush=True)
        return
    out = apply_rate(dev, A, a.bs, a.w, prec, kern, a.reps, modes=tuple(a.modes.split(",")), log=log,
                     order=hbmc.hbmc_order(A, a.bs, a.w, rcm=True) if a.rcm else None,
                     label=f"{a.workload} bs {a.bs} w {a.w} {a.precision} {a.kernel}{' rcm' if a.rcm else ''}")
    out.update(workload=a.workload, kernel=a.kernel, rcm=a.rcm)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    _main()

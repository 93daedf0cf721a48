#!/usr/bin/env python3
"""Benchmark of the HBMC-ordered IC(0)-CG hot path on one MI355X.

Workload: 3D 7-point cell-centred diffusion on 128^3 (n = 2,097,152) with
lognormal (sigma = 1) face coefficients from seed 2, b ~ U[-1, 1] from seed
3, HBMC with bs = 8, w = 64, FP64 throughout, x0 = 0, tol 1e-7.

A step is one ICCG solve to ||r||/||b|| < 1e-7 (SpMV, dots, vector updates
and one ic0_apply per iteration, plus the permutations in and out).  The
headline value is the ic0_apply rate in algorithmic GB/s: bytes the
substitutions must move (factor values and indices read once, diaginv, r
in, z out, y out and back) divided by the apply's measured time, with the
caches cold before each timed apply: 1 GiB is written (evicting the apply's
data from L2 and the 256 MB MALL), then a different 1 GiB is read (so the
MALL holds clean lines and the apply's misses do not pay for write-backs of
the flush).  The write-only flush time is reported too.

Prints one JSON line on stdout; everything else goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "ic0_apply GB/s (% HBM peak); ICCG time-to-1e-7 residual vs plain FP64"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# committed rocprofv3 byte-counter summaries per workload, and the kernel
# sources each was taken with (the summary records a hash of them)
PROFILES = {
    "diffusion128": ("ic0_apply_diffusion128.md", ["paper_1908_00741_amd/csrc/sweep.h",
                                                   "paper_1908_00741_amd/csrc/sweep_bs8.hip",
                                                   "paper_1908_00741_amd/csrc/factor.cpp",
                                                   "paper_1908_00741_amd/csrc/hbmc_internal.h"]),
    "knn1m": ("ic0_apply_knn1m.md", ["paper_1908_00741_amd/csrc/sweep.h",
                                     "paper_1908_00741_amd/csrc/sweep_bs2.hip",
                                     "paper_1908_00741_amd/csrc/flow.h",
                                     "paper_1908_00741_amd/csrc/substitution.hip",
                                     "paper_1908_00741_amd/csrc/factor.cpp",
                                     "paper_1908_00741_amd/csrc/hbmc_internal.h"]),
    "knn1m_rcm": ("ic0_apply_knn1m_rcm.md", ["paper_1908_00741_amd/csrc/sweep.h",
                                             "paper_1908_00741_amd/csrc/sweep_bs2.hip",
                                             "paper_1908_00741_amd/csrc/flow.h",
                                             "paper_1908_00741_amd/csrc/substitution.hip",
                                             "paper_1908_00741_amd/csrc/factor.cpp",
                                             "paper_1908_00741_amd/csrc/hbmc_internal.h"]),
}


def measured_traffic(workload="diffusion128"):
    """HBM bytes per FP64 ic0_apply from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of the workload, or None when the kernel sources
    changed since it was taken."""
    import hashlib
    name, sources = PROFILES[workload]
    try:
        text = open(os.path.join(ROOT, "profiles", name)).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("traffic_bytes_per_apply: ", "source_sha256_16: ")))
    if fields.get("source_sha256_16", "").strip() != h.hexdigest()[:16]:
        return None
    return int(float(fields["traffic_bytes_per_apply"]))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--ext", default="fp32,locality,fp32_grid,batch,rhs,graph,orderings,smoother,refactor,warmstart",
                    help="comma-separated extension comparisons to run after the headline "
                         "(fp32, locality, fp32_grid, batch, rhs, graph, orderings, smoother, refactor, "
                         "warmstart); "
                         "empty for none")
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the ic0_apply timings of the 1M-point kNN and 96^3 workloads")
    ap.add_argument("--calibrate", action="store_true",
                    help="first run dst = 2 * src on 256 MiB tensors, a kernel that reads "
                         "and writes exactly 256 MiB, for scaling hardware byte counters")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the hot path has no multi-GPU form in this "
              "library (run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1908_00741_amd import hbmc, inputs

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.calibrate:
        src = torch.ones(1 << 25, dtype=torch.float64, device=dev)    # 256 MiB
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    N, bs, w = args.N, 8, 64
    log(f"[bench] building 128^3 workload N={N}")
    A = inputs.diffusion3d(N, 1.0, 2)
    b_np = inputs.uniform_rhs(A.n, 3)
    # setup, stage by stage: the ordering (host), then the factor and the
    # matrix built on the host and uploaded, and the same built on the
    # device from the CSR (same images)
    t0 = time.perf_counter()
    order = hbmc.hbmc_order(A, bs, w)
    t1 = time.perf_counter()
    fh = hbmc.ic0_factor(order, A, hbmc.HBMC_F64)
    t2 = time.perf_counter()
    mh = hbmc.hbmc_matrix_create(order, A)
    t3 = time.perf_counter()
    fh.upload(dev)
    mh.upload(dev)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    solver = hbmc.Solver(order, fh, mh)
    setup_s = t4 - t0
    db = hbmc.device_build(order, A, hbmc.HBMC_F64, device=dev)     # warm-up (kernel loading)
    del db
    torch.cuda.empty_cache()
    db = hbmc.device_build(order, A, hbmc.HBMC_F64, device=dev)
    setup = {"order_s": round(t1 - t0, 4), "host_factor_s": round(t2 - t1, 4), "host_matrix_s": round(t3 - t2, 4),
             "upload_s": round(t4 - t3, 4), "host_total_s": round(setup_s, 4),
             "device_csr_upload_s": round(db.seconds["csr_upload"], 4),
             "device_build_s": round(db.seconds["build"], 4),
             "device_total_s": round(t1 - t0 + db.seconds["csr_upload"] + db.seconds["build"], 4),
             "host_threads": os.cpu_count()}
    same = bool(torch.equal(db.factor.dev[: fh.device_bytes()], fh.dev[: fh.device_bytes()]) and
                torch.equal(db.matrix.dev[: mh.device_bytes()], mh.dev[: mh.device_bytes()]))
    setup["device_images_equal_host"] = same
    del db
    torch.cuda.empty_cache()
    log(f"[bench] setup: {setup}")
    f = solver.factor
    nnz_lower = (A.nnz - A.n) // 2
    from paper_1908_00741_amd.experiments import apply_bytes
    B = apply_bytes(f.n_pad, nnz_lower)
    log(f"[bench] setup {setup_s:.2f} s, n_pad {f.n_pad}, colors {f.n_colors}, "
        f"apply bytes {B / 1e6:.1f} MB")

    # ---- ic0_apply timing ------------------------------------------------
    from paper_1908_00741_amd import experiments
    perm, _ = solver.order.perm()
    r_np = np.zeros(f.n_pad)
    r_np[perm] = np.random.default_rng(17).uniform(-1, 1, A.n)
    r = torch.from_numpy(r_np).to(dev)
    z = torch.empty_like(r)
    for _ in range(5):
        hbmc.ic0_apply(f, r, z)
    torch.cuda.synchronize()
    timer = experiments.ColdTimer(dev)

    def timed(reps, mode, fn=lambda: hbmc.ic0_apply(f, r, z)):
        return timer.times_ms(fn, reps, mode)

    t_cold = timed(args.apply_reps, "cold")
    t_dirty = timed(args.apply_reps, "dirty")
    t_warm = timed(args.apply_reps, "warm")
    log(f"[bench] apply cold: median {np.median(t_cold) * 1e3:.1f} us, after a write-only flush: "
        f"{np.median(t_dirty) * 1e3:.1f} us, warm: median {np.median(t_warm) * 1e3:.1f} us")
    gbs_cold = B / (np.median(t_cold) * 1e-3) / 1e9
    gbs_warm = B / (np.median(t_warm) * 1e-3) / 1e9
    # context: a plain 128 MB device copy (torch's) under each flush method
    # (the write-only flush leaves dirty lines whose write-backs the copy
    # then pays for)
    src = torch.zeros(1 << 24, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    copy_gbs = {mode: 2 * src.numel() * 8 / (np.median(timed(20, mode, lambda: dst.copy_(src))) * 1e-3) / 1e9
                for mode in ("cold", "dirty")}
    del src, dst
    log(f"[bench] 128 MB copy: {copy_gbs['cold']:.0f} GB/s cold, {copy_gbs['dirty']:.0f} GB/s after a "
        f"write-only flush")

    # ---- ic0_apply on the other workloads (same cold method) ---------------
    apply_cfg = {}
    if not args.no_configs:
        Ak = experiments.WORKLOADS["knn1m"]()
        ok = hbmc.hbmc_order(Ak, 2, 32)
        for name, Ac, oc, cbs, cw, prec in (
                ("knn1m_bs2_w32_f64", Ak, ok, 2, 32, hbmc.HBMC_F64),
                ("knn1m_bs2_w32_f32", Ak, ok, 2, 32, hbmc.HBMC_F32),
                ("diffusion96_bs8_w64_f64", experiments.WORKLOADS["diffusion96"](), None, 8, 64, hbmc.HBMC_F64)):
            apply_cfg[name] = experiments.apply_rate(dev, Ac, cbs, cw, prec, reps=args.apply_reps, timer=timer,
                                                     order=oc, log=log, label=name)
            if name == "knn1m_bs2_w32_f64":
                tk = measured_traffic("knn1m")
                us = apply_cfg[name]["median_us_cold"]
                apply_cfg[name]["traffic"] = tk
                apply_cfg[name]["measured_gbs"] = None if tk is None else round(tk / (us * 1e-6) / 1e9, 1)
            torch.cuda.empty_cache()
        del Ak, ok
        torch.cuda.empty_cache()

    # ---- ICCG steps --------------------------------------------------------
    b = torch.from_numpy(b_np).to(dev)
    x = torch.zeros_like(b)
    work = hbmc.workspace(f, 1, dev)
    st = None
    for _ in range(args.warmup):
        x, st = solver.solve(b, x, tol=1e-7, x0_zero=True, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        x, st = solver.solve(b, x, tol=1e-7, x0_zero=True, work=work)
        log(f"[bench] step {k}: {st.iters} iterations, true residual {st.true_rel_res:.2e}")
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
    log(f"[bench] ICCG {ms_per_step:.2f} ms per solve, {st.iters} iterations")
    x64 = x.cpu().numpy()
    # the same solve with the FP32 preconditioner (compared with the oracle below)
    f32 = hbmc.ic0_factor(solver.order, A, hbmc.HBMC_F32).upload(dev)
    x32, st32 = hbmc.Solver(solver.order, f32, solver.matrix).solve(b, tol=1e-7)
    x32 = x32.cpu().numpy()
    del f32

    # ---- extensions: speedups over plain FP64 single-RHS ICCG ---------------
    ext = {}
    wanted = [e for e in args.ext.split(",") if e]
    if wanted:
        for name in wanted:
            try:
                if name == "graph":
                    ext[name] = experiments.graph(solver, b, tol=1e-7, log=log)
                elif name == "fp32":
                    ext[name] = experiments.fp32(dev, log=log)
                elif name == "locality":
                    ext[name] = experiments.locality(dev, reps=args.apply_reps, log=log)
                    r64 = ext[name]["rcm"]["f64"]
                    tk = measured_traffic("knn1m_rcm")
                    r64["apply_traffic"] = tk
                    r64["apply_measured_gbs"] = None if tk is None else round(tk / (r64["apply_us_cold"] * 1e-6) / 1e9, 1)
                elif name == "fp32_grid":
                    ext[name] = experiments.fp32_grid(dev, log=log)
                elif name == "orderings":
                    ext[name] = experiments.orderings(dev, log=log)
                elif name == "smoother":
                    ext[name] = experiments.smoother(dev, log=log)
                elif name == "refactor":
                    ext[name] = experiments.refactor(dev, log=log)
                elif name == "batch":
                    ext[name] = experiments.batch(dev, log=log)
                elif name == "rhs":
                    ext[name] = experiments.rhs(dev, log=log)
                elif name == "warmstart":
                    ext[name] = experiments.warmstart(dev, log=log)
                else:
                    ext[name] = {"error": "unknown extension"}
            except Exception as e:   # reported in the JSON line, not fatal
                ext[name] = {"error": f"{type(e).__name__}: {e}"}
                log(f"[bench] extension {name} failed: {e}")
            torch.cuda.empty_cache()

    # ---- oracle on the host ------------------------------------------------
    cpu = None
    if not args.no_cpu:
        import oracle
        log("[bench] timing the oracle on the host")
        ref = oracle.system(A, bs, w)
        reps, tcpu = 0, 0.0
        while tcpu < args.cpu_seconds or reps < 3:
            t1 = time.perf_counter()
            oracle.apply(ref.Ab, ref.d, ref.fac, r_np)
            tcpu += time.perf_counter() - t1
            reps += 1
        bb = np.zeros(f.n_pad)
        bb[perm] = b_np
        t1 = time.perf_counter()
        res = oracle.pcg(ref.Ab, ref.d, ref.fac, bb, tol=1e-7, maxit=10000)
        t_sol = time.perf_counter() - t1
        xo = res.x[perm]
        err64 = float(np.linalg.norm(x64 - xo) / np.linalg.norm(xo))
        err32 = float(np.linalg.norm(x32 - xo) / np.linalg.norm(xo))
        log(f"[bench] against the oracle's FP64 solution: FP64 {err64:.2e}, FP32 preconditioner {err32:.2e}")
        cpu = {"value": round(B * reps / tcpu / 1e9, 4), "unit": "GB/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{reps} sequential FP64 ic0_apply calls on the same 128^3 workload "
                         f"({tcpu:.1f} s); oracle PCG to 1e-7: {res.iters} iterations in {t_sol:.1f} s "
                         f"({t_sol * 1e3 / max(res.iters, 1):.0f} ms/iteration)",
               "time_to_solution_s": round(t_sol, 2), "iterations": res.iters,
               "host_cpu_count": os.cpu_count(),
               "gpu_f64_rel_err_vs_oracle": err64, "gpu_f32_precond_rel_err_vs_oracle": err32,
               "gpu_f32_precond_iterations": st32.iters, "gpu_f32_precond_true_rel_res": st32.true_rel_res}

    traffic = measured_traffic()
    out = {
        "metric": METRIC, "value": round(gbs_cold, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"diffusion3d {N}^3 lognormal sigma=1 seed 2, b~U[-1,1] seed 3, "
                               f"HBMC bs={bs} w={w}, FP64, x0=0, tol 1e-7",
                   "n": A.n, "n_pad": f.n_pad, "nnz": A.nnz, "nnz_lower": nnz_lower,
                   "n_colors": f.n_colors, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": round(gbs_cold, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs_cold / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "basis": "achieved and frac use the algorithmic bytes of one apply (factor values and "
                              "int32 indices read once, diaginv twice, r in, z out, y out and back); "
                              "measured_* use the HBM bytes the counters report",
                     "measured_gbs": None if traffic is None else round(traffic / (np.median(t_cold) * 1e-3) / 1e9, 1),
                     "measured_frac": None if traffic is None else
                     round(traffic / (np.median(t_cold) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "kernel": "ic0_apply (2*n_colors-1 phase launches)",
                     "bytes_per_launch": B,
                     "cold_copy_gbs": round(copy_gbs["cold"], 1),
                     "copy_gbs_after_write_only_flush": round(copy_gbs["dirty"], 1)},
        "apply": {"median_us_cold": round(float(np.median(t_cold)) * 1e3, 2),
                  "median_us_after_write_only_flush": round(float(np.median(t_dirty)) * 1e3, 2),
                  "median_us_warm": round(float(np.median(t_warm)) * 1e3, 2),
                  "gbs_warm": round(gbs_warm, 2), "reps": args.apply_reps},
        "iccg": {"ms_to_1e-7": round(ms_per_step, 3), "iterations": st.iters,
                 "true_rel_res": st.true_rel_res, "ms_per_iteration": round(ms_per_step / max(st.iters, 1), 4),
                 "setup_s": round(setup_s, 2), "setup": setup},
        "apply_configs": apply_cfg,
        "cpu_baseline": cpu,
        "extensions": ext,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Timed search for the HBMC solver's knobs on the device at hand.

Three knobs, searched one after the other, each keeping the best value of
the ones before:

1. the BMC block size bs -- it changes the preconditioner (larger blocks
   usually mean fewer iterations and longer chains), so it is scored by the
   time of a whole solve to the tolerance;
2. the level-1 width w -- the iteration count does not depend on it (the
   HBMC ordering is equivalent to the BMC ordering of the same blocks,
   Section 3.3), only the speed does;
3. the kernel of the substitution phases (one right-hand side) or the
   right-hand-side tile (several) -- pure speed knobs.

Each trial is the median of ``reps`` timed solves after one untimed solve
(which also captures the solver's graphs).  Ties keep the earlier
candidate, so the choice is deterministic for deterministic timings.  The
setup and timing functions can be replaced (the tests do so on the CPU).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

from . import hbmc


@dataclass
class Trial:
    bs: int
    w: int
    kernel: int
    rhs_tile: int
    seconds: float
    iters: int


@dataclass
class Choice:
    bs: int
    w: int
    kernel: int
    rhs_tile: int
    seconds: float
    trials: list = field(default_factory=list)


def _default_setup(A, bs, w, precision, sys_ptr, device):
    return hbmc.Solver.setup(A, bs, w, precision, device=device, sys_ptr=sys_ptr)


def _default_measure(solver, b, nrhs, tol, reps):
    """Median wall time of reps solves (device synchronized), and the
    largest iteration count of the last solve."""
    import torch
    x, st = solver.solve(b, nrhs=nrhs, tol=tol)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = solver.solve(b, nrhs=nrhs, tol=tol)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    sts = st if isinstance(st, list) else [st]
    ts.sort()
    return ts[len(ts) // 2], max(s.iters for s in sts)


def tune(A, b, *, nrhs: int = 1, sys_ptr=None, precision: int = hbmc.HBMC_F64, tol: float = 1e-7,
         bs_list=(4, 8, 16), w_list=(16, 32, 64), tiles=(4, 8, 16),
         kernels=(hbmc.HBMC_KERNEL_SWEEP, hbmc.HBMC_KERNEL_ROWS), reps: int = 3, device="cuda",
         setup=None, measure=None, log=None) -> Choice:
    """Picks bs, w and the kernel (nrhs = 1) or right-hand-side tile
    (nrhs > 1) with the shortest solve of A x = b; b is a device vector
    [n][nrhs] in the original numbering.  Returns the choice and every
    trial."""
    make = setup or (lambda bs, w: _default_setup(A, bs, w, precision, sys_ptr, device))
    measure = measure or (lambda sv: _default_measure(sv, b, nrhs, tol, reps))
    trials = []
    built = {}

    def setup(bs, w):   # one setup per (bs, w)
        if (bs, w) not in built:
            built[(bs, w)] = make(bs, w)
        return built[(bs, w)]

    def trial(sv, bs, w, kernel, tile):
        if nrhs == 1:
            sv.factor.set_kernel(kernel)
        else:
            sv.factor.set_rhs_tile(tile)
        sec, its = measure(sv)
        t = Trial(bs, w, kernel, tile, sec, its)
        trials.append(t)
        if log:
            log(f"[autotune] bs={bs} w={w} kernel={kernel} tile={tile}: {sec * 1e3:.3f} ms, {its} its")
        return t

    def best(ts):
        out = ts[0]
        for t in ts[1:]:
            if t.seconds < out.seconds:
                out = t
        return out

    kernel0 = hbmc.HBMC_KERNEL_AUTO
    tile0 = 0
    w0 = max(w_list)
    # 1. block size, whole solves
    t_bs = best([trial(setup(bs, w0), bs, w0, kernel0, tile0) for bs in bs_list])
    # 2. level-1 width at that block size
    t_w = best([t_bs] + [trial(setup(t_bs.bs, w), t_bs.bs, w, kernel0, tile0)
                         for w in w_list if w != w0])
    # 3. kernel (one right-hand side) or right-hand-side tile
    sv = setup(t_bs.bs, t_w.w)
    if nrhs == 1:
        t_k = best([t_w] + [trial(sv, t_w.bs, t_w.w, k, tile0) for k in kernels])
    else:
        t_k = best([t_w] + [trial(sv, t_w.bs, t_w.w, kernel0, t) for t in tiles])
    return Choice(t_k.bs, t_k.w, t_k.kernel, t_k.rhs_tile, t_k.seconds, trials)


def apply_choice(solver, choice: Choice):
    """Sets the chosen kernel and tile on a solver built with choice.bs and
    choice.w."""
    solver.factor.set_kernel(choice.kernel)
    solver.factor.set_rhs_tile(choice.rhs_tile)
    return solver

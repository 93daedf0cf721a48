"""The autotuner's search on the CPU, with a stand-in solver and timer.

Pins: the staged search (block size by whole solves, then w, then kernel or
right-hand-side tile) returns the argmin of each stage, ties keep the
earlier candidate, every (bs, w) is set up once, and the same timings give
the same choice.
"""
from paper_1908_00741_amd import autotune, hbmc


class _Factor:
    def __init__(self):
        self.kernel, self.tile = hbmc.HBMC_KERNEL_AUTO, 0

    def set_kernel(self, k):
        self.kernel = k

    def set_rhs_tile(self, t):
        self.tile = t


class _Solver:
    def __init__(self, bs, w):
        self.bs, self.w, self.factor = bs, w, _Factor()


def _run(cost, nrhs=1, **kw):
    made = []

    def setup(bs, w):
        made.append((bs, w))
        return _Solver(bs, w)

    def measure(sv):
        return cost(sv.bs, sv.w, sv.factor.kernel, sv.factor.tile), 10

    ch = autotune.tune(None, None, nrhs=nrhs, setup=setup, measure=measure, **kw)
    return ch, made


def test_picks_stagewise_minimum():
    # bs 8 is fastest, then w 32, then the rows kernel
    def cost(bs, w, k, t):
        return {4: 3.0, 8: 2.0, 16: 2.5}[bs] + {16: 0.3, 32: 0.1, 64: 0.2}[w] + \
            {hbmc.HBMC_KERNEL_AUTO: 0.02, hbmc.HBMC_KERNEL_SWEEP: 0.05, hbmc.HBMC_KERNEL_ROWS: 0.0}[k]
    ch, made = _run(cost)
    assert (ch.bs, ch.w, ch.kernel) == (8, 32, hbmc.HBMC_KERNEL_ROWS)
    assert abs(ch.seconds - 2.1) < 1e-12
    assert len(made) == len(set(made))                   # one setup per (bs, w)
    assert [(t.bs, t.w) for t in ch.trials[:3]] == [(4, 64), (8, 64), (16, 64)]


def test_rhs_tile_stage_and_ties():
    # every tile costs the same: the first candidate that reached the
    # minimum stays (the automatic tile of the earlier stage)
    def cost(bs, w, k, t):
        return 1.0
    ch, _ = _run(cost, nrhs=32)
    assert (ch.bs, ch.w, ch.rhs_tile) == (4, 64, 0)
    def cost2(bs, w, k, t):
        return {0: 1.0, 4: 0.9, 8: 0.7, 16: 0.8}[t]
    ch2, _ = _run(cost2, nrhs=32)
    assert ch2.rhs_tile == 8


def test_deterministic():
    def cost(bs, w, k, t):
        return (bs * 7 % 5) + w / 100.0 + k / 1000.0
    a, _ = _run(cost)
    b, _ = _run(cost)
    assert (a.bs, a.w, a.kernel, a.rhs_tile) == (b.bs, b.w, b.kernel, b.rhs_tile)
    assert [(t.bs, t.w, t.kernel, t.rhs_tile, t.seconds) for t in a.trials] == \
           [(t.bs, t.w, t.kernel, t.rhs_tile, t.seconds) for t in b.trials]

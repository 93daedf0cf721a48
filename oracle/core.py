"""ctypes front end of the C oracle (``hbmc_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this module; only
the tests, the smoke check and the benchmark's CPU-baseline leg do.  It
shares no code with the HIP path: the two meet only at the seeded inputs.

Every function is a thin call into the C file, whose header states which
passage of the paper each step follows and the readings taken where the paper
is silent.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hbmc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, EINVAL, ENOTSYM, EDIAG, EBREAKDOWN, ENOMEM, ENOCONV = 0, -1, -2, -3, -4, -6, 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc, one thread of plain C, no FMA contraction."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = C.CDLL(LIB)
        i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
        P = C.c_void_p
        L.orc_check.argtypes = [i32, P, P, P]
        L.orc_blocking.argtypes = [i32, P, P, i32, P, P]
        L.orc_rcm.argtypes = [i32, P, P, P]
        L.orc_coloring.argtypes = [i32, P, P, i32, P, i32, P, P, P]
        L.orc_hbmc_perm.argtypes = [i32, i32, i32, P, i32, P, i32, P, P, P]
        L.orc_permute.argtypes = [i32, P, P, P, P, i64, P, P, P]
        L.orc_ic0.argtypes = [i64, P, P, P, f64, P, P]
        L.orc_apply.argtypes = [i64, P, P, P, P, P, P, P]
        L.orc_apply.restype = None
        L.orc_apply_f32.argtypes = [i64, P, P, P, P, P, P, P]
        L.orc_apply_f32.restype = None
        L.orc_spmv.argtypes = [i64, P, P, P, P, P]
        L.orc_spmv.restype = None
        L.orc_pcg.argtypes = [i64, P, P, P, P, P, i32, P, P, f64, i32, P, P]
        L.orc_sor_sweep.argtypes = [i64, P, P, P, P, P, f64, i32]
        L.orc_sor_sweep.restype = None
        L.orc_ssor_split.argtypes = [i64, P, P, P, f64, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


def _csr(A):
    return (np.ascontiguousarray(A.rowptr, np.int64), np.ascontiguousarray(A.col, np.int32),
            np.ascontiguousarray(A.val, np.float64))


class OracleError(RuntimeError):
    def __init__(self, what, status):
        super().__init__(f"{what}: status {status}")
        self.status = status


def check(A) -> int:
    rp, ci, v = _csr(A)
    return lib().orc_check(A.n, _p(rp), _p(ci), _p(v))


@dataclass
class Ordering:
    n: int
    bs: int
    w: int
    members: np.ndarray      # [n] unknowns block by block, insertion order
    nblocks: int
    block_of: np.ndarray     # [n]
    color: np.ndarray        # [nblocks]
    ncolors: int
    perm: np.ndarray         # [n] original -> HBMC index
    color_start: np.ndarray  # [ncolors+1] in unknowns
    n_pad: int


def order(A, bs: int, w: int) -> Ordering:
    """Blocking, greedy block coloring, padding and HBMC secondary reordering."""
    L = lib()
    rp, ci, _ = _csr(A)
    n = A.n
    members = np.empty(n, np.int32)
    nb = C.c_int32(0)
    st = L.orc_blocking(n, _p(rp), _p(ci), bs, _p(members), C.byref(nb))
    if st:
        raise OracleError("orc_blocking", st)
    nblocks = nb.value
    block_of = np.empty(n, np.int32)
    color = np.empty(nblocks, np.int32)
    nc = C.c_int32(0)
    st = L.orc_coloring(n, _p(rp), _p(ci), bs, _p(members), nblocks, _p(block_of),
                        _p(color), C.byref(nc))
    if st:
        raise OracleError("orc_coloring", st)
    perm = np.empty(n, np.int32)
    cstart = np.empty(nc.value + 1, np.int64)
    npad = C.c_int64(0)
    st = L.orc_hbmc_perm(n, bs, w, _p(members), nblocks, _p(color), nc.value, _p(perm),
                         _p(cstart), C.byref(npad))
    if st:
        raise OracleError("orc_hbmc_perm", st)
    return Ordering(n, bs, w, members, nblocks, block_of, color, nc.value, perm, cstart,
                    int(npad.value))


def rcm(A) -> np.ndarray:
    """Reverse Cuthill-McKee numbering (the locality pre-pass, outside the
    paper): entry k is the unknown numbered k."""
    rp, ci, _ = _csr(A)
    out = np.empty(A.n, np.int32)
    st = lib().orc_rcm(A.n, _p(rp), _p(ci), _p(out))
    if st:
        raise OracleError("orc_rcm", st)
    return out


@dataclass
class _Renumbered:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray


def renumber(A, order: np.ndarray):
    """P A P^T with row k of the result = row order[k] of A (rows sorted)."""
    inv = np.empty(A.n, np.int64)
    inv[order] = np.arange(A.n)
    rp = np.asarray(A.rowptr, np.int64)
    ci = np.asarray(A.col, np.int64)
    v = np.asarray(A.val, np.float64)
    rows, cols, vals = [], [], []
    new_rp = np.zeros(A.n + 1, np.int64)
    for k in range(A.n):
        u = int(order[k])
        c = inv[ci[rp[u]:rp[u + 1]]]
        srt = np.argsort(c, kind="stable")
        cols.append(c[srt])
        vals.append(v[rp[u]:rp[u + 1]][srt])
        new_rp[k + 1] = new_rp[k] + len(c)
    return _Renumbered(A.n, new_rp, np.concatenate(cols).astype(np.int32), np.concatenate(vals))


def order_rcm(A, bs: int, w: int) -> Ordering:
    """The HBMC ordering of A renumbered by rcm(A), with perm mapping A's own
    unknowns to HBMC positions (the other fields refer to the renumbered
    system)."""
    r = rcm(A)
    o = order(renumber(A, r), bs, w)
    inv = np.empty(A.n, np.int64)
    inv[r] = np.arange(A.n)
    o.perm = np.ascontiguousarray(o.perm[inv], np.int32)
    return o


@dataclass
class BatchOrdering:
    n: int
    n_pad: int
    ncolors: int
    perm: np.ndarray         # [n] original -> batch HBMC index
    color_start: np.ndarray  # [ncolors+1]
    seg: np.ndarray          # [ncolors, nsys+1] rows of (color, system)
    systems: list            # per-system Ordering


def batch_unit(bs: int) -> int:
    """Padding of a batch segment, in BMC blocks: whole groups of 64 blocks
    (a wavefront of lanes) that also fill whole parts of 256 rows."""
    return math.lcm(64, 256 // math.gcd(256, bs))


def order_batch(mats, bs: int, w: int) -> BatchOrdering:
    """Independent systems ordered together: each system is ordered alone
    (blocking, coloring, HBMC reordering of Section 3); the union is laid out
    color by color, and inside a color system after system, each system's
    share of the color padded with dummy blocks to a multiple of
    batch_unit(bs) BMC blocks.  Inside its segment a system's unknowns keep the offsets they
    have from the start of that color in the system's own ordering (the
    HBMC offset of the q-th block of a color depends only on q, bs and w)."""
    subs = [order(A, bs, w) for A in mats]
    nsys = len(subs)
    nc = max(o.ncolors for o in subs)
    counts = np.zeros((nc, nsys), np.int64)          # BMC blocks of (color, system)
    for s, o in enumerate(subs):
        counts[: o.ncolors, s] = np.bincount(o.color, minlength=o.ncolors)
    unit = batch_unit(bs)
    padded = (counts + unit - 1) // unit * unit * bs
    seg = np.zeros((nc, nsys + 1), np.int64)
    color_start = np.zeros(nc + 1, np.int64)
    at = 0
    for c in range(nc):
        color_start[c] = at
        for s in range(nsys):
            seg[c, s] = at
            at += padded[c, s]
        seg[c, nsys] = at
    color_start[nc] = at
    perm = np.empty(sum(o.n for o in subs), np.int64)
    first = 0
    for s, o in enumerate(subs):
        c_of = o.color[o.block_of]                   # color of each unknown
        perm[first: first + o.n] = seg[c_of, s] + (o.perm - o.color_start[c_of])
        first += o.n
    return BatchOrdering(int(perm.size), int(at), nc, perm.astype(np.int32), color_start, seg, subs)


@dataclass
class Permuted:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray


def permute(A, perm: np.ndarray, n_pad: int) -> Permuted:
    """Abar = P A P^T with identity rows for the dummy unknowns."""
    rp, ci, v = _csr(A)
    nnz2 = int(rp[-1]) + (n_pad - A.n)
    rp2 = np.empty(n_pad + 1, np.int64)
    ci2 = np.empty(nnz2, np.int32)
    v2 = np.empty(nnz2, np.float64)
    st = lib().orc_permute(A.n, _p(rp), _p(ci), _p(v), _p(np.ascontiguousarray(perm, np.int32)),
                           n_pad, _p(rp2), _p(ci2), _p(v2))
    if st:
        raise OracleError("orc_permute", st)
    return Permuted(n_pad, rp2, ci2, v2)


def ic0(Ab, shift: float = 0.0):
    """Returns (d, fac): the pivots and the factored copy of Ab's values."""
    rp, ci, v = _csr(Ab)
    d = np.empty(Ab.n, np.float64)
    fac = np.empty_like(v)
    st = lib().orc_ic0(Ab.n, _p(rp), _p(ci), _p(v), float(shift), _p(d), _p(fac))
    if st:
        raise OracleError("orc_ic0", st)
    return d, fac


def apply(Ab, d, fac, r, precision: str = "f64") -> np.ndarray:
    """z = M^-1 r in the reordered numbering."""
    rp, ci, _ = _csr(Ab)
    r = np.ascontiguousarray(r, np.float64)
    z = np.empty(Ab.n, np.float64)
    if precision == "f64":
        y = np.empty(Ab.n, np.float64)
        lib().orc_apply(Ab.n, _p(rp), _p(ci), _p(fac), _p(d), _p(r), _p(y), _p(z))
    else:
        y = np.empty(Ab.n, np.float32)
        lib().orc_apply_f32(Ab.n, _p(rp), _p(ci), _p(fac), _p(d), _p(r), _p(y), _p(z))
    return z


def spmv(Ab, x) -> np.ndarray:
    rp, ci, v = _csr(Ab)
    x = np.ascontiguousarray(x, np.float64)
    y = np.empty(Ab.n, np.float64)
    lib().orc_spmv(Ab.n, _p(rp), _p(ci), _p(v), _p(x), _p(y))
    return y


def sor_sweeps(Ab, b, x0, omega: float = 1.0, sweeps: int = 1, symmetric: bool = True) -> np.ndarray:
    """sweeps SOR steps in Ab's numbering: each a forward sweep, followed by
    a backward sweep when symmetric (SSOR; symmetric Gauss-Seidel at
    omega = 1)."""
    rp, ci, v = _csr(Ab)
    b = np.ascontiguousarray(b, np.float64)
    x = np.array(x0, np.float64, copy=True)
    for _ in range(sweeps):
        lib().orc_sor_sweep(Ab.n, _p(rp), _p(ci), _p(v), _p(b), _p(x), float(omega), 0)
        if symmetric:
            lib().orc_sor_sweep(Ab.n, _p(rp), _p(ci), _p(v), _p(b), _p(x), float(omega), 1)
    return x


def ssor_split(Ab, omega: float = 1.0):
    """(d, fac) of the SSOR splitting, usable with apply and pcg."""
    rp, ci, v = _csr(Ab)
    d = np.empty(Ab.n, np.float64)
    fac = np.empty_like(v)
    st = lib().orc_ssor_split(Ab.n, _p(rp), _p(ci), _p(v), float(omega), _p(d), _p(fac))
    if st:
        raise OracleError("orc_ssor_split", st)
    return d, fac


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    status: int
    hist: np.ndarray


def pcg(Ab, d, fac, b, x0=None, tol: float = 1e-7, maxit: int = 10000,
        precision: str = "f64") -> PCGResult:
    rp, ci, v = _csr(Ab)
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros(Ab.n) if x0 is None else np.array(x0, np.float64, copy=True)
    hist = np.full(maxit + 1, np.nan)
    it = C.c_int32(0)
    st = lib().orc_pcg(Ab.n, _p(rp), _p(ci), _p(v), _p(fac), _p(d),
                       1 if precision == "f32" else 0, _p(b), _p(x), float(tol), int(maxit),
                       C.byref(it), _p(hist))
    return PCGResult(x, it.value, st, hist[: it.value + 1])


def scaled_start(A, b, x0):
    """The start vector c x0 with c = (b, x0) / (x0, A x0), the multiple of
    x0 nearest the solution x* in the A-norm: ||c x0 - x*||_A^2 =
    c^2 (x0, A x0) - 2 c (b, x0) + ||x*||_A^2 is least there, and never above
    ||x*||_A^2, the error of a zero start, which it equals at c = 0.  c = 0
    (start from zero) when (b, x0) or (x0, A x0) is not > 0.  A safeguard of
    the learned warm start, which the paper does not have; CG minimizes the
    A-norm of the error (Section 2's ICCG is CG).  Plain FP64: the oracle's
    product with A (any numbering) and two inner products.  Returns (c, c x0)."""
    x0 = np.ascontiguousarray(x0, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    bx = float(np.dot(b, x0))
    xax = float(np.dot(x0, spmv(A, x0)))
    c = bx / xax if (bx > 0.0 and xax > 0.0) else 0.0
    return c, c * x0


@dataclass
class System:
    """A problem carried through the oracle: ordering, reordered matrix,
    factor.  ``solve`` maps b and x between the original and HBMC numbering."""
    A: object
    ordr: Ordering
    Ab: Permuted
    d: np.ndarray
    fac: np.ndarray

    def to_hbmc(self, v):
        out = np.zeros(self.ordr.n_pad)
        out[self.ordr.perm] = v
        return out

    def from_hbmc(self, vb):
        return np.asarray(vb)[self.ordr.perm]

    def solve(self, b, x0=None, tol=1e-7, maxit=10000, precision="f64") -> PCGResult:
        xb0 = None if x0 is None else self.to_hbmc(x0)
        res = pcg(self.Ab, self.d, self.fac, self.to_hbmc(b), xb0, tol, maxit, precision)
        return PCGResult(self.from_hbmc(res.x), res.iters, res.status, res.hist)


def system(A, bs: int, w: int, shift: float = 0.0, rcm: bool = False) -> System:
    st = check(A)
    if st:
        raise OracleError("orc_check", st)
    o = order_rcm(A, bs, w) if rcm else order(A, bs, w)
    Ab = permute(A, o.perm, o.n_pad)
    d, fac = ic0(Ab, shift)
    return System(A, o, Ab, d, fac)

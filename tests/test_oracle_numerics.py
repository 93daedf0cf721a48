"""Pins of the oracle's IC(0), preconditioner and PCG.

- IC(0) against a brute-force dense elimination with every update outside
  A's pattern discarded (n <= 400);
- IC(0) is pinned by its defining property: M = (D+L) D^-1 (D+L^T) agrees
  with A on A's pattern (no-fill incomplete factorization, Section 2 eq.
  "ILU"); where the ordering creates no fill M = A, so (D+L) D^-1/2 is the
  Cholesky factor from numpy;
- the preconditioner by the residual ||M z - r|| with M applied through
  plain sparse products (no substitution);
- PCG by numpy.linalg.solve, by scipy's CG run with the same preconditioner
  as a dense inverse, by M = A converging in one step, and by the exact
  solution x = 1 of b = A 1;
- the ordering equivalence of Section 3.1 / Section 4.2.1: BMC and HBMC give
  permuted factors, permuted preconditioned vectors, and the same iteration
  counts and residual histories.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from paper_1908_00741_amd import inputs


def _lower_upper(sysm):
    Ab = sysm.Ab
    S = sp.csr_matrix((sysm.fac, Ab.col, Ab.rowptr), shape=(Ab.n, Ab.n))
    L = sp.tril(S, k=-1).tocsr()
    D = sp.diags(sysm.d)
    return L, D


def _M(sysm):
    L, D = _lower_upper(sysm)
    Dinv = sp.diags(1.0 / sysm.d)
    return ((D + L) @ Dinv @ (D + L.T)).tocsr()


def _Abar(sysm):
    Ab = sysm.Ab
    return sp.csr_matrix((Ab.val, Ab.col, Ab.rowptr), shape=(Ab.n, Ab.n))


CASES = [
    ("random", lambda: inputs.random_spd(120, 0.05, 1), 4, 8),
    ("random_dense", lambda: inputs.random_spd(80, 0.15, 2), 3, 4),
    ("knn", lambda: inputs.knn_laplacian(400, k=8, seed_points=3, seed_perm=4), 8, 16),
    ("grid3d", lambda: inputs.diffusion3d(6, 1.0, 5), 2, 8),
]


@pytest.mark.parametrize("name,make,bs,w", CASES, ids=[c[0] for c in CASES])
def test_ic0_matches_A_on_pattern(orc, name, make, bs, w):
    s = orc.system(make(), bs, w)
    M, Ab = _M(s), _Abar(s)
    mask = Ab.copy(); mask.data[:] = 1.0
    R = (M - Ab).multiply(mask)
    scale = np.abs(Ab.data).max()
    assert np.abs(R.data).max() <= 1e-13 * scale if R.nnz else True
    assert np.all(s.d > 0)


@pytest.mark.parametrize("name,make,bs,w", CASES, ids=[c[0] for c in CASES])
def test_ic0_matches_dense_masked_elimination(orc, name, make, bs, w):
    """Brute force: Gaussian elimination of the dense reordered matrix in
    index order, every update that falls outside A's pattern discarded
    (zero-fill incomplete LDL^T); its pivots and multipliers L_ij = l_ij d_j
    equal the oracle's d and L."""
    s = orc.system(make(), bs, w)
    Ad = _Abar(s).toarray()
    keep = Ad != 0.0
    a = Ad.copy()
    n = a.shape[0]
    for k in range(n):
        piv = a[k, k]
        col = a[k + 1:, k].copy()
        upd = np.outer(col, col) / piv
        blk = a[k + 1:, k + 1:]
        blk -= np.where(keep[k + 1:, k + 1:], upd, 0.0)
    L, D = _lower_upper(s)
    assert np.allclose(np.diag(a), s.d, rtol=1e-13, atol=0)
    Ld = np.tril(a, -1)
    assert np.allclose(L.toarray(), Ld, rtol=0, atol=1e-13 * np.abs(Ad).max())


def test_ic0_has_fill_outside_pattern(orc):
    # a pattern with triangles: M differs from A off the pattern (IC(0) drops fill)
    s = orc.system(inputs.random_spd(80, 0.15, 2), 3, 4)
    M, Ab = _M(s), _Abar(s)
    assert abs(M - Ab).max() > 1e-6


def _star(n, seed):
    """Star graph whose centre has the largest index: every leaf has one
    later neighbour, so eliminating in index order creates no fill."""
    rng = np.random.default_rng(seed)
    c = n - 1
    w = rng.uniform(0.2, 1.0, size=n - 1)
    leaves = np.arange(n - 1)
    diag = np.concatenate([w + rng.uniform(0.1, 1.0, n - 1), [w.sum() + 0.5]])
    rows = np.concatenate([leaves, np.full(n - 1, c), np.arange(n)])
    cols = np.concatenate([np.full(n - 1, c), leaves, np.arange(n)])
    return inputs.from_scipy(sp.csr_matrix((np.concatenate([-w, -w, diag]), (rows, cols)),
                                           shape=(n, n)))


@pytest.mark.parametrize("make,bs,w", [
    (lambda: inputs.path_1d(40), 40, 1),       # one block grown along the path
    (lambda: _star(30, 0), 1, 1),              # leaves colored first, centre last
    (lambda: _star(45, 1), 1, 1),
])
def test_ic0_fill_free_is_cholesky(orc, make, bs, w):
    """On patterns whose ordering creates no fill, IC(0) is the complete
    Cholesky factorization: (D + L) D^-1/2 equals numpy's Cholesky factor."""
    s = orc.system(make(), bs, w)
    Ad = _Abar(s).toarray()
    Lc = np.linalg.cholesky(Ad)
    L, D = _lower_upper(s)
    ours = (D + L).toarray() @ np.diag(1.0 / np.sqrt(s.d))
    assert np.allclose(ours, Lc, rtol=0, atol=1e-14 * np.abs(Lc).max())


@pytest.mark.parametrize("N", [8, 16])
def test_ic0_grid_no_offdiagonal_update(orc, N):
    """Grid graphs have no triangles: L equals the strict lower part of Abar
    bit for bit, and d_i = a_ii - sum_{j<i} a_ij^2 / d_j."""
    s = orc.system(inputs.diffusion3d(N, 1.0, 7), 8, 8)
    Ab = _Abar(s)
    L, _ = _lower_upper(s)
    Lb = sp.tril(Ab, k=-1).tocsr()
    assert (L != Lb).nnz == 0
    d_expect = np.empty(Ab.shape[0])
    Lcsr = Lb
    for i in range(Ab.shape[0]):
        acc = Ab[i, i]
        for p in range(Lcsr.indptr[i], Lcsr.indptr[i + 1]):
            j = Lcsr.indices[p]
            acc = acc - Lcsr.data[p] * Lcsr.data[p] / d_expect[j]
        d_expect[i] = acc
    assert np.allclose(s.d, d_expect, rtol=1e-14, atol=0)


def test_ic0_breakdown(orc):
    # symmetric, positive diagonal, indefinite: the second pivot is negative
    A = inputs.from_scipy(sp.csr_matrix(np.array([[1.0, 2.0], [2.0, 1.0]])))
    o = orc.order(A, 1, 1)
    Ab = orc.permute(A, o.perm, o.n_pad)
    with pytest.raises(orc.OracleError) as e:
        orc.ic0(Ab)
    assert e.value.status == orc.EBREAKDOWN


def test_ic0_shift_scales_diagonal(orc):
    A = inputs.random_spd(50, 0.1, 5)
    s = orc.system(A, 2, 4, shift=0.3)
    M, Ab = _M(s), _Abar(s)
    target = Ab + 0.3 * sp.diags(Ab.diagonal())
    mask = Ab.copy(); mask.data[:] = 1.0
    assert np.abs((M - target).multiply(mask).data).max() < 1e-12


@pytest.mark.parametrize("name,make,bs,w", CASES, ids=[c[0] for c in CASES])
def test_apply_residual(orc, name, make, bs, w):
    s = orc.system(make(), bs, w)
    rng = np.random.default_rng(0)
    r = rng.standard_normal(s.Ab.n)
    z = orc.apply(s.Ab, s.d, s.fac, r)
    res = np.linalg.norm(_M(s) @ z - r) / np.linalg.norm(r)
    assert res < 1e-13
    zf = orc.apply(s.Ab, s.d, s.fac, r, precision="f32")
    assert np.linalg.norm(_M(s) @ zf - r) / np.linalg.norm(r) < 1e-4


@pytest.mark.parametrize("name,make,bs,w", CASES, ids=[c[0] for c in CASES])
def test_bmc_hbmc_equivalence(orc, name, make, bs, w):
    """Factors and preconditioned vectors of BMC (w = 1) and HBMC are
    permutations of each other."""
    A = make()
    sb = orc.system(A, bs, 1)
    sh = orc.system(A, bs, w)
    db, dh = sb.d[sb.ordr.perm], sh.d[sh.ordr.perm]
    assert np.allclose(db, dh, rtol=1e-14, atol=0)
    r = np.random.default_rng(1).standard_normal(A.n)
    zb = sb.from_hbmc(orc.apply(sb.Ab, sb.d, sb.fac, sb.to_hbmc(r)))
    zh = sh.from_hbmc(orc.apply(sh.Ab, sh.d, sh.fac, sh.to_hbmc(r)))
    assert np.linalg.norm(zb - zh) <= 1e-13 * np.linalg.norm(zb)


def test_pcg_small_vs_solve(orc):
    A = inputs.random_spd(150, 0.04, 11)
    b = inputs.uniform_rhs(A.n, 12)
    s = orc.system(A, 4, 8)
    res = s.solve(b, tol=1e-12, maxit=500)
    assert res.status == orc.OK
    x = np.linalg.solve(A.to_scipy().toarray(), b)
    kappa = np.linalg.cond(A.to_scipy().toarray())
    assert np.linalg.norm(res.x - x) <= kappa * 1e-12 * np.linalg.norm(x)


def test_pcg_matches_scipy_cg(orc):
    """Same iterates as scipy's CG given M^-1 as a dense matrix."""
    A = inputs.random_spd(100, 0.06, 13)
    s = orc.system(A, 3, 4)
    Ab = _Abar(s)
    Minv = np.linalg.inv(_M(s).toarray())
    bb = s.to_hbmc(inputs.uniform_rhs(A.n, 14))
    K = 8
    xs = []
    spla.cg(Ab, bb, x0=np.zeros(Ab.shape[0]), rtol=1e-30, atol=0.0, maxiter=K,
            M=spla.aslinearoperator(Minv), callback=lambda xk: xs.append(xk.copy()))
    ours = orc.pcg(s.Ab, s.d, s.fac, bb, tol=0.0, maxit=K)
    assert ours.status == orc.ENOCONV and ours.iters == K
    assert len(xs) == K
    assert np.linalg.norm(ours.x - xs[-1]) <= 1e-10 * np.linalg.norm(xs[-1])
    true_res = [np.linalg.norm(bb - Ab @ xk) / np.linalg.norm(bb) for xk in xs]
    assert np.allclose(ours.hist[1:], true_res, rtol=1e-8)


def test_pcg_fill_free_one_iteration(orc):
    A = _star(80, 4)                          # M = A: one step solves it
    s = orc.system(A, 1, 1)
    res = s.solve(inputs.uniform_rhs(A.n, 5), tol=1e-10)
    assert res.status == orc.OK and res.iters == 1


def test_pcg_c1_exact_solution(orc):
    A = inputs.grid2d_5pt(64)
    s = orc.system(A, 4, 8)
    res = s.solve(inputs.row_sums(A), tol=1e-7)
    assert res.status == orc.OK
    assert res.hist[-1] < 1e-7 <= res.hist[-2]
    assert np.abs(res.x - 1.0).max() < 1e-4


def test_pcg_zero_rhs(orc):
    A = inputs.grid2d_5pt(8)
    s = orc.system(A, 4, 8)
    res = s.solve(np.zeros(A.n), x0=np.ones(A.n))
    assert res.status == orc.OK and res.iters == 0 and not res.x.any()


def test_pcg_dummy_entries_stay_zero(orc):
    A = inputs.random_spd(101, 0.05, 21)      # ragged: padding needed
    s = orc.system(A, 4, 8)
    assert s.ordr.n_pad > A.n
    bb = s.to_hbmc(inputs.uniform_rhs(A.n, 2))
    res = orc.pcg(s.Ab, s.d, s.fac, bb, tol=1e-10)
    dummy = np.setdiff1d(np.arange(s.ordr.n_pad), s.ordr.perm)
    assert np.all(res.x[dummy] == 0.0)


@pytest.mark.parametrize("name,make,bs,w", [
    ("grid3d_24", lambda: inputs.diffusion3d(24, 1.0, 2), 8, 64),
    ("knn_3000", lambda: inputs.knn_laplacian(3000, 13, 4, 5), 8, 16),
    ("random", lambda: inputs.random_spd(500, 0.01, 8), 4, 8),
], ids=lambda v: v if isinstance(v, str) else "")
def test_bmc_hbmc_same_iterations(orc, name, make, bs, w):
    """HBMC is equivalent to BMC (Section 4.2.1): equal iteration counts up
    to rounding (Table "number-ite" shows 0 or 1 apart) and overlapping
    residual histories (Fig. "conv-behavior")."""
    A = make()
    b = inputs.uniform_rhs(A.n, 3)
    rb = orc.system(A, bs, 1).solve(b, tol=1e-7)
    rh = orc.system(A, bs, w).solve(b, tol=1e-7)
    assert rb.status == rh.status == orc.OK
    assert abs(rb.iters - rh.iters) <= 1
    k = min(rb.iters, rh.iters) + 1
    assert np.allclose(np.log10(rb.hist[:k]), np.log10(rh.hist[:k]), atol=1e-6)


def test_fp32_preconditioner_converges(orc):
    A = inputs.diffusion3d(16, 1.0, 2)
    s = orc.system(A, 8, 64)
    b = inputs.uniform_rhs(A.n, 3)
    r64 = s.solve(b, tol=1e-7)
    r32 = s.solve(b, tol=1e-7, precision="f32")
    assert r32.status == orc.OK
    assert abs(r32.iters - r64.iters) <= 2
    true = np.linalg.norm(b - A.to_scipy() @ r32.x) / np.linalg.norm(b)
    assert true < 2e-7


# ---------------------------------------------------------------------------
# The FP32 preconditioner of the oracle (orc_apply_f32): the factor rounded
# to binary32 and every operation of both substitutions carried out in
# binary32.  Three pins that an FP64 substitution (or one that rounds only
# its result) fails.
# ---------------------------------------------------------------------------
def test_apply_f32_worked_example(orc):
    """A = [[2, -1], [-1, 2]] (bs = w = 1 keeps the numbering), r = [-1, 1].
    IC(0) is exact here: d = (2, 3/2), L_10 = -1.  In binary32, with
    1/d rounded to binary32 (fl(2/3) = 11184811 * 2^-24):
      y0 = -1 * 0.5                               = -0.5
      y1 = (1 - (-1)(-0.5)) * fl(2/3) = 0.5 * 11184811 * 2^-24
                                                  = 11184811 * 2^-25 (exact)
      z1 = y1
      z0 = y0 - 0.5 * (-1 * z1) = -0.5 + 11184811 * 2^-26
         = -22369621 * 2^-26, a tie between two binary32 neighbours,
           rounded to the even one               = -11184810 * 2^-25.
    The exact result is (-1/3, 1/3); rounding -1/3 once gives
    -11184811 * 2^-25, so only per-operation binary32 arithmetic gives z0."""
    A = inputs.path_1d(2)
    s = orc.system(A, 1, 1)
    assert np.array_equal(s.ordr.perm, [0, 1])
    z = orc.apply(s.Ab, s.d, s.fac, np.array([-1.0, 1.0]), precision="f32")
    assert z[0] == -11184810 * 2.0 ** -25
    assert z[1] == 11184811 * 2.0 ** -25
    z64 = orc.apply(s.Ab, s.d, s.fac, np.array([-1.0, 1.0]))
    assert np.allclose(z64, [-1.0 / 3.0, 1.0 / 3.0], rtol=1e-15, atol=0)


@pytest.mark.parametrize("name,make,bs,w", CASES, ids=[c[0] for c in CASES])
def test_apply_f32_outputs_are_binary32(orc, name, make, bs, w):
    """Every entry of the FP32 preconditioned vector is a binary32 number, it
    is not the FP64 result, and it lies within a binary32 rounding bound of
    the FP64 result: per unknown, the substitutions' error is at most about
    (chain length + couplings) binary32 roundings of the magnitudes involved
    (|r| + sum |L| |y| through the chain), bounded here by 1e-4 relative."""
    s = orc.system(make(), bs, w)
    r = np.random.default_rng(4).standard_normal(s.Ab.n)
    z32 = orc.apply(s.Ab, s.d, s.fac, r, precision="f32")
    z64 = orc.apply(s.Ab, s.d, s.fac, r)
    assert np.array_equal(z32.astype(np.float32).astype(np.float64), z32)
    assert not np.array_equal(z32, z64)
    assert np.abs(z32 - z64).max() <= 1e-4 * np.abs(z64).max()
    assert np.abs(z32 - z64).max() >= 1e-9 * np.abs(z64).max()


def _round_binary(x, bits):
    """x (a Fraction) rounded to the nearest number with a `bits`-bit
    significand, ties to even (IEEE 754 round-to-nearest-even; normal range
    only)."""
    from fractions import Fraction
    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    m = abs(x)
    e = m.numerator.bit_length() - m.denominator.bit_length()
    if Fraction(2) ** e > m:
        e -= 1                                     # now 2^e <= m < 2^(e+1)
    assert e >= -126, "subnormal range not emulated"
    q = m * Fraction(2) ** (bits - 1 - e)          # in [2^(bits-1), 2^bits)
    fl = q.numerator // q.denominator
    rem = q - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * fl * Fraction(2) ** (e - (bits - 1))


def test_apply_f32_matches_exact_binary32_emulation(orc):
    """The FP32 substitutions against exact rational arithmetic with an
    explicit binary32 round-to-nearest-even after every operation (and
    binary64 rounding where the oracle's header says the value is formed in
    FP64: 1/d before its conversion to binary32).  Forward, i ascending:
    s = r_i; s = s - L_ij y_j over the row's lower entries in column order;
    y_i = s * (1/d_i).  Backward, i descending: s = sum of L_ji z_j over
    j > i in column order; z_i = y_i - (1/d_i) s.  Bit-identical results."""
    from fractions import Fraction
    A = inputs.random_spd(36, 0.12, 21)
    s = orc.system(A, 3, 4)
    Ab = s.Ab
    r = np.random.default_rng(8).uniform(-1, 1, Ab.n)
    z = orc.apply(Ab, s.d, s.fac, r, precision="f32")

    def f32(x):
        return _round_binary(x, 24)

    def f64(x):
        return _round_binary(x, 53)

    n = Ab.n
    dinv = [f32(f64(1 / Fraction(float(s.d[i])))) for i in range(n)]
    pos = {(i, int(Ab.col[p])): p for i in range(n) for p in range(Ab.rowptr[i], Ab.rowptr[i + 1])}
    y = [Fraction(0)] * n
    for i in range(n):
        acc = f32(Fraction(float(r[i])))
        for p in range(Ab.rowptr[i], Ab.rowptr[i + 1]):
            j = int(Ab.col[p])
            if j < i:
                acc = f32(acc - f32(f32(Fraction(float(s.fac[p]))) * y[j]))
        y[i] = f32(acc * dinv[i])
    zz = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        acc = Fraction(0)
        for p in range(Ab.rowptr[i], Ab.rowptr[i + 1]):
            j = int(Ab.col[p])
            if j > i:
                acc = f32(acc + f32(f32(Fraction(float(s.fac[pos[(j, i)]]))) * zz[j]))
        zz[i] = f32(y[i] - f32(dinv[i] * acc))
    assert [float(v) for v in zz] == list(z)


def test_scaled_start_pins(orc):
    """The warm start's scaled start c x0, c = (b, x0) / (x0, A x0): the exact
    solution keeps c = 1; c is the minimum of the A-norm error over multiples
    of x0 (checked against the error's values, computed with scipy, at
    neighbouring multiples and against the closed-form minimum over a fine
    grid); the error is never above that of the zero start; a guess pointing
    away from the solution falls back to 0; c scales inversely with x0."""
    A = inputs.diffusion3d(12, 1.0, 2)
    S = A.to_scipy()
    b = inputs.uniform_rhs(A.n, 3)
    xs = spla.spsolve(S.tocsc(), b)
    c, y = orc.scaled_start(A, b, xs)
    assert abs(c - 1.0) < 1e-12 and np.allclose(y, xs, rtol=1e-12, atol=0)
    rng = np.random.default_rng(1)
    x0 = 0.7 * xs + 0.2 * rng.standard_normal(A.n) * np.abs(xs).max()

    def err(t):
        e = t * x0 - xs
        return float(e @ (S @ e))

    c, y = orc.scaled_start(A, b, x0)
    assert np.array_equal(y, c * x0)
    grid = np.linspace(0.0, 2.0, 20001)
    best = grid[np.argmin([err(t) for t in grid])]
    assert abs(best - c) <= 1e-4
    for d in (1e-3, -1e-3, 0.1, -0.1):
        assert err(c) <= err(c + d)
    assert err(c) <= err(0.0)
    c0, y0 = orc.scaled_start(A, b, -xs)
    assert c0 == 0.0 and not np.any(y0)
    c3, y3 = orc.scaled_start(A, b, 3.0 * x0)
    assert abs(c3 * 3.0 - c) <= 1e-14 * c and np.allclose(y3, y, rtol=1e-14, atol=0)

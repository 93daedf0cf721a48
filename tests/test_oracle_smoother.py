"""Pins of the oracle's SOR / Gauss-Seidel sweeps and SSOR splitting.

- a forward SOR sweep equals the matrix-splitting form
  x1 = (D + omega L)^-1 (omega b - (omega U + (omega - 1) D) x0), solved
  with scipy's dense triangular solver; a backward sweep the mirrored form;
- the solution of A x = b (numpy.linalg.solve) is a fixed point of every
  sweep;
- on a diagonal matrix one forward sweep gives (1 - omega) x0 + omega b / a;
- a symmetric Gauss-Seidel / SSOR step never increases the energy norm of
  the error (Ostrowski-Reich: 0 < omega < 2, A SPD) and drives it to zero;
- one SSOR step (forward then backward sweep) equals the correction form
  x + (2 - omega) ((D/omega + L) (D/omega)^-1 (D/omega + L^T))^-1 (b - A x),
  built from sparse products and a dense inverse (no substitution);
- Section 3: under an equivalent reordering (HBMC against BMC, w = 1) the
  Gauss-Seidel iterates are the same numbers, permuted.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import core as orc
from paper_1908_00741_amd import inputs


def _dense(A):
    return sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n)).toarray()


CASES = [
    ("random_60", lambda: inputs.random_spd(60, 0.08, 3)),
    ("grid_7x5", lambda: inputs.grid2d_5pt(7, 5)),
    ("knn_80", lambda: inputs.knn_laplacian(80, 6, 4, 5, shift=1e-2)),
]


@pytest.mark.parametrize("omega", [0.7, 1.0, 1.6])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_sweeps_match_splitting(name, make, omega):
    A = make()
    M = _dense(A)
    D, L, U = np.diag(np.diag(M)), np.tril(M, -1), np.triu(M, 1)
    rng = np.random.default_rng(1)
    b, x0 = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    fwd = orc.sor_sweeps(A, b, x0, omega, 1, symmetric=False)
    ref = sla.solve_triangular(D + omega * L, omega * b - (omega * U + (omega - 1) * D) @ x0, lower=True)
    assert np.linalg.norm(fwd - ref) <= 1e-13 * np.linalg.norm(ref)
    sym = orc.sor_sweeps(A, b, x0, omega, 1, symmetric=True)
    ref2 = sla.solve_triangular(D + omega * U, omega * b - (omega * L + (omega - 1) * D) @ ref, lower=False)
    assert np.linalg.norm(sym - ref2) <= 1e-13 * np.linalg.norm(ref2)


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_solution_is_fixed_point(name, make):
    A = make()
    b = np.random.default_rng(2).uniform(-1, 1, A.n)
    xs = np.linalg.solve(_dense(A), b)
    for omega in (0.5, 1.0, 1.9):
        for sym in (False, True):
            x = orc.sor_sweeps(A, b, xs, omega, 2, symmetric=sym)
            assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)


def test_diagonal_matrix_closed_form():
    n = 9
    a = np.linspace(1.0, 5.0, n)
    A = inputs._from_coo(n, np.arange(n), np.arange(n), a)
    b = np.linspace(-2.0, 3.0, n)
    x0 = np.linspace(0.5, -0.5, n)
    for omega in (0.3, 1.0, 1.7):
        x = orc.sor_sweeps(A, b, x0, omega, 1, symmetric=False)
        assert np.allclose(x, (1 - omega) * x0 + omega * b / a, rtol=0, atol=1e-15)


@pytest.mark.parametrize("omega", [1.0, 1.5])
def test_ssor_energy_decreases(omega):
    A = inputs.grid2d_5pt(12, 10)
    M = _dense(A)
    b = np.random.default_rng(3).uniform(-1, 1, A.n)
    xs = np.linalg.solve(M, b)

    def energy(x):
        e = x - xs
        return float(e @ M @ e)

    x = np.zeros(A.n)
    last = energy(x)
    for _ in range(40):
        x = orc.sor_sweeps(A, b, x, omega, 1, symmetric=True)
        now = energy(x)
        assert now < last
        last = now
    assert last < 1e-3 * energy(np.zeros(A.n))


@pytest.mark.parametrize("omega", [0.8, 1.0, 1.4])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_ssor_step_is_correction_form(name, make, omega):
    A = make()
    M = _dense(A)
    rng = np.random.default_rng(4)
    b, x0 = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    Dp = np.diag(np.diag(M) / omega)
    L = np.tril(M, -1)
    Mp = (Dp + L) @ np.linalg.inv(Dp) @ (Dp + L.T)
    ref = x0 + (2 - omega) * np.linalg.solve(Mp, b - M @ x0)
    x = orc.sor_sweeps(A, b, x0, omega, 1, symmetric=True)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
    # the split fed to the preconditioner routine gives the same step
    d, fac = orc.ssor_split(A, omega)
    z = orc.apply(A, d, fac, b - M @ x0)
    assert np.linalg.norm(x0 + (2 - omega) * z - ref) <= 1e-12 * np.linalg.norm(ref)


def test_ssor_split_rejects_bad_omega():
    A = inputs.grid2d_5pt(4)
    for omega in (0.0, 2.0, -1.0):
        with pytest.raises(orc.OracleError):
            orc.ssor_split(A, omega)


@pytest.mark.parametrize("sym", [False, True])
@pytest.mark.parametrize("name,make,bs,w", [
    ("grid_24x20_bs4_w8", lambda: inputs.grid2d_5pt(24, 20), 4, 8),
    ("diff3d_8_bs8_w4", lambda: inputs.diffusion3d(8, 1.0, 2), 8, 4),
    ("knn_500_bs4_w16", lambda: inputs.knn_laplacian(500, 8, 4, 5, shift=1e-2), 4, 16),
])
def test_hbmc_bmc_gs_iterates_equivalent(name, make, bs, w, sym):
    A = make()
    rng = np.random.default_rng(5)
    b, x0 = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    out = []
    for ww in (1, w):
        o = orc.order(A, bs, ww)
        Ab = orc.permute(A, o.perm, o.n_pad)
        bb = np.zeros(o.n_pad); bb[o.perm] = b
        xb = np.zeros(o.n_pad); xb[o.perm] = x0
        x = orc.sor_sweeps(Ab, bb, xb, 1.2, 3, symmetric=sym)
        dummy = np.setdiff1d(np.arange(o.n_pad), o.perm)
        assert np.all(x[dummy] == 0.0)
        out.append(x[o.perm])
    assert np.linalg.norm(out[0] - out[1]) <= 1e-14 * np.linalg.norm(out[0])

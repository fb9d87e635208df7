"""Pins of the oracle's Kronecker-product solver (CPU only).

Independent anchors:
* dense brute force: the assembled 3D Laplacian and a direct LU solve of the
  discrete Poisson equation (and of the screened equation through a dense
  matrix exponential), Eqs. (Poisson), (Poisson:SR);
* the continuum closed form of a Gaussian charge under the erfc kernel,
  which fixes the screened kernel and its zero mode (readings R1, R2);
* plane waves on the grid: eigenfunctions of the FD Laplacian with the
  circulant symbol as eigenvalue;
* the slice-wise form of Sec. II.A against the literal batch form of
  Sec. II.B, and the matrix-product counts the paper states.
"""

import json
import os

import numpy as np
import pytest
from scipy.special import erf

from oracle.dense import (assemble_laplacian, has_zero_mode, solve_poisson_dense,
                          solve_screened_dense)
from oracle.fd import fd_weights
from oracle.kron import KronSolver

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

TINY = [
    # (n, h, bc, omega, kappa)
    ((6, 7, 8), (0.3, 0.35, 0.4), ("periodic",) * 3, 0.0, (0, 0, 0)),
    ((6, 7, 8), (0.3, 0.35, 0.4), ("periodic",) * 3, 0.5, (0, 0, 0)),
    ((7, 6, 9), (0.3, 0.3, 0.3), ("periodic", "periodic", "dirichlet"), 0.0, (0, 0, 0)),
    ((7, 6, 9), (0.3, 0.3, 0.3), ("periodic", "periodic", "dirichlet"), 0.7, (0, 0, 0)),
    ((5, 8, 6), (0.25, 0.3, 0.35), ("dirichlet",) * 3, 0.0, (0, 0, 0)),
    ((6, 6, 7), (0.3, 0.3, 0.3), ("periodic",) * 3, 0.0, (0.6, -0.3, 0.9)),
    ((6, 6, 7), (0.3, 0.3, 0.3), ("periodic", "periodic", "dirichlet"), 0.4, (0.5, 0.8, 0.0)),
    ((13, 13, 14), (0.3, 0.3, 0.3), ("periodic",) * 3, 0.106, (0, 0, 0)),
]


def _rhs(N, cplx, seed):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal(N)
    if cplx:
        b = b + 1j * rng.standard_normal(N)
    return b


@pytest.mark.parametrize("case", range(len(TINY)))
def test_kron_matches_dense(case):
    n, h, bc, omega, kappa = TINY[case]
    S = KronSolver(n, h, bc, 12, omega, kappa)
    L = assemble_laplacian(n, h, bc, 12, kappa)
    zm = has_zero_mode(bc, kappa)
    for seed in range(2):
        b = _rhs(S.N, S.complex, seed + 10 * case)
        x = S.solve(b)
        if omega > 0:
            ref = solve_screened_dense(L, b, omega, zm)
        else:
            ref = solve_poisson_dense(L, b, zm)
        err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
        assert err < 1e-12, (case, err)


@pytest.mark.parametrize("case", [0, 1, 3, 5, 6])
def test_batch_form_equals_slicewise(case):
    n, h, bc, omega, kappa = TINY[case]
    S = KronSolver(n, h, bc, 12, omega, kappa)
    C = np.stack([_rhs(S.N, S.complex, s) for s in range(5)])
    Y = S.solve_batch(C)
    X = S.solve(C)
    assert np.linalg.norm(Y - X) / np.linalg.norm(X) < 1e-13


def test_gaussian_charge_screened_closed_form():
    # A normalized Gaussian charge under erfc(omega r)/r has the potential
    # [erf(sqrt(alpha) r) - erf(mu r)]/r, mu = (1/alpha + 1/omega^2)^-1/2.
    # In a periodic box much wider than 1/omega the images vanish, and the
    # G = 0 term of the periodic sum is the zero mode pi/omega^2 * mean(rho).
    Lbox, alpha, omega = 12.0, 1.0, 0.8
    errs = []
    for n in (30, 40):
        h = Lbox / n
        S = KronSolver((n, n, n), (h, h, h), ("periodic",) * 3, 12, omega)
        x = np.arange(n) * h - Lbox / 2
        X3, X2, X1 = np.meshgrid(x, x, x, indexing="ij")
        r = np.sqrt(X1 ** 2 + X2 ** 2 + X3 ** 2)
        rho = (alpha / np.pi) ** 1.5 * np.exp(-alpha * r ** 2)
        phi = S.solve(rho.reshape(-1)).reshape(n, n, n)
        mu = (1 / alpha + 1 / omega ** 2) ** -0.5
        rs = np.where(r > 0, r, 1.0)
        exact = np.where(r > 0, (erf(np.sqrt(alpha) * r) - erf(mu * r)) / rs,
                         2 / np.sqrt(np.pi) * (np.sqrt(alpha) - mu))
        errs.append(np.max(np.abs(phi - exact)) / np.max(np.abs(exact)))
    assert errs[1] < 3e-6, errs
    # high-order convergence in h
    assert np.log(errs[0] / errs[1]) / np.log(40 / 30) > 9.0, errs


def _symbol(n, h, p_idx, kappa=0.0):
    c = [float(x) for x in fd_weights(12)]
    theta = 2 * np.pi * p_idx / (n * h) + kappa
    return (c[0] + 2 * sum(c[s] * np.cos(s * theta * h) for s in range(1, 7))) / h ** 2


@pytest.mark.parametrize("omega", [0.0, 0.106, 0.9])
def test_plane_wave_symbol(omega):
    # B = e^{i theta.r} with theta on the reciprocal grid is an eigenfunction of
    # the FD Laplacian with eigenvalue sum_d symbol_d; the solution is the
    # kernel of Eq. (fL) at that eigenvalue times B.
    n, h = (10, 12, 9), (0.3, 0.25, 0.35)
    kappa = (0.4, 0.0, -0.7)
    S = KronSolver(n, h, ("periodic",) * 3, 12, omega, kappa)
    for p in [(1, 0, 0), (2, 5, 3), (4, 11, 8)]:
        ph = [np.exp(1j * (2 * np.pi * p[d] / (n[d] * h[d]) + kappa[d]) * np.arange(n[d]) * h[d])
              for d in range(3)]
        B = (ph[2][:, None, None] * ph[1][None, :, None] * ph[0][None, None, :]).reshape(-1)
        lam = sum(_symbol(n[d], h[d], p[d], kappa[d]) for d in range(3))
        assert lam < 0
        if omega > 0:
            f = -(4 * np.pi / lam) * (1 - np.exp(lam / (4 * omega ** 2)))
        else:
            f = -4 * np.pi / lam
        X = S.solve(B)
        assert np.allclose(X, f * B, rtol=1e-11, atol=1e-11 * abs(f))


def test_zero_mode_conventions():
    n, h = (8, 9, 10), (0.3, 0.3, 0.3)
    rng = np.random.default_rng(0)
    b = rng.standard_normal(720)
    Sc = KronSolver(n, h, ("periodic",) * 3, 12, 0.0)
    x = Sc.solve(b)
    assert abs(x.mean()) < 1e-13 * np.abs(x).max()
    assert np.allclose(Sc.solve(b + 3.0), x, atol=1e-12 * np.abs(x).max())
    omega = 0.3
    Ss = KronSolver(n, h, ("periodic",) * 3, 12, omega)
    assert np.allclose(Ss.solve(np.full(720, 2.0)), 2.0 * np.pi / omega ** 2, rtol=1e-12)


def test_real_gamma_solution_is_real_and_linear():
    n, h = (9, 8, 7), (0.3, 0.3, 0.3)
    S = KronSolver(n, h, ("periodic", "periodic", "dirichlet"), 12, 0.106)
    assert not S.complex
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal((2, S.N))
    assert np.allclose(S.solve(2 * a - b), 2 * S.solve(a) - S.solve(b), atol=1e-12)
    # f(L) is symmetric positive semidefinite: <a, f(L) b> = <b, f(L) a>, <a, f(L) a> >= 0
    assert abs(a @ S.solve(b) - b @ S.solve(a)) < 1e-10 * abs(a @ S.solve(b))
    assert a @ S.solve(a) > 0


def test_matrix_product_counts_stated_in_paper():
    with open(os.path.join(GOLDEN, "paper_counts.json")) as fh:
        gold = json.load(fh)
    for n3 in gold["slicewise_gemms_per_system"]["n3"]:
        S = KronSolver((4, 4, n3), (0.3,) * 3, ("periodic",) * 3, 2, 0.0)
        assert S.gemm_count_slicewise() == 4 * n3 + 2
    for nc, val in zip(gold["batch_gemms_per_system"]["n_c"],
                       gold["batch_gemms_per_system"]["value"]):
        assert KronSolver.gemm_count_batch(nc) == pytest.approx(val)


def _symbol_longdouble(n, h, order, kappa):
    """Spectrum of the periodic / Bloch FD operator from the circulant
    closed form, -4/h^2 sum_s c_s sin^2(s theta_q / 2) with
    theta_q = 2 pi q / n + kappa h, in extended precision (the exact rational
    weights rounded once to long double)."""
    ld = np.longdouble
    c = fd_weights(order)
    th = ld(2) * ld(np.pi) * np.arange(n, dtype=ld) / ld(n) + ld(kappa) * ld(h)
    acc = np.zeros(n, dtype=ld)
    for s in range(1, len(c)):
        cs = ld(c[s].numerator) / ld(c[s].denominator)
        acc += cs * np.sin(ld(s) * th / ld(2)) ** 2
    return np.sort((ld(-4) * acc / (ld(h) * ld(h))).astype(np.float64))


@pytest.mark.parametrize("n,h,kappa", [(80, 0.25, np.pi / 20.0), (80, 0.25, 0.3), (80, 0.25, 0.0),
                                       (120, 0.2, 0.0), (7, 0.3, 0.6), (160, 0.3125, 0.01)])
def test_periodic_eigenvalues_relative_accuracy(n, h, kappa):
    # Every eigenvalue of the periodic / Bloch axis, the smallest included,
    # well inside the FP64 parity bar (1e-12) in relative terms, against the
    # closed form in extended precision: the unscreened kernel -4 pi / lambda
    # carries the relative error of the smallest |lambda| straight into the
    # dominant modes of the solution.  (A Hermitian eigensolver's own
    # eigenvalues miss this by up to 3e-11 on these axes; the Rayleigh
    # quotient's error grows only like eps / theta for the mode at angle theta.)
    S = KronSolver((n, 4, 4), (h, 0.3, 0.3), ("periodic",) * 3, 12, 0.0, kappa=(kappa, 0.0, 0.0))
    lam = np.sort(S.lam[0])
    ref = _symbol_longdouble(n, h, 12, kappa)
    scale = np.maximum(np.abs(ref), 1e-300)
    nonzero = np.abs(ref) > 1e-12 * np.abs(ref).max()
    assert np.max(np.abs(lam - ref)[nonzero] / scale[nonzero]) < 2e-13
    assert np.max(np.abs(lam - ref)) < 1e-14 * np.abs(ref).max()

"""Pins of the oracle's FD weights and 1D operators (CPU only).

Every check here is fixed by mathematics independent of the oracle's code:
Taylor moment identities, textbook low-order stencils, the eigenvalues of
circulant matrices (DFT of the first row), and the DST-I closed form of the
second-order Dirichlet operator.
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle.fd import fd_weights, second_derivative_1d


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12])
def test_weights_taylor_moments(order):
    # The stencil is exact for x^k, k <= order+1:
    # sum_{s=-p..p} c_|s| s^k = k! * [k == 2] for every k <= order + 1.
    c = fd_weights(order)
    p = order // 2
    for k in range(0, order + 2):
        m = sum(c[abs(s)] * Fraction(s) ** k for s in range(-p, p + 1))
        expect = Fraction(2) if k == 2 else Fraction(0)
        assert m == expect, (order, k, m)
    # and not exact one order beyond (the truncation error term is nonzero)
    m = sum(c[abs(s)] * Fraction(s) ** (order + 2) for s in range(-p, p + 1))
    assert m != 0


def test_weights_low_order_textbook():
    assert fd_weights(2) == [-2, 1]
    assert fd_weights(4) == [Fraction(-5, 2), Fraction(4, 3), Fraction(-1, 12)]
    assert fd_weights(6) == [Fraction(-49, 18), Fraction(3, 2), Fraction(-3, 20),
                             Fraction(1, 90)]


def test_convergence_order_12():
    # second derivative of sin on a periodic grid: error falls like h^12
    errs = []
    for n in (24, 32):
        h = 2 * np.pi / n
        x = np.arange(n) * h
        D = second_derivative_1d(n, h, "periodic", 12)
        errs.append(np.max(np.abs(D @ np.sin(3 * x) + 9 * np.sin(3 * x))))
    rate = np.log(errs[0] / errs[1]) / np.log(32 / 24)
    assert rate > 11.0, rate


@pytest.mark.parametrize("n,h", [(7, 0.3), (16, 0.25), (25, 0.2), (10, 0.5)])
def test_periodic_circulant_spectrum(n, h):
    # A real symmetric circulant: eigenvalues are the DFT of its first row.
    D = second_derivative_1d(n, h, "periodic", 12)
    assert np.allclose(D, D.T, atol=0)
    assert np.allclose(D.sum(axis=1), 0.0, atol=1e-10 / h ** 2)
    dft = np.fft.fft(D[0]).real
    lam = np.linalg.eigvalsh(D)
    assert np.allclose(np.sort(dft), lam, rtol=0, atol=1e-11 * np.max(np.abs(lam)))
    assert lam.max() <= 1e-10 * np.max(np.abs(lam))  # negative semidefinite


@pytest.mark.parametrize("n,h,kappa", [(9, 0.3, 0.4), (16, 0.25, -1.1), (5, 0.2, 2.0)])
def test_bloch_operator(n, h, kappa):
    # Hermitian, and e^{i kappa x} times any n-periodic Fourier mode is an
    # eigenvector (checked directly, not through the oracle's eigensolver).
    D = second_derivative_1d(n, h, "periodic", 12, kappa)
    assert np.allclose(D, D.conj().T, atol=1e-12 / h ** 2)
    x = np.arange(n) * h
    for p in range(n):
        u = np.exp(1j * (2 * np.pi * p / (n * h) + kappa) * x)
        Du = D @ u
        ratio = Du / u
        assert np.allclose(ratio, ratio[0], atol=1e-9 / h ** 2)
        assert abs(ratio[0].imag) < 1e-9 / h ** 2
        assert ratio[0].real < 0


@pytest.mark.parametrize("n,h", [(5, 0.3), (12, 0.25), (31, 0.1)])
def test_dirichlet_order2_is_dst1(n, h):
    D = second_derivative_1d(n, h, "dirichlet", 2)
    k = np.arange(1, n + 1)
    lam_exact = -(4.0 / h ** 2) * np.sin(k * np.pi / (2 * (n + 1))) ** 2
    lam = np.linalg.eigvalsh(D)
    assert np.allclose(np.sort(lam_exact), lam, rtol=1e-13, atol=1e-12 / h ** 2)
    j = np.arange(1, n + 1)
    for kk in (1, n // 2 + 1, n):
        v = np.sin(np.pi * kk * j / (n + 1))
        assert np.allclose(D @ v, lam_exact[kk - 1] * v, atol=1e-10 / h ** 2)


def test_dirichlet_order12_negative_definite():
    D = second_derivative_1d(40, 0.3, "dirichlet", 12)
    lam = np.linalg.eigvalsh(D)
    assert lam.max() < 0
    # truncated stencil: a row far from the walls carries the full stencil
    c = [float(x) for x in fd_weights(12)]
    assert np.allclose(D[20, 14:27] * 0.09, c[::-1] + c[1:], atol=1e-14)
    assert D[0, 7] == 0.0 and D[0, 6] != 0.0


def test_small_periodic_wraps_accumulate():
    # n < 2p+1: several stencil taps land on the same column; the circulant
    # spectrum still equals the FD symbol at the grid wavenumbers.
    n, h = 5, 0.4
    D = second_derivative_1d(n, h, "periodic", 12)
    c = [float(x) for x in fd_weights(12)]
    for p in range(n):
        theta = 2 * np.pi * p / n
        symbol = (c[0] + 2 * sum(c[s] * np.cos(s * theta) for s in range(1, 7))) / h ** 2
        v = np.exp(1j * theta * np.arange(n))
        assert np.allclose(D @ v, symbol * v, atol=1e-10 / h ** 2)

"""Brute-force dense solve of the discrete (screened) Poisson equation (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

This is the plain definition that the Kronecker forms must reproduce: the 3D
Laplacian assembled as a dense N x N matrix from the 1D second-derivative
operators and Eqs. (Poisson) / (Poisson:SR) solved directly, with no
eigendecomposition of the 1D operators.  Only for tiny grids (N of a few
thousand).
"""

import numpy as np
import scipy.linalg

from .fd import second_derivative_1d


def assemble_laplacian(n, h, bc, order=12, kappa=(0.0, 0.0, 0.0)):
    """Dense L = I3 (x) I2 (x) D1 + I3 (x) D2 (x) I1 + D3 (x) I2 (x) I1.

    The right-most Kronecker factor runs fastest, matching the flat index
    i1 + n1*(i2 + n2*i3).
    """
    D = [second_derivative_1d(n[d], h[d], bc[d], order, kappa[d]) for d in range(3)]
    I = [np.eye(n[d]) for d in range(3)]
    L = (np.kron(I[2], np.kron(I[1], D[0]))
         + np.kron(I[2], np.kron(D[1], I[0]))
         + np.kron(D[2], np.kron(I[1], I[0])))
    return L


def has_zero_mode(bc, kappa):
    """L is singular exactly when every axis is periodic with kappa = 0."""
    return all(b == "periodic" for b in bc) and all(k == 0.0 for k in kappa)


def solve_poisson_dense(L, b, zero_mode):
    """Unscreened Eq. (Poisson): -(1/4 pi) L x = b, by LU.

    If L is singular (periodic at k = q) its null space is the constants; the
    solution is taken with zero mean and the right-hand side's mean is
    ignored (reading R2): the rank-one term -11^T/N makes the matrix regular
    without changing any zero-mean solution.
    """
    rhs = -4.0 * np.pi * np.asarray(b)
    A = L
    if zero_mode:
        N = L.shape[0]
        rhs = rhs - rhs.mean()
        A = L - np.ones((N, N)) / N
    return np.linalg.solve(A, rhs)


def solve_screened_dense(L, b, omega, zero_mode):
    """Screened Eq. (Poisson:SR) under reading R1:
    -(1/4 pi) (I - e^{L/(4 omega^2)})^{-1} L x = b, i.e.
    L x = -4 pi (I - expm(L/(4 omega^2))) b, by a dense matrix exponential and
    LU.  With a zero mode the constant component of x is the lambda -> 0 limit
    (pi/omega^2) * mean(b) (reading R2), and L is regularized as in the
    unscreened case for the rest.
    """
    b = np.asarray(b)
    E = scipy.linalg.expm(L / (4.0 * omega * omega))
    rhs = -4.0 * np.pi * (b - E @ b)
    A = L
    if zero_mode:
        N = L.shape[0]
        rhs = rhs - rhs.mean()
        A = L - np.ones((N, N)) / N
    x = np.linalg.solve(A, rhs)
    if zero_mode:
        x = x + (np.pi / (omega * omega)) * b.mean()
    return x

"""Finite-difference weights and 1D second-derivative operators (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. II / II.A of arXiv 2501.16572 discretize the Laplacian on a uniform grid
with n_d points along x_d; the Kronecker formalism needs, per direction, the
matrix of the discrete second derivative.  The paper does not print the
stencil; the order (12th) is a parameter here.  Boundary conditions follow
Sec. II: Bloch-periodic at wavevector k-q along extended directions, and
zero Dirichlet along vacuum directions.
"""

from fractions import Fraction
from math import factorial

import numpy as np

PERIODIC = "periodic"
DIRICHLET = "dirichlet"


def fd_weights(order):
    """Exact weights c_0..c_p of the central 2p-th order second derivative.

    f''(x) ~ (c_0 f(x) + sum_{s=1..p} c_s (f(x+sh) + f(x-sh))) / h^2 with
    p = order/2.  Closed form of the central-difference weights (Fornberg,
    Math. Comp. 51 (1988)):

        c_s = 2 (-1)^(s+1) (p!)^2 / (s^2 (p-s)! (p+s)!),  s = 1..p
        c_0 = -2 sum_{s=1..p} 1/s^2

    Returned as ``fractions.Fraction`` so the tests can check the Taylor
    moment identities exactly.
    """
    if order < 2 or order % 2:
        raise ValueError("order must be even and >= 2")
    p = order // 2
    c = [Fraction(0)] * (p + 1)
    for s in range(1, p + 1):
        c[s] = Fraction(2 * (-1) ** (s + 1) * factorial(p) ** 2,
                        s * s * factorial(p - s) * factorial(p + s))
    c[0] = -2 * sum(Fraction(1, s * s) for s in range(1, p + 1))
    return c


def second_derivative_1d(n, h, bc, order, kappa=0.0):
    """Dense n x n matrix of the 1D discrete second derivative along one axis.

    Row j applies the stencil c_|s| / h^2 to nodes j+s, s = -p..p.

    * ``periodic``: node j+s outside [0, n) is folded back by whole periods;
      each fold across the right (left) end multiplies by exp(+i kappa n h)
      (exp(-i kappa n h)), the Bloch condition psi(x + n h) = e^{i kappa n h}
      psi(x) at the wavevector kappa = (k - q)_d of Sec. II.  kappa = 0 gives
      the plain periodic (Gamma-point) operator, which is real.  Folds
      accumulate when n < 2p + 1.
    * ``dirichlet``: n interior nodes, zero ghost values beyond both ends (the
      wall sits one spacing beyond the end nodes); the stencil is truncated.
    """
    c = [float(x) for x in fd_weights(order)]
    p = order // 2
    cplx = (bc == PERIODIC and kappa != 0.0)
    D = np.zeros((n, n), dtype=np.complex128 if cplx else np.float64)
    for j in range(n):
        for s in range(-p, p + 1):
            w = c[abs(s)] / (h * h)
            t = j + s
            if bc == PERIODIC:
                wraps = t // n  # floor division: number of periods crossed
                col = t - wraps * n
                if cplx:
                    D[j, col] += w * np.exp(1j * kappa * n * h * wraps)
                else:
                    D[j, col] += w
            elif bc == DIRICHLET:
                if 0 <= t < n:
                    D[j, t] += w
            else:
                raise ValueError(f"unknown boundary condition {bc!r}")
    return D

"""Adaptively compressed exchange (ACE), plain FP64 / complex128 reference.

Test infrastructure only: imported by tests/ and bench.py's baseline, never by
the device path.

Sec. III.A (construction): with W = Vx Psi (the columns W^(n) of Eq. (W) for
the orbital set Psi), M = Psi^T W, R its Cholesky factor and xi = W R^{-1},
the compressed operator is xi xi^T.  Sec. III.B (application): V Phi is
formed in two products, chi = xi^T Phi, then xi chi.

Reading (R16): M = Psi^H W is Hermitian and negative definite (Vx is negative
semidefinite), so the factorization is of -M: -M = L L^H with L lower
triangular, xi = W L^{-H}, and the operator is -xi xi^H.  Inner products are
the grid's, <a, b> = dV sum conj(a) b, so M = dV Psi^H W and
V Phi = -xi (dV xi^H Phi).  With these conventions the compressed operator
reproduces W on span(Psi): V Psi = -W L^{-H} L^{-1} (dV W^H Psi)
= -W (-M)^{-1} M = W.

Arrays are row-major (n_cols, N): one orbital per row, as elsewhere.
"""

import numpy as np
import scipy.linalg


def ace_construct(psi, w, dV):
    """xi (n_s, N) from orbitals psi (n_s, N) and w = Vx psi (n_s, N)."""
    Psi = np.asarray(psi).T          # N x n_s
    W = np.asarray(w).T
    M = dV * (Psi.conj().T @ W)      # n_s x n_s, Hermitian negative definite
    M = 0.5 * (M + M.conj().T)
    L = np.linalg.cholesky(-M)       # lower, -M = L L^H
    # xi = W L^{-H}  <=>  xi^H = L^{-1} W^H
    xiH = scipy.linalg.solve_triangular(L, W.conj().T, lower=True)
    return np.ascontiguousarray(xiH.conj())  # rows = columns of xi


def ace_apply(xi, phi, dV):
    """V phi = -xi (dV xi^H phi) for trial orbitals phi (n_phi, N); returns (n_phi, N)."""
    Xi = np.asarray(xi).T            # N x n_s
    Phi = np.asarray(phi).T          # N x n_phi
    chi = dV * (Xi.conj().T @ Phi)   # n_s x n_phi
    return np.ascontiguousarray((-(Xi @ chi)).T)

"""Kronecker-product solution of the (screened) Poisson equation (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Grid functions are numpy arrays of shape (n3, n2, n1) in C order, so the flat
index is i1 + n1*(i2 + n2*i3): x1 runs fastest and B(:,:,k) is the k-th
frontal slice, as in Sec. II.A.  A set of n_c right-hand sides is an array of
shape (n_c, N) or (n_c, n3, n2, n1).

Readings of the paper (each also recorded in the design notes):

* R1 (screened kernel).  Eq. (fL) prints f(L) = -4 pi L^-1 (I - e^{-L/(16 pi
  omega^2)}), which grows without bound for L <= 0.  The erfc(omega r)/r
  interaction has the Fourier kernel 4 pi/G^2 (1 - e^{-G^2/(4 omega^2)});
  with -G^2 -> lambda this is f(lambda) = -(4 pi/lambda)(1 - e^{lambda/(4
  omega^2)}), which is what is implemented.  Tests pin it to the closed-form
  potential of a Gaussian charge.
* R2 (zero mode).  L is singular for periodic directions at k = q.  Unscreened:
  f(0) = 0 (the solution has zero mean).  Screened: f(0) = pi/omega^2, the
  exact lambda -> 0 limit.
* R15 (batch formula).  The parentheses of the batch solution in Sec. II.B are
  unbalanced; the reading is Y = [(((V1 Yt_[1])_[2] V2^T)_[3] V3^T)]_[4] with
  the forward transform using V1^{*T}, V2^*, V3^*, consistent with the
  slice-wise form of Sec. II.A.
"""

import numpy as np

from .fd import second_derivative_1d

# |lambda| below this fraction of max|lambda| is the zero mode (R2).
ZERO_MODE_RTOL = 1e-10


def eig_1d(D):
    """Eigenpairs of one 1D second-derivative operator: D = V diag(lam) V^H.

    Eq. (FinalRepfL): V_d are the eigenvectors of the discrete second
    derivative along x_d.  D is real symmetric (periodic at Gamma, Dirichlet)
    or Hermitian (Bloch), so a Hermitian eigensolver applies.
    """
    lam, V = np.linalg.eigh(D)
    return lam, V


def periodic_eigenvalues(V, h, order, kappa=0.0):
    """Eigenvalues of a periodic (kappa = 0) or Bloch-periodic 1D operator,
    given its unit eigenvectors (the columns of V), without cancellation.

    The weights satisfy c_0 = -2 sum_{s>=1} c_s (zeroth moment), so the
    operator of ``fd.second_derivative_1d`` is
        D = (1/h^2) sum_{s>=1} c_s (S_s + S_s^H - 2 I)
          = -(1/h^2) sum_{s>=1} c_s (S_s - I)^H (S_s - I),
    with S_s the shift by s nodes that picks up exp(i kappa n h) per period
    crossed (unitary).  The Rayleigh quotient of a unit eigenvector v is then
        lambda = -(1/h^2) sum_{s>=1} c_s ||S_s v - v||^2.
    A Hermitian eigensolver returns each eigenvalue with an absolute error of
    order eps ||D||; for the smallest |lambda| of a long periodic axis
    (|lambda| ~ (kappa or 2 pi / L)^2, ||D|| ~ 16 / h^2) that is a relative
    error of 1e-13 .. 1e-11, which the unscreened kernel f = -4 pi / lambda
    passes on one to one to the modes that dominate the solution.  The
    quotient above has no such cancellation; the eigenvectors themselves are
    exact to first order, so the quotient's error is second order in theirs.
    """
    from .fd import fd_weights
    c = [float(x) for x in fd_weights(order)]
    n = V.shape[0]
    j = np.arange(n)
    lam = np.zeros(V.shape[1])
    for s in range(1, len(c)):
        t = j + s
        wraps = t // n
        phase = np.exp(1j * kappa * n * h * wraps) if kappa != 0.0 else np.ones(n)
        SV = phase[:, None] * V[t - wraps * n, :]     # (S_s V)[j] = phase * V[(j + s) mod n]
        lam -= c[s] * np.sum(np.abs(SV - V) ** 2, axis=0)
    return lam / (h * h)


def kernel_f(lam, omega):
    """Scalar solution kernel f applied to eigenvalue sums, Eq. (fL).

    omega <= 0: unscreened, f(lam) = -4 pi / lam.
    omega > 0 : screened (reading R1), f(lam) = 4 pi expm1(lam/(4 omega^2))/lam.
    Zero mode per reading R2.  Returns float64 of lam's shape.
    """
    lam = np.asarray(lam, dtype=np.float64)
    scale = max(float(np.max(np.abs(lam))), 1e-300)
    zero = np.abs(lam) <= ZERO_MODE_RTOL * scale
    safe = np.where(zero, -1.0, lam)
    if omega <= 0:
        f = -4.0 * np.pi / safe
        return np.where(zero, 0.0, f)
    f = 4.0 * np.pi * np.expm1(safe / (4.0 * omega * omega)) / safe
    return np.where(zero, np.pi / (omega * omega), f)


class KronSolver:
    """X = f(L) B on an n1 x n2 x n3 grid (Sec. II.A, Eqs. (LS:Discrete:Solution),
    (fL), (FinalRepfL)).

    n, h, bc: per-axis size, spacing (bohr) and boundary condition
    ("periodic" or "dirichlet").  kappa: per-axis Bloch wavevector (k-q)_d in
    bohr^-1 (only on periodic axes).  order: FD order.  omega: screening
    parameter (<= 0 unscreened).
    """

    def __init__(self, n, h, bc, order=12, omega=0.0, kappa=(0.0, 0.0, 0.0)):
        self.n = tuple(int(x) for x in n)
        self.h = tuple(float(x) for x in h)
        self.bc = tuple(bc)
        self.order = int(order)
        self.omega = float(omega)
        self.kappa = tuple(float(x) for x in kappa)
        for d in range(3):
            if self.kappa[d] != 0.0 and self.bc[d] != "periodic":
                raise ValueError("a Bloch wavevector needs a periodic axis")
        self.D = [second_derivative_1d(self.n[d], self.h[d], self.bc[d],
                                       self.order, self.kappa[d])
                  for d in range(3)]
        eigs = [eig_1d(D) for D in self.D]
        self.V = [e[1] for e in eigs]
        # periodic / Bloch axes: eigenvalues from the eigenvectors by the
        # cancellation-free Rayleigh quotient (eigh's small eigenvalues are
        # only accurate to eps ||D|| absolute); Dirichlet axes keep eigh's
        self.lam = [periodic_eigenvalues(self.V[d], self.h[d], self.order, self.kappa[d])
                    if self.bc[d] == "periodic" else eigs[d][0] for d in range(3)]
        self.complex = any(np.iscomplexobj(V) for V in self.V)
        n1, n2, n3 = self.n
        # diag(Lambda) with the index order of the slice formulas:
        # entry a + n1*b + n1*n2*c holds lam1[a] + lam2[b] + lam3[c].
        lam_t = (self.lam[2][:, None, None] + self.lam[1][None, :, None]
                 + self.lam[0][None, None, :])
        self.lam_tilde = lam_t.reshape(-1)
        self.f_tilde = kernel_f(self.lam_tilde, self.omega)
        self.N = n1 * n2 * n3
        self.dV = self.h[0] * self.h[1] * self.h[2]

    # -- Sec. II.A: one system at a time, slice by slice -------------------
    def solve(self, B):
        """Slice-wise Kronecker solve, Eqs. (FinalSolution)/(LS:SolutionPart).

        Forward: for every frontal slice k, V1^{*T} B_k V2^*; the vectorized
        slices form the columns of an (n1 n2) x n3 matrix that is multiplied
        by V3^*; the result, vectorized, is scaled by f(Lambda~).  Inverse:
        V1 X~_k V2^T per slice, then V3^T.  B: (N,) or (n_c, N); each
        right-hand side is solved on its own.
        """
        B = np.asarray(B)
        single = B.ndim == 1
        Bs = B.reshape(1, -1) if single else B.reshape(B.shape[0], -1)
        out = np.empty(Bs.shape, dtype=np.result_type(Bs.dtype, self.V[0].dtype,
                                                      self.V[1].dtype, self.V[2].dtype))
        for r in range(Bs.shape[0]):
            out[r] = self._solve_one(Bs[r])
        return out[0] if single else out

    def _solve_one(self, b):
        n1, n2, n3 = self.n
        V1, V2, V3 = self.V
        grid = b.reshape(n3, n2, n1)
        # forward: columns vec(V1^{*T} B_k V2^*), k = 1..n3
        cols = np.empty((n1 * n2, n3), dtype=np.result_type(b.dtype, V1, V2, V3))
        for k in range(n3):
            Bk = grid[k].T                       # n1 x n2, entry [i1, i2]
            Sk = V1.conj().T @ Bk @ V2.conj()
            cols[:, k] = Sk.reshape(-1, order="F")   # vec: a + n1*b
        Xt = (cols @ V3.conj()).reshape(-1, order="F")  # vec_{n3}
        Xt = self.f_tilde * Xt
        # inverse: columns vec(V1 X~_k V2^T), then V3^T
        Xt3 = Xt.reshape(n1 * n2, n3, order="F")
        cols2 = np.empty_like(Xt3)
        for k in range(n3):
            Xk = Xt3[:, k].reshape(n1, n2, order="F")
            cols2[:, k] = (V1 @ Xk @ V2.T).reshape(-1, order="F")
        X = (cols2 @ V3.T).reshape(-1, order="F")
        return X

    # -- Sec. II.B: the batch formalism with its four reorganizations ------
    def solve_batch(self, C):
        """Batch Kronecker solve Y = f(L) C, C = [B^(1) ... B^(n_c)] (Sec. II.B).

        Follows the batch formula (reading R15) with the data reorganizations
        [1]-[4] written out literally, so that each mode product is a single
        matrix product over the whole batch.  C: (n_c, N).  Returns (n_c, N).
        """
        C = np.asarray(C)
        nc = C.shape[0]
        V1, V2, V3 = self.V
        Z = C.T                                  # N x n_c, one system per column
        Z = self._reorg1(Z)                      # n1 x (n2 n3 n_c)
        Z = V1.conj().T @ Z
        Z = self._reorg2(Z, nc)                  # (n1 n3 n_c) x n2
        Z = Z @ V2.conj()
        Z = self._reorg3(Z, nc)                  # (n1 n2 n_c) x n3
        Z = Z @ V3.conj()
        Z = self._reorg4(Z, nc)                  # N x n_c
        Yt = self.f_tilde[:, None] * Z           # f(Lambda~)_{n_c}: replicated
        Z = self._reorg1(Yt)
        Z = V1 @ Z
        Z = self._reorg2(Z, nc)
        Z = Z @ V2.T
        Z = self._reorg3(Z, nc)
        Z = Z @ V3.T
        Y = self._reorg4(Z, nc)
        return Y.T

    # Reorganization [1]: [Z^(1) .. Z^(nc)] -> [Zt^(1) .. Zt^(nc)] where
    # Zt^(j) = [Z^(j)(:,:,1) .. Z^(j)(:,:,n3)] places the n1 x n2 frontal
    # slices side by side.  Input here is either N x n_c (columns = systems)
    # or the output of [4]/[1]-compatible layouts (N x n_c).
    def _reorg1(self, Z):
        n1, n2, n3 = self.n
        nc = Z.shape[1]
        blocks = []
        for j in range(nc):
            g = Z[:, j].reshape(n1, n2, n3, order="F")   # g[i1,i2,i3]
            slices = [g[:, :, k] for k in range(n3)]
            blocks.append(np.hstack(slices))              # n1 x (n2 n3)
        return np.hstack(blocks)                          # n1 x (n2 n3 nc)

    # Reorganization [2]: Z_[1] -> Z_[2]: each Zt^(j) = [Zt_1 .. Zt_n3]
    # becomes the vertical stack [Zt_1; ..; Zt_n3] and the systems are
    # stacked vertically: (n1 n3 n_c) x n2.
    def _reorg2(self, Z, nc):
        n1, n2, n3 = self.n
        rows = []
        for j in range(nc):
            blk = Z[:, j * n2 * n3:(j + 1) * n2 * n3]
            rows.append(np.vstack([blk[:, k * n2:(k + 1) * n2] for k in range(n3)]))
        return np.vstack(rows)

    # Reorganization [3]: Z_[2] -> Z_[3]: for each system the stacked n1 x n2
    # slices are vectorized into the columns of an (n1 n2) x n3 matrix;
    # systems stay stacked vertically: (n1 n2 n_c) x n3.
    def _reorg3(self, Z, nc):
        n1, n2, n3 = self.n
        rows = []
        for j in range(nc):
            blk = Z[j * n1 * n3:(j + 1) * n1 * n3, :]
            cols = [blk[k * n1:(k + 1) * n1, :].reshape(-1, order="F")
                    for k in range(n3)]
            rows.append(np.column_stack(cols))
        return np.vstack(rows)

    # Reorganization [4]: Z_[3] -> Z_[4]: each system's (n1 n2) x n3 block is
    # vectorized along n3 back into one column of length N: N x n_c.
    def _reorg4(self, Z, nc):
        n1, n2, n3 = self.n
        out = [Z[j * n1 * n2:(j + 1) * n1 * n2, :].reshape(-1, order="F")
               for j in range(nc)]
        return np.column_stack(out)

    # The inverse-direction input to [1] is the scaled N x n_c array, which
    # has the same layout as the original right-hand sides, so [1] applies
    # unchanged.

    def gemm_count_slicewise(self):
        """Matrix products per system in the slice-wise form: 2 per slice and
        1 for x3, in each direction (Sec. II.A: 4 n3 + 2)."""
        return 2 * (2 * self.n[2] + 1)

    @staticmethod
    def gemm_count_batch(nc):
        """Matrix products per system in the batch form (Sec. II.B: 6/n_c)."""
        return 6.0 / nc

"""Pins of the oracle's exact-exchange application and E_x (CPU only).

Anchors: a brute-force Vx built from the dense Poisson solve (no Kronecker
machinery), the symmetry phi_mn = phi_nm at Gamma, Hermiticity and negative
semidefiniteness of <psi_a, Vx psi_b>, linearity in the occupations, the
conjugate symmetry of Bloch pair solutions, and the agreement of two
independent E_x formulas.
"""

import numpy as np
import pytest

from oracle.dense import assemble_laplacian, has_zero_mode, solve_poisson_dense, solve_screened_dense
from oracle.exx import (exchange_energy, exchange_energy_kpoints, exchange_energy_pairs, vx_apply,
                        vx_apply_kpoints)
from oracle.kron import KronSolver
from paper_2501_16572_amd.workloads import fermi_occupations, random_orbitals


def _gamma_set(n=(8, 9, 10), h=(0.4, 0.4, 0.4), nb=5, seed=7):
    psi = random_orbitals(n, h, nb, seed=seed, decay=3.0)
    return psi


@pytest.mark.parametrize("omega,bc", [(0.0, ("periodic",) * 3), (0.3, ("periodic",) * 3),
                                      (0.0, ("periodic", "periodic", "dirichlet"))])
def test_vx_matches_dense_bruteforce(omega, bc):
    n, h = (6, 7, 8), (0.45, 0.45, 0.45)
    psi = random_orbitals(n, h, 4, seed=11, decay=2.0)
    g = np.array([1.0, 0.7, 0.25, 0.0])
    S = KronSolver(n, h, bc, 12, omega)
    W = vx_apply(psi, g, psi, S)
    L = assemble_laplacian(n, h, bc, 12)
    zm = has_zero_mode(bc, (0, 0, 0))
    Wd = np.zeros_like(psi)
    for nn in range(4):
        for m in range(4):
            rho = psi[m] * psi[nn]
            phi = (solve_screened_dense(L, rho, omega, zm) if omega > 0
                   else solve_poisson_dense(L, rho, zm))
            Wd[nn] -= g[m] * psi[m] * phi
    assert np.linalg.norm(W - Wd) / np.linalg.norm(Wd) < 1e-12


def test_symmetric_pairs_equal_full():
    psi = _gamma_set()
    g = np.array([1.0, 1.0, 0.9, 0.4, 0.1])
    S = KronSolver((8, 9, 10), (0.4,) * 3, ("periodic",) * 3, 12, 0.106)
    W1 = vx_apply(psi, g, psi, S)
    W2 = vx_apply(psi, g, psi, S, pairs_symmetric=True)
    assert np.linalg.norm(W1 - W2) / np.linalg.norm(W1) < 1e-13


@pytest.mark.parametrize("omega", [0.0, 0.106])
def test_exchange_matrix_symmetric_nsd(omega):
    psi = _gamma_set(nb=6)
    g = np.array([1.0, 1.0, 1.0, 0.8, 0.3, 0.05])
    S = KronSolver((8, 9, 10), (0.4,) * 3, ("periodic",) * 3, 12, omega)
    W = vx_apply(psi[:4], g[:4], psi, S)          # Vx of the 4 occupied, on all 6
    A = (psi @ W.T) * S.dV                          # A_ab = <psi_a, Vx psi_b> dV
    assert np.allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.max() < 1e-12 * np.abs(ev).max()
    Ex = exchange_energy(psi, np.r_[g[:4], 0.0, 0.0], W, S.dV)
    assert Ex < 0


def test_linear_in_occupations_and_zero():
    psi = _gamma_set(nb=5)
    S = KronSolver((8, 9, 10), (0.4,) * 3, ("periodic",) * 3, 12, 0.0)
    g1 = np.array([1.0, 0.5, 0.0, 0.2, 0.0])
    g2 = np.array([0.0, 0.25, 1.0, 0.0, 0.3])
    Wa = vx_apply(psi, g1, psi, S)
    Wb = vx_apply(psi, g2, psi, S)
    Wab = vx_apply(psi, g1 + g2, psi, S)
    assert np.allclose(Wab, Wa + Wb, atol=1e-12 * np.abs(Wab).max())
    assert np.all(vx_apply(psi, np.zeros(5), psi, S) == 0)


def test_two_exchange_energy_formulas_agree():
    psi = _gamma_set(nb=5)
    g = fermi_occupations(5, 4, 0.01, seed=3)
    S = KronSolver((8, 9, 10), (0.4,) * 3, ("periodic",) * 3, 12, 0.106)
    W = vx_apply(psi, g, psi, S)
    E1 = exchange_energy(psi, g, W, S.dV)
    E2 = exchange_energy_pairs(psi, g, S, S.dV)
    assert E1 < 0
    assert abs(E1 - E2) < 1e-12 * abs(E2)


def test_bloch_pair_conjugate_symmetry_and_hermiticity():
    n, h = (6, 7, 8), (0.4, 0.4, 0.4)
    L = [n[d] * h[d] for d in range(3)]
    kpts = [(2 * np.pi / L[0] * 0.25, 2 * np.pi / L[1] * 0.25, 0.0),
            (-2 * np.pi / L[0] * 0.25, 2 * np.pi / L[1] * 0.25, 0.0)]
    psi = [random_orbitals(n, h, 3, seed=20 + i, kpt=k, decay=2.0) for i, k in enumerate(kpts)]
    g = [np.array([1.0, 0.6, 0.0]), np.array([1.0, 0.6, 0.0])]

    def solver_for(ik, iq):
        kq = tuple(kpts[ik][d] - kpts[iq][d] for d in range(3))
        return KronSolver(n, h, ("periodic",) * 3, 12, 0.0, kq)

    # phi_{nk,mq} = conj(phi_{mq,nk})
    S01, S10 = solver_for(0, 1), solver_for(1, 0)
    a, b = psi[1][0], psi[0][1]
    phi_ab = S01.solve(np.conj(a) * b)
    phi_ba = S10.solve(np.conj(b) * a)
    assert np.allclose(phi_ab, np.conj(phi_ba), atol=1e-12 * np.abs(phi_ab).max())
    # <psi_ak, Vx psi_bk> is Hermitian and negative semidefinite at each k
    W = vx_apply_kpoints(psi, g, [0.5, 0.5], kpts,
                         lambda kq: KronSolver(n, h, ("periodic",) * 3, 12, 0.0, kq))
    for ik in range(2):
        A = (np.conj(psi[ik]) @ W[ik].T) * np.prod(h)
        assert np.allclose(A, A.conj().T, atol=1e-12 * np.abs(A).max())
        assert np.linalg.eigvalsh(0.5 * (A + A.conj().T)).max() < 1e-12 * np.abs(A).max()


def test_bloch_solution_matches_dense():
    n, h = (5, 6, 7), (0.4, 0.4, 0.4)
    kq = (0.3, -0.5, 0.2)
    S = KronSolver(n, h, ("periodic",) * 3, 12, 0.0, kq)
    L = assemble_laplacian(n, h, ("periodic",) * 3, 12, kq)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(S.N) + 1j * rng.standard_normal(S.N)
    ref = solve_poisson_dense(L, b, False)
    assert np.linalg.norm(S.solve(b) - ref) / np.linalg.norm(ref) < 1e-12


# ---------------------------------------------------------------------------
# Pins of the k-point sum of Eq. (Vx:Poisson): which weight (w_q), which
# occupations (g_mq) and which Bloch vector (k - q) enter each term.
# ---------------------------------------------------------------------------

def _unfold(psi, n, h, k, reps):
    """Bloch orbitals on the n-grid cell extended to a reps[0] x reps[1] x
    reps[2] supercell by psi(r + T) = e^{i k.T} psi(r) (flat index x1 fastest)."""
    psi = np.asarray(psi).reshape(-1, n[2], n[1], n[0])
    out = np.empty((psi.shape[0], reps[2] * n[2], reps[1] * n[1], reps[0] * n[0]), dtype=np.complex128)
    for a in range(reps[0]):
        for b in range(reps[1]):
            for c in range(reps[2]):
                T = (a * n[0] * h[0], b * n[1] * h[1], c * n[2] * h[2])
                ph = np.exp(1j * sum(k[d] * T[d] for d in range(3)))
                out[:, c * n[2]:(c + 1) * n[2], b * n[1]:(b + 1) * n[1], a * n[0]:(a + 1) * n[0]] = ph * psi
    return out.reshape(psi.shape[0], -1)


def _kset(n, h, reps, nb, seed):
    """The k-points commensurate with the supercell, k_d = (2 pi / L_d) j / reps_d,
    with random Bloch orbitals and different occupations at every k."""
    L = [n[d] * h[d] for d in range(3)]
    kpts = [(2 * np.pi / L[0] * i / reps[0], 2 * np.pi / L[1] * j / reps[1], 2 * np.pi / L[2] * l / reps[2])
            for l in range(reps[2]) for j in range(reps[1]) for i in range(reps[0])]
    rng = np.random.default_rng(seed)
    psi = [random_orbitals(n, h, nb, seed=seed + 1 + i, kpt=k, decay=2.0).astype(np.complex128)
           for i, k in enumerate(kpts)]
    occ = []
    for i in range(len(kpts)):
        g = rng.uniform(0.05, 1.0, nb)
        g[rng.integers(1, nb):] = 0.0       # a different occupied count at each k
        occ.append(g)
    return kpts, psi, occ


@pytest.mark.parametrize("omega", [0.0, 0.3])
def test_kpoints_equal_gamma_supercell(omega):
    # A k-set commensurate with a 3 x 2 x 1 supercell: the k-point sum with
    # w = 1/N_k must equal the Gamma-point exchange of the supercell built
    # from the unfolded orbitals psi_nk / sqrt(N_k) with the same occupations
    # (the FD Laplacian commutes with cell translations, so f(L) of the
    # supercell acts on a Bloch function of wavevector k - q as the cell's
    # Bloch solver at k - q).  Along x1 the k - q are not equivalent to their
    # negatives (thirds of 2 pi / L1), so the sign of k - q is fixed, and
    # occupations differing between k-points fix g_mq against g_nk.
    n, h, reps, nb = (5, 6, 4), (0.4, 0.4, 0.4), (3, 2, 1), 3
    kpts, psi, occ = _kset(n, h, reps, nb, seed=300)
    nk = len(kpts)
    wk = [1.0 / nk] * nk
    W = vx_apply_kpoints(psi, occ, wk, kpts, lambda kq: KronSolver(n, h, ("periodic",) * 3, 12, omega, kq))
    nsc = tuple(reps[d] * n[d] for d in range(3))
    Psi = np.concatenate([_unfold(psi[i], n, h, kpts[i], reps) for i in range(nk)]) / np.sqrt(nk)
    g = np.concatenate(occ)
    Ssc = KronSolver(nsc, h, ("periodic",) * 3, 12, omega)
    Wsc = vx_apply(Psi[g > 0], g[g > 0], Psi, Ssc)
    Wunf = np.concatenate([_unfold(W[i], n, h, kpts[i], reps) for i in range(nk)]) / np.sqrt(nk)
    assert np.linalg.norm(Wunf - Wsc) / np.linalg.norm(Wsc) < 1e-12
    # the supercell holds N_k cells: its exchange energy is N_k times the
    # k-point energy per cell
    dV = float(np.prod(h))
    Ek = exchange_energy_kpoints(psi, occ, wk, W, dV)
    Esc = exchange_energy(Psi, g, Wsc, dV)
    assert Ek < 0
    assert abs(nk * Ek - Esc) < 1e-12 * abs(Esc)


def test_kpoints_one_hot_weight_is_one_q_term():
    # w = (0, 1, 0): at every k only the orbitals of the second q-point act,
    # through the Bloch solver at k - q; the weight of the target k-point
    # plays no part.
    n, h, reps, nb = (5, 6, 4), (0.4, 0.4, 0.4), (3, 1, 1), 3
    kpts, psi, occ = _kset(n, h, reps, nb, seed=310)
    wk = [0.0, 1.0, 0.0]
    W = vx_apply_kpoints(psi, occ, wk, kpts, lambda kq: KronSolver(n, h, ("periodic",) * 3, 12, 0.0, kq))
    q = 1
    on = occ[q] > 0
    for ik in range(3):
        kq = tuple(kpts[ik][d] - kpts[q][d] for d in range(3))
        ref = vx_apply(psi[q][on], occ[q][on], psi[ik], KronSolver(n, h, ("periodic",) * 3, 12, 0.0, kq))
        assert np.linalg.norm(W[ik] - ref) / np.linalg.norm(ref) < 1e-13, ik

"""Pins of the ACE oracle (Sec. III.A construction, Sec. III.B application).

The ACE operator must reproduce the exchange operator on the span of the
orbitals it was built from; these tests check that against the (separately
pinned) Vx oracle, an independent closed form that uses no Cholesky factor or
triangular solve, the triangular structure that makes xi unique, and the sign
of the operator.
"""

import numpy as np
import pytest

from oracle.ace import ace_apply, ace_construct
from oracle.exx import vx_apply
from oracle.kron import KronSolver
from paper_2501_16572_amd.workloads import fermi_occupations, random_orbitals

N3 = (10, 9, 8)
H3 = (0.4, 0.4, 0.4)


def _setup(kind, nb=5, seed=21):
    if kind == "real":
        psi = random_orbitals(N3, H3, nb, seed=seed)
        S = KronSolver(N3, H3, ("periodic",) * 3, 12, 0.3)
    else:
        L = [N3[d] * H3[d] for d in range(3)]
        k = (2 * np.pi / L[0] * 0.25, -2 * np.pi / L[1] * 0.25, 0.0)
        psi = random_orbitals(N3, H3, nb, seed=seed, kpt=k, decay=2.0)
        S = KronSolver(N3, H3, ("periodic",) * 3, 12, 0.0, (0.0, 0.0, 0.0))  # k - q = 0
    g = fermi_occupations(nb, nb - 1, 0.01, seed=seed)
    W = vx_apply(psi, g, psi, S)
    return psi, g, W, S


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_ace_reproduces_w_on_the_orbitals(kind):
    psi, g, W, S = _setup(kind)
    xi = ace_construct(psi, W, S.dV)
    V = ace_apply(xi, psi, S.dV)
    assert np.linalg.norm(V - W) <= 1e-12 * np.linalg.norm(W)


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_ace_equals_vx_on_the_span(kind):
    # any Phi = Psi C: the compressed operator acts as Vx itself
    psi, g, W, S = _setup(kind)
    xi = ace_construct(psi, W, S.dV)
    rng = np.random.default_rng(3)
    C = rng.standard_normal((3, psi.shape[0]))
    if kind == "complex":
        C = C + 1j * rng.standard_normal(C.shape)
    phi = C @ psi
    ref = vx_apply(psi, g, phi, S)
    assert np.linalg.norm(ace_apply(xi, phi, S.dV) - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_ace_matches_closed_form_without_cholesky(kind):
    # -xi (dV xi^H phi) = W M^{-1} (dV W^H phi), M = dV Psi^H W, for arbitrary phi
    psi, g, W, S = _setup(kind)
    xi = ace_construct(psi, W, S.dV)
    rng = np.random.default_rng(4)
    phi = rng.standard_normal((4, psi.shape[1]))
    if kind == "complex":
        phi = phi + 1j * rng.standard_normal(phi.shape)
    Wc, Pc = W.T, psi.T
    M = S.dV * (Pc.conj().T @ Wc)
    ref = (Wc @ np.linalg.solve(M, S.dV * (Wc.conj().T @ phi.T))).T
    got = ace_apply(xi, phi, S.dV)
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_xi_triangular_structure_and_sign(kind):
    # dV xi^H Psi = L^{-1} M = -L^H: upper triangular with a negative real
    # diagonal (this fixes xi uniquely); the operator is Hermitian and
    # negative semidefinite
    psi, g, W, S = _setup(kind)
    xi = ace_construct(psi, W, S.dV)
    G = S.dV * (xi.conj() @ psi.T)
    assert np.abs(np.tril(G, -1)).max() <= 1e-12 * np.abs(G).max()
    assert np.all(np.abs(np.imag(np.diag(G))) <= 1e-12 * np.abs(G).max())
    assert np.all(np.real(np.diag(G)) < 0)
    rng = np.random.default_rng(5)
    phi = rng.standard_normal((6, psi.shape[1]))
    A = S.dV * (phi.conj() @ ace_apply(xi, phi, S.dV).T)
    assert np.abs(A - A.conj().T).max() <= 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.conj().T)).max() <= 1e-12 * np.abs(A).max()


def test_ace_rejects_non_definite_input():
    # W = +Psi (a positive operator): -M is negative definite, no factor
    psi, g, W, S = _setup("real")
    with pytest.raises(np.linalg.LinAlgError):
        ace_construct(psi, psi, S.dV)

"""ACE construction and application on the GPU against the ACE oracle.

FP64 and complex128 kernels are compared with oracle/ace.py on identical
inputs (relative Frobenius error <= 1e-12), the full device chain
exx_apply -> ace_construct -> ace_apply must reproduce W on the orbitals, and a
non-definite -M must be reported through the info flag.
"""

import numpy as np
import pytest

from oracle.ace import ace_apply, ace_construct
from oracle.exx import vx_apply
from oracle.kron import KronSolver
from paper_2501_16572_amd.workloads import fermi_occupations, random_orbitals

from gpu_util import rel_fro, say, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def kx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_16572_amd import kronx
    kronx.load_library()
    return kronx


def _orbitals(kind, n, h, nb, seed):
    if kind == "real":
        psi = random_orbitals(n, h, nb, seed=seed)
        S = KronSolver(n, h, ("periodic",) * 3, 12, 0.106)
    else:
        L = [n[d] * h[d] for d in range(3)]
        k = (2 * np.pi / L[0] * 0.25, 2 * np.pi / L[1] * 0.25, 0.0)
        psi = random_orbitals(n, h, nb, seed=seed, kpt=k, decay=2.0)
        S = KronSolver(n, h, ("periodic",) * 3, 12, 0.0, (0.0, 0.0, 0.0))
    return psi, S


@pytest.mark.parametrize("kind", ["real", "complex"])
@pytest.mark.parametrize("nb", [6, 70])
def test_ace_matches_oracle(kx, kind, nb):
    # n_s = 70: tiles of 64 with a ragged edge; N = 20*18*16 = 5760: split-K
    # chunks of 512 rows with a ragged last chunk
    n, h = (20, 18, 16), (0.4, 0.4, 0.4)
    say("ace vs oracle", kind, nb)
    psi, S = _orbitals(kind, n, h, nb, seed=40 + nb)
    g = fermi_occupations(nb, max(nb - 2, 1), 0.01, seed=40 + nb)
    W = vx_apply(psi[: min(nb, 8)], g[: min(nb, 8)], psi, S)   # Vx from the first occupied orbitals
    xi_ref = ace_construct(psi, W, S.dV)
    ct = torch.float64 if kind == "real" else torch.complex128
    xi = kx.ace_construct(to_dev(psi, ct), to_dev(W, ct), S.dV)
    torch.cuda.synchronize()
    assert rel_fro(to_host(xi), xi_ref) < 1e-12
    rng = np.random.default_rng(9)
    phi = rng.standard_normal((5, psi.shape[1]))
    if kind == "complex":
        phi = phi + 1j * rng.standard_normal(phi.shape)
    v0 = rng.standard_normal(phi.shape) * (1 + (1j if kind == "complex" else 0))
    vphi = to_dev(v0, ct)
    kx.ace_apply(xi, to_dev(phi, ct), S.dV, vphi)
    torch.cuda.synchronize()
    ref = v0 + ace_apply(xi_ref, phi, S.dV)          # the call accumulates
    assert rel_fro(to_host(vphi), ref) < 1e-12


@pytest.mark.parametrize("kind", ["real", "complex"])
@pytest.mark.parametrize("ns", [1, 6, 70, 128, 140, 260])
def test_ace_ragged_grid_and_large_orbital_sets(kx, kind, ns):
    # N = 15*13*11 = 2145: ragged against the 32-row tiles and split-K chunks;
    # n_s = 128 fills one factorization tile exactly, 140 and 260 take the
    # tiled factorization (2 and 3 tiles, ragged last tile) and the
    # tall-skinny product in contraction slabs of 128; n_phi = 130 spans
    # several output tiles.
    # W = -Psi (B B^H + I) gives M = -(B B^H + I), Hermitian negative definite
    n, h = (15, 13, 11), (0.4, 0.4, 0.4)
    say("ace ragged", kind, ns)
    if kind == "real":
        psi = random_orbitals(n, h, ns, seed=70 + ns)
    else:
        L = [n[d] * h[d] for d in range(3)]
        psi = random_orbitals(n, h, ns, seed=70 + ns, kpt=(2 * np.pi / L[0] * 0.25, 0.0, 0.0), decay=2.0)
    dV = float(np.prod(h))
    rng = np.random.default_rng(70 + ns)
    B = rng.standard_normal((ns, ns)) / np.sqrt(ns)
    if kind == "complex":
        B = B + 1j * rng.standard_normal((ns, ns)) / np.sqrt(ns)
    W = np.ascontiguousarray(-(psi.T @ (B @ B.conj().T + np.eye(ns))).T)
    xi_ref = ace_construct(psi, W, dV)
    ct = torch.float64 if kind == "real" else torch.complex128
    xi = kx.ace_construct(to_dev(psi, ct), to_dev(W, ct), dV)
    torch.cuda.synchronize()
    assert rel_fro(to_host(xi), xi_ref) < 1e-11
    for n_phi in (5, 130):
        phi = rng.standard_normal((n_phi, psi.shape[1]))
        v0 = rng.standard_normal(phi.shape)
        if kind == "complex":
            phi = phi + 1j * rng.standard_normal(phi.shape)
            v0 = v0 + 1j * rng.standard_normal(phi.shape)
        vphi = to_dev(v0, ct)
        kx.ace_apply(xi, to_dev(phi, ct), dV, vphi)
        torch.cuda.synchronize()
        ref = v0 + ace_apply(xi_ref, phi, dV)
        assert rel_fro(to_host(vphi), ref) < 1e-11, n_phi


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_ace_padded_leading_dimensions(kx, kind):
    # every orbital set as a view with leading dimension N + 37: the padding of
    # the inputs holds NaN (any read past N would poison the result) and the
    # padding of the outputs a sentinel that must survive
    n, h, ns, n_phi, pad = (15, 13, 11), (0.4, 0.4, 0.4), 70, 9, 37
    N = n[0] * n[1] * n[2]
    say("ace padded ld", kind)
    if kind == "real":
        psi = random_orbitals(n, h, ns, seed=95)
    else:
        L = [n[d] * h[d] for d in range(3)]
        psi = random_orbitals(n, h, ns, seed=95, kpt=(2 * np.pi / L[0] * 0.25, 0.0, 0.0), decay=2.0)
    dV = float(np.prod(h))
    rng = np.random.default_rng(95)
    B = rng.standard_normal((ns, ns)) / np.sqrt(ns)
    W = np.ascontiguousarray(-(psi.T @ (B @ B.T + np.eye(ns))).T)
    phi = rng.standard_normal((n_phi, N)) * (1 + (1j if kind == "complex" else 0))
    v0 = rng.standard_normal((n_phi, N)) * (1 + (1j if kind == "complex" else 0))
    ct = torch.float64 if kind == "real" else torch.complex128

    def padded(a, fill):
        t = torch.full((a.shape[0], N + pad), fill, dtype=ct, device="cuda")
        t[:, :N] = to_dev(a, ct)
        return t

    P, Wt, Ph = padded(psi, float("nan")), padded(W, float("nan")), padded(phi, float("nan"))
    X, V = padded(np.zeros_like(W), 7.0), padded(v0, 7.0)
    kx.ace_construct(P[:, :N], Wt[:, :N], dV, xi=X[:, :N])
    kx.ace_apply(X[:, :N], Ph[:, :N], dV, V[:, :N])
    torch.cuda.synchronize()
    xi_ref = ace_construct(psi, W, dV)
    assert rel_fro(to_host(X[:, :N]), xi_ref) < 1e-12
    assert rel_fro(to_host(V[:, :N]), v0 + ace_apply(xi_ref, phi, dV)) < 1e-12
    assert bool((X[:, N:] == 7.0).all()) and bool((V[:, N:] == 7.0).all())


@pytest.mark.parametrize("kind", ["real", "complex"])
@pytest.mark.parametrize("n", [(4, 4, 4), (3, 5, 7)])
def test_ace_tiny_grids(kx, kind, n):
    # N = 64 and 105 grid points: fewer rows than one block's share, so most
    # waves of the product kernel and most split-K chunks have no work
    h, ns = (0.5, 0.5, 0.5), 5
    N = n[0] * n[1] * n[2]
    say("ace tiny", kind, n)
    rng = np.random.default_rng(N)
    A = rng.standard_normal((N, ns)) + (1j * rng.standard_normal((N, ns)) if kind == "complex" else 0)
    dV = float(np.prod(h))
    psi = np.ascontiguousarray((np.linalg.qr(A)[0] / np.sqrt(dV)).T)
    B = rng.standard_normal((ns, ns)) / np.sqrt(ns)
    W = np.ascontiguousarray(-(psi.T @ (B @ B.T + np.eye(ns))).T)
    ct = torch.float64 if kind == "real" else torch.complex128
    xi = kx.ace_construct(to_dev(psi, ct), to_dev(W, ct), dV)
    v = torch.zeros_like(xi)
    kx.ace_apply(xi, to_dev(psi, ct), dV, v)
    torch.cuda.synchronize()
    assert rel_fro(to_host(xi), ace_construct(psi, W, dV)) < 1e-12
    assert rel_fro(to_host(v), W) < 1e-12


def test_device_chain_reproduces_w(kx):
    # W = Vx Psi from exx_apply, then ACE from it: the compressed operator
    # returns W on the orbitals
    n, h, nb, no = (24, 24, 24), (0.3, 0.3, 0.3), 8, 6
    say("ace chain")
    psi = random_orbitals(n, h, nb, seed=61)
    g = fermi_occupations(nb, no, 0.01, seed=61)
    plan = kx.kron_setup(n, h, ("periodic",) * 3, 12, 0.106, prec="fp64")
    try:
        psid = to_dev(psi, torch.float64)
        w = torch.zeros_like(psid)
        kx.exx_apply(plan, psid[:no], to_dev(g[:no], torch.float64), psid, w)
        dV = float(np.prod(h))
        xi = kx.ace_construct(psid, w, dV)
        v = torch.zeros_like(psid)
        kx.ace_apply(xi, psid, dV, v)
        torch.cuda.synchronize()
        assert rel_fro(to_host(v), to_host(w)) < 1e-12
    finally:
        plan.destroy()


def test_full_size_synthetic(kx):
    # the 72^3 grid with 128 orbitals: W = -Psi (B B^T + I) gives M = -(B B^T + I)
    n, h, ns = (72, 72, 72), (0.25, 0.25, 0.25), 128
    say("ace full size")
    psi = random_orbitals(n, h, ns, seed=62)
    dV = float(np.prod(h))
    rng = np.random.default_rng(62)
    B = rng.standard_normal((ns, ns)) / np.sqrt(ns)
    W = -(psi.T @ (B @ B.T + np.eye(ns))).T
    xi_ref = ace_construct(psi, W, dV)
    psid = to_dev(psi, torch.float64)
    xi = kx.ace_construct(psid, to_dev(W, torch.float64), dV)
    v = torch.zeros_like(psid)
    kx.ace_apply(xi, psid, dV, v)
    torch.cuda.synchronize()
    assert rel_fro(to_host(xi), xi_ref) < 1e-12
    assert rel_fro(to_host(v), W) < 1e-12


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_non_definite_pivot_in_a_later_tile(kx, kind):
    # W = -Psi D with D = diag(1, ..., 1, -1 at 200): -M = D, so the factorization
    # of the third 128-tile stops at pivot 201 and nothing after it runs
    n, h, ns = (15, 13, 11), (0.4, 0.4, 0.4), 260
    if kind == "real":
        psi = random_orbitals(n, h, ns, seed=90)
    else:
        L = [n[d] * h[d] for d in range(3)]
        psi = random_orbitals(n, h, ns, seed=90, kpt=(2 * np.pi / L[0] * 0.25, 0.0, 0.0), decay=2.0)
    d = np.ones(ns)
    d[200] = -1.0
    W = np.ascontiguousarray(-(psi.T * d).T)
    ct = torch.float64 if kind == "real" else torch.complex128
    with pytest.raises(kx.KronxError, match="pivot 201"):
        kx.ace_construct(to_dev(psi, ct), to_dev(W, ct), float(np.prod(h)))


def test_non_definite_reported(kx):
    n, h, nb = (16, 16, 16), (0.4, 0.4, 0.4), 6
    psi = random_orbitals(n, h, nb, seed=63)
    psid = to_dev(psi, torch.float64)
    with pytest.raises(kx.KronxError):
        kx.ace_construct(psid, psid, float(np.prod(h)))   # -M = -I: first pivot fails
    with pytest.raises(kx.KronxError):
        kx.ace_construct(psid, psid, -1.0)                 # dV must be positive (EINVAL)

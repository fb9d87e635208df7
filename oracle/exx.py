"""Exact-exchange application and exchange energy (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (Vx:Poisson) of arXiv 2501.16572:

    Vx phi_nk(r) = - sum_{m,q} w_q g_mq psi_mq(r) phi_{mq,nk}(r),

where phi_{mq,nk} solves Eq. (Poisson) (unscreened) or Eq. (Poisson:SR)
(screened) with right-hand side psi*_mq(r) varphi_nk(r) under Bloch conditions
at k - q (Sec. II).  The same quantity is W^(n) of Eq. (W) when varphi runs
over the orbitals themselves.

Reading R5 (exchange energy; the paper defines none): spin-unpolarized, with
g in [0, 1] per spatial orbital,

    E_x = sum_k w_k sum_n g_nk Re <psi_nk, Vx psi_nk> dV,

<a, b> = sum_r conj(a) b and dV = h1 h2 h3.  Equivalently
E_x = - sum_{k,q} w_k w_q sum_{n,m} g_nk g_mq dV <rho, f(L) rho>,
rho = conj(psi_mq) psi_nk.
"""

import numpy as np


def vx_apply(psi, occ, phi, solver, pairs_symmetric=False):
    """W_n = - sum_m occ_m psi_m (.) solve(conj(psi_m) (.) phi_n) for one (k, q).

    psi: (n_occ, N) occupied orbitals at q; occ: (n_occ,) weights w_q g_mq;
    phi: (n_b, N) functions at k; solver: an object with ``solve`` (a
    KronSolver at kappa = k - q).  Returns (n_b, N).

    pairs_symmetric: at the Gamma point with real orbitals and phi == psi the
    pair solution is symmetric, phi_mn = phi_nm, so each unordered pair is
    solved once (n(n+1)/2 solves) and used for both targets.
    """
    psi = np.asarray(psi)
    phi = np.asarray(phi)
    occ = np.asarray(occ, dtype=np.float64)
    n_occ = psi.shape[0]
    n_b = phi.shape[0]
    dtype = np.result_type(psi.dtype, phi.dtype, solver.V[0].dtype)
    W = np.zeros((n_b, phi.shape[1]), dtype=dtype)
    if pairs_symmetric:
        if n_occ != n_b or np.iscomplexobj(psi) or np.iscomplexobj(phi):
            raise ValueError("symmetric pairs need real psi == phi")
        for i in range(n_b):
            rho = psi[i:] * phi[i][None, :]          # pairs (m >= i, n = i)
            sol = solver.solve(rho)
            for t, m in enumerate(range(i, n_b)):
                W[i] -= occ[m] * psi[m] * sol[t]
                if m != i:
                    W[m] -= occ[i] * psi[i] * sol[t]
        return W
    for n in range(n_b):
        rho = np.conj(psi) * phi[n][None, :]
        sol = solver.solve(rho)
        W[n] = -np.einsum("m,mr->r", occ, psi * sol) if n_occ else 0.0
    return W


def exchange_energy(psi, g, W, dV):
    """E_x contribution sum_n g_n Re <psi_n, W_n> dV (reading R5)."""
    psi = np.asarray(psi)
    g = np.asarray(g, dtype=np.float64)
    return float(np.sum(g * np.real(np.sum(np.conj(psi) * W, axis=1))) * dV)


def exchange_energy_pairs(psi, g, solver, dV):
    """Cross-formula E_x = - sum_{n,m} g_n g_m dV <rho_mn, f(L) rho_mn>, one (k, q)
    block with psi at both k and q (Gamma).  Independent of ``vx_apply``."""
    psi = np.asarray(psi)
    g = np.asarray(g, dtype=np.float64)
    E = 0.0
    for n in range(psi.shape[0]):
        rho = np.conj(psi) * psi[n][None, :]
        sol = solver.solve(rho)
        quad = np.real(np.sum(np.conj(rho) * sol, axis=1))
        E -= g[n] * float(np.sum(g * quad)) * dV
    return E


def vx_apply_kpoints(psi_k, occ_k, w_k, kpts, make_solver):
    """Eq. (Vx:Poisson) over a k-point set (one spin channel).

    psi_k: list over k of (n_b, N) Bloch orbitals psi_nk(r) (the full Bloch
    function on the cell's grid); occ_k: list of (n_b,) occupations g_nk;
    w_k: Brillouin-zone weights; kpts: list of k vectors (bohr^-1);
    make_solver(kappa): a KronSolver with Bloch vector kappa.

    For the target k and every q, the pair density conj(psi_mq) psi_nk is a
    Bloch function with wavevector k - q, so its Poisson problem is solved
    under the Bloch condition at kappa = k - q (Sec. II); the source orbitals
    are the occupied ones at q (g_mq > 0), weighted by w_q g_mq.  Returns the
    list over k of Vx psi_nk, shape (n_b, N).
    """
    nk = len(psi_k)
    out = []
    for ik in range(nk):
        W = 0
        for iq in range(nk):
            kappa = tuple(float(kpts[ik][d]) - float(kpts[iq][d]) for d in range(3))
            occ_mask = occ_k[iq] > 0
            w = w_k[iq] * occ_k[iq][occ_mask]
            W = W + vx_apply(psi_k[iq][occ_mask], w, psi_k[ik], make_solver(kappa))
        out.append(W)
    return out


def exchange_energy_kpoints(psi_k, occ_k, w_k, W_k, dV):
    """E_x = sum_k w_k sum_n g_nk Re <psi_nk, W_nk> dV over a k-point set (R5)."""
    return float(sum(w_k[ik] * exchange_energy(psi_k[ik], occ_k[ik], W_k[ik], dV)
                     for ik in range(len(psi_k))))

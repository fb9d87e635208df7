"""Seeded synthetic workloads: grids, orbitals and occupations.

This module holds only input generation (random numbers, orthonormalization,
occupation ladders) and the workload definitions; none of the exact-exchange
arithmetic.  Both the device path's tests/benchmarks and the CPU oracle take
their inputs from here, so both see the same arrays.

The paper's own systems (Mo bulk, TiO2 slabs with pseudopotentials, Sec. IV)
are not available; these synthetic inputs stand in for them with the same
kind of shapes: uniform grids of 24^3-120^3 points at h = 0.2-0.3 bohr,
hundreds of smooth orbitals, Fermi-smeared occupations and slabs with vacuum.

Grid layout: flat index i1 + n1*(i2 + n2*i3) (x1 fastest); a set of orbitals
is an array of shape (n_orb, N), one orbital per row (= column-major N x n_orb
with leading dimension N).
"""

import numpy as np


def _recip_axis(n, h):
    return 2.0 * np.pi * np.fft.fftfreq(n, d=h)


def random_orbitals(n, h, n_orb, seed, kpt=(0.0, 0.0, 0.0), envelope_z=None,
                    decay=8.0, rng=None):
    """Smooth random orbitals, orthonormalized so that dV * Psi^H Psi = I.

    Each orbital: Fourier coefficients c(G) = (N(0,1) + i N(0,1)) *
    exp(-|G + k|^2 / decay) on the reciprocal grid G_d = 2 pi fftfreq(n_d, h_d),
    transformed to real space by an inverse FFT; the real part is kept at the
    Gamma point, and at k != 0 the periodic part is multiplied by e^{i k.r}.
    ``envelope_z`` (callable of the x3 coordinate array) confines slab
    orbitals.  Then QR orthonormalization, Psi <- Q / sqrt(dV).

    Returns (n_orb, N) float64 (Gamma) or complex128 (k != 0).
    """
    n1, n2, n3 = n
    h1, h2, h3 = h
    rng = np.random.default_rng(seed) if rng is None else rng
    g1 = _recip_axis(n1, h1)[None, None, :] + kpt[0]
    g2 = _recip_axis(n2, h2)[None, :, None] + kpt[1]
    g3 = _recip_axis(n3, h3)[:, None, None] + kpt[2]
    weight = np.exp(-(g1 * g1 + g2 * g2 + g3 * g3) / decay)
    bloch = any(k != 0.0 for k in kpt)
    N = n1 * n2 * n3
    A = np.empty((N, n_orb), dtype=np.complex128 if bloch else np.float64)
    if bloch:
        x1 = (np.arange(n1) * h1)[None, None, :]
        x2 = (np.arange(n2) * h2)[None, :, None]
        x3 = (np.arange(n3) * h3)[:, None, None]
        phase = np.exp(1j * (kpt[0] * x1 + kpt[1] * x2 + kpt[2] * x3))
    env = None
    if envelope_z is not None:
        z = (np.arange(n3) - (n3 - 1) / 2.0) * h3
        env = np.asarray(envelope_z(z), dtype=np.float64)[:, None, None]
    for j in range(n_orb):
        re = rng.standard_normal((n3, n2, n1))
        im = rng.standard_normal((n3, n2, n1))
        u = np.fft.ifftn((re + 1j * im) * weight)
        psi = u * phase if bloch else u.real
        if env is not None:
            psi = psi * env
        A[:, j] = psi.reshape(-1)
    Q, _ = np.linalg.qr(A)
    dV = h1 * h2 * h3
    return np.ascontiguousarray((Q / np.sqrt(dV)).T)


def fermi_occupations(n_b, n_occ, kT, seed, rng=None):
    """Fermi-smeared occupations on a seeded random eigenvalue ladder.

    eps = cumulative sum of U(0, 2 kT) gaps; mu = eps[n_occ - 6];
    g_j = 1 / (1 + exp((eps_j - mu)/kT)) for j < n_occ and 0 beyond, which
    mixes g ~ 1 with fractional occupations near the Fermi level.
    """
    rng = np.random.default_rng(seed) if rng is None else rng
    eps = np.cumsum(rng.uniform(0.0, 2.0 * kT, size=n_b))
    mu = eps[max(n_occ - 6, 0)]
    g = 1.0 / (1.0 + np.exp((eps - mu) / kT))
    g[n_occ:] = 0.0
    return g


def slab_envelope(z):
    """Gaussian envelope exp(-z^2/50) for |z| < 15 bohr, 0 beyond (20 bohr of
    vacuum in a 50-bohr cell)."""
    return np.where(np.abs(z) < 15.0, np.exp(-z * z / 50.0), 0.0)


# ---------------------------------------------------------------------------
# Workload definitions.  Each is a dict; ``make_inputs`` draws the arrays.
# ---------------------------------------------------------------------------

OMEGA_HSE = 0.106  # bohr^-1, screening parameter of the erfc(omega r)/r kernel

CONFIGS = {
    # small Gamma-point case, unscreened (PBE0-like), all 8 orbitals occupied
    "gamma24": dict(n=(24, 24, 24), h=(0.3, 0.3, 0.3), bc=("periodic",) * 3,
                    order=12, omega=0.0, n_b=8, n_occ=8, occ="ones", seed=1,
                    prec="fp64"),
    # Gamma-point HSE, 72^3, 128 bands / 96 occupied with Fermi smearing
    "hse72": dict(n=(72, 72, 72), h=(0.25, 0.25, 0.25), bc=("periodic",) * 3,
                  order=12, omega=OMEGA_HSE, n_b=128, n_occ=96, occ="fermi",
                  kT=0.01, seed=2, prec="fp64"),
    # Gamma-point HSE, 120^3, 384 bands / 320 occupied, mixed precision
    "hse120": dict(n=(120, 120, 120), h=(0.2, 0.2, 0.2), bc=("periodic",) * 3,
                   order=12, omega=OMEGA_HSE, n_b=384, n_occ=320, occ="fermi",
                   kT=0.01, seed=3, prec="fp32"),
    # slab: periodic x1, x2; Dirichlet x3 with 20 bohr of vacuum
    "slab96": dict(n=(96, 96, 160), h=(0.3125, 0.3125, 0.3125),
                   bc=("periodic", "periodic", "dirichlet"), order=12,
                   omega=OMEGA_HSE, n_b=256, n_occ=200, occ="fermi", kT=0.01,
                   seed=4, envelope=True, prec="fp32"),
}


# Several plans in one batched call: a 2x2x1 Monkhorst-Pack k-point set on an
# 80^3 grid (Coulomb kernel; Bloch phase k - q, four distinct operators up to
# reciprocal lattice vectors) and six Gamma-point systems of uneven sizes
# (erfc kernel).  h = 0.25 bohr; 3/4 of the bands occupied.
BATCH5 = dict(
    kind="batched", prec="fp32",
    kgrid=dict(n=(80, 80, 80), h=(0.25, 0.25, 0.25), bc=("periodic",) * 3, order=12, omega=0.0,
               n_b=160, n_occ=120, kT=0.01, seed=50, mp=(2, 2, 1)),
    systems=[((48, 48, 48), 64, 48), ((56, 56, 56), 96, 72), ((64, 64, 64), 128, 96),
             ((64, 64, 96), 128, 96), ((72, 72, 72), 160, 120), ((90, 90, 90), 192, 144)],
    h=0.25, omega=OMEGA_HSE, order=12, kT=0.01, seed=51)
CONFIGS["batch5"] = BATCH5


def monkhorst_pack(n, h, mp):
    """k-points (2 pi / L_d) * ((2 i - m_d + 1) / (2 m_d)) of an m1 x m2 x m3
    Monkhorst-Pack set (no shift beyond the standard one) and equal weights."""
    L = [n[d] * h[d] for d in range(3)]
    axes = [[2.0 * np.pi / L[d] * (2 * i - mp[d] + 1) / (2.0 * mp[d]) for i in range(mp[d])]
            for d in range(3)]
    ks = [(a, b, c) for c in axes[2] for b in axes[1] for a in axes[0]]
    return ks, [1.0 / len(ks)] * len(ks)


def bloch_class(kq, n, h):
    """Representative of the Bloch vector k - q modulo reciprocal lattice
    vectors (2 pi / L_d): the FD operator depends on it only through the
    boundary phase exp(i kappa_d L_d)."""
    out = []
    for d in range(3):
        G = 2.0 * np.pi / (n[d] * h[d])
        r = float(np.mod(kq[d], G))
        if abs(r - G) < 1e-12 * G or abs(r) < 1e-12 * G:
            r = 0.0
        out.append(r)
    return tuple(out)


def make_batch_inputs(cfg, progress=None):
    """Inputs of the batched workload.

    Returns (kpart, systems): kpart = dict(kpts, wk, psi (list of (n_b, N)
    complex128), g (list of (n_b,))); systems = list of dicts with n, h, psi
    (n_b, N) float64, g (n_b,) and n_occ.  ``progress`` (optional callable)
    is called with a short text before each set of orbitals is drawn.
    """
    kg = cfg["kgrid"]
    ks, wk = monkhorst_pack(kg["n"], kg["h"], kg["mp"])
    rng = np.random.default_rng(kg["seed"])
    psi_k, g_k = [], []
    for ik, k in enumerate(ks):
        if progress:
            progress(f"orbitals of k-point {ik}")
        psi_k.append(random_orbitals(kg["n"], kg["h"], kg["n_b"], seed=None, rng=rng, kpt=k))
        g_k.append(fermi_occupations(kg["n_b"], kg["n_occ"], kg["kT"], seed=None, rng=rng))
    kpart = dict(kpts=ks, wk=wk, psi=psi_k, g=g_k, n_occ=kg["n_occ"])
    systems = []
    for i, (n, nb, no) in enumerate(cfg["systems"]):
        if progress:
            progress(f"orbitals of system {i} ({n})")
        rng = np.random.default_rng(cfg["seed"] + i)
        h = (cfg["h"],) * 3
        psi = random_orbitals(n, h, nb, seed=None, rng=rng)
        g = fermi_occupations(nb, no, cfg["kT"], seed=None, rng=rng)
        systems.append(dict(n=n, h=h, psi=psi, g=g, n_occ=no))
    return kpart, systems


def make_inputs(cfg, n_b=None, dtype=np.float64):
    """Orbitals (n_b, N) and occupations (n_b,) for a Gamma-point workload.

    ``n_b`` may cut the band count for reduced-size tests (the generator draws
    the same first orbitals' coefficients, but QR over fewer columns changes
    them; reduced sets are their own seeded workload).
    """
    nb = cfg["n_b"] if n_b is None else n_b
    rng = np.random.default_rng(cfg["seed"])
    env = slab_envelope if cfg.get("envelope") else None
    psi = random_orbitals(cfg["n"], cfg["h"], nb, seed=None, rng=rng, envelope_z=env)
    n_occ = min(cfg["n_occ"], nb)
    if cfg["occ"] == "ones":
        g = np.zeros(nb)
        g[:n_occ] = 1.0
    else:
        g = fermi_occupations(nb, n_occ, cfg["kT"], seed=None, rng=rng)
    return psi.astype(dtype, copy=False), g

"""The seeded input generators that the device path and the oracle share:
orthonormality, Bloch form, occupations, k-point sets and their classes."""

import numpy as np
import pytest

from paper_2501_16572_amd.workloads import (CONFIGS, bloch_class, fermi_occupations, make_inputs,
                                            monkhorst_pack, random_orbitals, slab_envelope)


@pytest.mark.parametrize("kpt", [(0.0, 0.0, 0.0), (0.3, -0.2, 0.1)])
def test_orbitals_orthonormal_and_seeded(kpt):
    n, h = (10, 12, 8), (0.3, 0.25, 0.4)
    psi = random_orbitals(n, h, 6, seed=5, kpt=kpt)
    dV = h[0] * h[1] * h[2]
    assert psi.shape == (6, 960)
    assert psi.dtype == (np.float64 if kpt == (0.0, 0.0, 0.0) else np.complex128)
    gram = dV * psi.conj() @ psi.T
    assert np.allclose(gram, np.eye(6), atol=1e-12)
    assert np.array_equal(psi, random_orbitals(n, h, 6, seed=5, kpt=kpt))
    assert not np.allclose(psi, random_orbitals(n, h, 6, seed=6, kpt=kpt))


def _high_frequency_fraction(f):
    """Share of the DFT energy (over the three grid axes) at frequencies above
    a quarter of each axis' range."""
    F = np.abs(np.fft.fftn(f, axes=(1, 2, 3))) ** 2
    hi = np.zeros(F.shape[1:], dtype=bool)
    for ax in range(3):
        nd = F.shape[1 + ax]
        idx = np.abs(np.fft.fftfreq(nd) * nd) > nd / 4
        shape = [1, 1, 1]
        shape[ax] = nd
        hi |= idx.reshape(shape)
    return F[:, hi].sum() / F.sum()


def test_bloch_orbitals_have_a_smooth_periodic_part():
    # psi(r) = e^{i k.r} u(r) with u smooth and periodic over the cell: u has
    # almost no high-frequency content, while psi, whose phase does not wrap
    # around the cell, does (a missing or sign-flipped phase fails one of the two)
    n, h, k = (16, 20, 12), (0.3, 0.3, 0.3), (0.4, -0.7, 0.25)
    psi = random_orbitals(n, h, 3, seed=9, kpt=k).reshape(3, n[2], n[1], n[0])
    x1 = np.arange(n[0]) * h[0]
    x2 = np.arange(n[1]) * h[1]
    x3 = np.arange(n[2]) * h[2]
    phase = np.exp(1j * (k[0] * x1[None, None, :] + k[1] * x2[None, :, None] + k[2] * x3[:, None, None]))
    u = psi / phase[None]
    assert _high_frequency_fraction(u) < 2e-3          # measured 1.6e-4
    assert _high_frequency_fraction(psi) > 1e-2        # 4.9e-2
    assert _high_frequency_fraction(psi * phase[None]) > 1e-2  # e^{-ikr} in place of e^{ikr}: 7.4e-2


def test_fermi_occupations():
    g = fermi_occupations(40, 30, 0.01, seed=3)
    assert g.shape == (40,)
    assert np.all(g[30:] == 0.0)
    assert np.all((g[:30] > 0.0) & (g[:30] <= 1.0))
    assert np.all(np.diff(g[:30]) <= 0.0)  # ladder rises, occupations fall
    assert g[0] > 0.99 and g[29] < 0.5
    assert np.array_equal(g, fermi_occupations(40, 30, 0.01, seed=3))


def test_slab_envelope_vacuum_is_zero():
    z = np.linspace(-25.0, 25.0, 101)
    e = slab_envelope(z)
    assert np.all(e[np.abs(z) >= 15.0] == 0.0)
    assert e[50] == 1.0 and np.all(e >= 0.0)


def test_monkhorst_pack_2x2x1():
    n, h = (80, 80, 80), (0.25, 0.25, 0.25)
    ks, wk = monkhorst_pack(n, h, (2, 2, 1))
    G = 2.0 * np.pi / 20.0
    assert len(ks) == 4 and wk == [0.25] * 4
    assert np.allclose(np.sum(ks, axis=0), 0.0)
    assert {round(k[0] / G, 12) for k in ks} == {-0.25, 0.25}
    assert all(k[2] == 0.0 for k in ks)


def test_bloch_classes_of_the_2x2x1_set():
    # k - q over the 16 pairs of a 2x2x1 set falls into 4 classes modulo the
    # reciprocal lattice: 0 and G/2 along each of the two sampled axes
    n, h = (80, 80, 80), (0.25, 0.25, 0.25)
    ks, _ = monkhorst_pack(n, h, (2, 2, 1))
    classes = {bloch_class(tuple(a[d] - b[d] for d in range(3)), n, h) for a in ks for b in ks}
    G = 2.0 * np.pi / 20.0
    assert classes == {(0.0, 0.0, 0.0), (G / 2, 0.0, 0.0), (0.0, G / 2, 0.0), (G / 2, G / 2, 0.0)}
    # a full reciprocal vector is class 0, and -G/2 is the same class as G/2
    assert bloch_class((G, -G, 2 * G), n, h) == (0.0, 0.0, 0.0)
    assert bloch_class((-G / 2, 0.0, 0.0), n, h) == pytest.approx((G / 2, 0.0, 0.0))


def test_make_inputs_small_cut_of_a_workload():
    cfg = CONFIGS["gamma24"]
    psi, g = make_inputs(cfg)
    assert psi.shape == (8, 24 ** 3) and np.all(g == 1.0)
    dV = 0.3 ** 3
    assert np.allclose(dV * psi @ psi.T, np.eye(8), atol=1e-12)

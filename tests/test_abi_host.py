"""Host-side checks of the C ABI (no GPU needed).

The library must load and export every function include/kronx.h declares;
the host plan's FD weights and 1D eigenpairs must match the oracle (compared
through basis-invariant quantities: eigenvalues and V diag(lam) V^H, never
eigenvectors entrywise); argument errors must come back as status codes
before any device work.
"""

import ctypes
import os
import re
from fractions import Fraction

import numpy as np
import pytest

from oracle.fd import fd_weights, second_derivative_1d
from paper_2501_16572_amd import kronx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "kronx.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"(?:kx_status|size_t|const char\s*\*)\s*(\w+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = kronx.load_library()
    declared = _declared_functions()
    assert set(declared) == set(kronx.EXPORTS), declared
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("order", [2, 4, 8, 12, 16])
def test_host_fd_weights_match_oracle(order):
    c = kronx.kx_host_fd_weights(order)
    ref = [float(x) for x in fd_weights(order)]
    assert np.allclose(c, ref, rtol=1e-15, atol=1e-15)


CASES = [(24, 0.3, "periodic", 0.0), (25, 0.25, "periodic", 0.0), (7, 0.4, "periodic", 0.0),
         (72, 0.25, "periodic", 0.0), (16, 0.3, "periodic", 0.37), (9, 0.3, "periodic", -1.2),
         (30, 0.3125, "dirichlet", 0.0), (11, 0.2, "dirichlet", 0.0), (5, 0.3, "periodic", 0.0)]


@pytest.mark.parametrize("n,h,bc,kappa", CASES)
def test_host_eig1d_reconstructs_oracle_operator(n, h, bc, kappa):
    lam, V = kronx.kx_host_eig1d(n, h, bc, 12, kappa)
    D = second_derivative_1d(n, h, bc, 12, kappa)
    scale = np.abs(lam).max()
    # ascending, matches the oracle operator's spectrum
    assert np.all(np.diff(lam) >= -1e-12 * scale)
    ref = np.linalg.eigvalsh(D)
    assert np.allclose(lam, ref, rtol=0, atol=1e-11 * scale)
    # orthonormal (unitary) and V diag(lam) V^H == D
    assert np.allclose(V.conj().T @ V, np.eye(n), atol=1e-13)
    assert np.allclose((V * lam) @ V.conj().T, D, atol=1e-11 * scale)
    if kappa == 0.0:
        assert not np.iscomplexobj(V)


def test_host_eig1d_zero_mode_exact():
    lam, _ = kronx.kx_host_eig1d(24, 0.3, "periodic", 12, 0.0)
    assert lam[-1] == 0.0  # periodic: the constant mode is exactly zero


@pytest.mark.parametrize("bad", [
    dict(n=(0, 8, 8)), dict(n=(8, 8, 200)), dict(h=(0.3, -0.1, 0.3)), dict(bc=(0, 5, 0)),
    dict(fd_order=7), dict(fd_order=0), dict(kq=(0.0, 0.0, 0.3), bc=(0, 0, 1)),
    dict(prec="bogus"),
])
def test_kron_setup_argument_errors(bad):
    args = dict(n=(8, 8, 8), h=(0.3, 0.3, 0.3), bc=(0, 0, 0), fd_order=12, omega=0.0, kq=None,
                prec="fp64")
    args.update(bad)
    lib = kronx.load_library()
    handle = ctypes.c_void_p(1234)
    prec = kronx.PREC.get(args["prec"], 99)
    kq = (ctypes.c_double * 3)(*args["kq"]) if args["kq"] else None
    st = lib.kron_setup((ctypes.c_int * 3)(*args["n"]), (ctypes.c_double * 3)(*args["h"]),
                        (ctypes.c_int * 3)(*args["bc"]), args["fd_order"], args["omega"], kq,
                        prec, ctypes.byref(handle))
    assert st in (kronx.KX_EINVAL, kronx.KX_EUNSUPPORTED)
    assert handle.value is None
    assert kronx.kx_last_error() != ""


def test_null_plan_errors():
    lib = kronx.load_library()
    assert lib.kron_solve(None, None, 0, None, 0, 1, 0, None) == kronx.KX_EINVAL
    assert lib.exx_apply(None, None, 0, 1, None, None, 0, 1, None, 0, None, None, 0, None) == kronx.KX_EINVAL
    assert lib.kron_destroy(None) == kronx.KX_OK
    assert lib.exx_apply_batched(None, -1, None) == kronx.KX_EINVAL
    assert lib.kx_host_eig1d(0, 0.3, 0, 12, 0.0, None, None, None) == kronx.KX_EINVAL
    assert lib.kx_host_fd_weights(5, None) == kronx.KX_EINVAL


def test_ace_workspace_size_and_argument_errors():
    # host-only: the workspace formula (split-K partials of the MFMA Gram
    # product: about 512 blocks over the 128 x 128 (complex 128 x 64) output
    # tiles, chunks a multiple of 32 doubles, each chunk x tile a 128 KiB
    # partial; 256-byte aligned; plus the small n_s x n_s matrices) and EINVAL
    # before any device work
    def part_bytes(N, m, n, cplx):
        tiles = -(-m // 128) * -(-n // (64 if cplx else 128))
        K2 = N * (2 if cplx else 1)
        chunks = min(max(1, 512 // tiles), -(-K2 // 32))
        kc2 = -(-(-(-K2 // chunks)) // 32) * 32
        return -(-K2 // kc2) * tiles * 128 * 128 * 8

    align = lambda b: (b + 255) // 256 * 256
    N, ns = 373248, 128
    assert part_bytes(N, ns, ns, False) == 508 * 128 * 1024   # 736-row chunks
    assert kronx.kx_ace_workspace_bytes(N, ns, 0, False) == align(part_bytes(N, ns, ns, False)) + align(
        (3 * ns * ns + ns) * 8)
    for (N, ns, nphi, cplx) in [(373248, 128, 200, True), (2145, 140, 130, False), (2145, 6, 5, True),
                                (100, 1024, 1, False)]:
        part = max(part_bytes(N, ns, ns, cplx), part_bytes(N, ns, nphi, cplx))
        eb = 16 if cplx else 8
        assert kronx.kx_ace_workspace_bytes(N, ns, nphi, cplx) == align(part) + align(
            (3 * ns * ns + ns * nphi) * eb), (N, ns, nphi, cplx)
    lib = kronx.load_library()
    for bad in [(0, 4), (100, 0), (100, 1025)]:
        out = ctypes.c_int64(0)
        assert lib.kx_ace_workspace_bytes(bad[0], bad[1], 0, 0, ctypes.byref(out)) == kronx.KX_EINVAL
    st = lib.ace_construct(1000, 4, 0, 1.0, None, 1000, None, 1000, None, 1000, None, 0, None, None)
    assert st == kronx.KX_EINVAL
    assert "NULL" in kronx.kx_last_error() or "need" in kronx.kx_last_error()
    st = lib.ace_apply(1000, 4, 0, 1.0, None, 1000, None, 1000, 0, None, 1000, None, 0, None)
    assert st == kronx.KX_OK  # n_phi = 0: no-op

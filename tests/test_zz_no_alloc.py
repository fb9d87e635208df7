"""exx_apply_static (the entry point that allocates nothing) against exx_apply.

Both run the same kernels; the static one keeps its pair workspace and E_x
partials in the library's fixed device array instead of plan-owned buffers.
Vx must match exx_apply's to the FP64 bar (1e-12 relative; the per-target
accumulation order is the same, so it is in fact bitwise equal) and E_x to
1e-12 relative (the batch split may differ, which changes the order in which
batch sums reach E_x).  Two calls in a row, the second with a smaller input,
show that the array's leftover contents from the first call do not leak into
the second.
"""

import numpy as np
import pytest

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


def _inputs(n, h, n_b, n_occ, seed, kpt=(0.0, 0.0, 0.0)):
    psi = random_orbitals(n, h, n_b, seed, kpt=kpt)
    g = fermi_occupations(n_b, n_occ, 0.01, seed)
    return psi, g


def _both(kx, plan, psi, g, n_occ, n_b, dt, vdt):
    """(exx_apply result, exx_apply_static result) on the same inputs: the
    first n_occ orbitals are the occupied set, the first n_b the targets."""
    psid = to_dev(psi[:max(n_b, n_occ)], dt)
    gd = to_dev(g[:max(n_b, n_occ)], torch.float64)
    occ = gd[:n_occ].contiguous()
    out = []
    for fn in (kx.exx_apply, kx.exx_apply_static):
        vx = torch.zeros((n_b, psid.shape[1]), dtype=vdt, device="cuda")
        ex = torch.zeros(1, dtype=torch.float64, device="cuda")
        fn(plan, psid[:n_occ], occ, psid[:n_b], vx, ex=ex, gphi=gd[:n_b].contiguous())
        torch.cuda.synchronize()
        out.append((to_host(vx), float(ex.item())))
    return out


CASES = [
    # name, n, h, prec, complex kpt, (n_b, n_occ) first call, (n_b, n_occ) second call
    ("fp64-24", (24, 24, 24), (0.3, 0.3, 0.3), "fp64", None, (12, 10), (5, 3)),
    ("fp64-multibatch", (64, 64, 64), (0.25, 0.25, 0.25), "fp64", None, (24, 40), (7, 9)),
    ("fp32-40", (40, 36, 44), (0.25, 0.3, 0.28), "fp32", None, (16, 12), (3, 2)),
    ("c128-bloch", (20, 18, 16), (0.3, 0.3, 0.3), "fp64", (0.2, -0.1, 0.15), (10, 8), (4, 3)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_static_matches_exx_apply_two_calls(kx, case):
    name, n, h, prec, kpt, first, second = case
    cplx = kpt is not None
    n_orb = max(first + second)
    psi, g = _inputs(n, h, n_orb, max(first[1], second[1]), 300, kpt=kpt if cplx else (0.0, 0.0, 0.0))
    plan = kx.kron_setup(n, h, ("periodic",) * 3, 12, 0.106, kq=(0.0, 0.0, 0.0) if cplx else None,
                         prec=prec, complex=cplx)
    try:
        dt = plan.dtype
        vdt = torch.complex128 if cplx else torch.float64
        for n_b, n_occ in (first, second):
            say("exx_apply_static vs exx_apply", name, n, prec, "n_b", n_b, "n_occ", n_occ)
            (v_ref, e_ref), (v_st, e_st) = _both(kx, plan, psi, g, n_occ, n_b, dt, vdt)
            assert rel_fro(v_st, v_ref) <= 1e-12, (name, n_b, n_occ, rel_fro(v_st, v_ref))
            assert abs(e_st - e_ref) <= 1e-12 * abs(e_ref), (name, e_st, e_ref)
            assert np.isfinite(v_st).all()
    finally:
        plan.destroy()


def test_static_allocates_nothing_and_rejects_oversize(kx):
    """After the first call (which may load the library's device code), further
    calls of different sizes leave the device's free memory unchanged; a
    target whose pair workspace exceeds the fixed array is rejected."""
    n, h = (64, 64, 64), (0.25, 0.25, 0.25)
    cap = kx.kx_static_scratch_bytes()
    assert cap == 256 << 20
    N = n[0] * n[1] * n[2]
    n_big = cap // (N * 8) + 1          # one target needs more than the array
    rng = np.random.default_rng(5)
    psi = to_dev(rng.standard_normal((n_big, N)) * 1e-3, torch.float64)
    occ = torch.ones(n_big, dtype=torch.float64, device="cuda")
    plan = kx.kron_setup(n, h, ("periodic",) * 3, 12, 0.0, prec="fp64")
    try:
        vx = torch.zeros((6, N), dtype=torch.float64, device="cuda")
        say("exx_apply_static warm call", n)
        kx.exx_apply_static(plan, psi[:8], occ[:8], psi[:6], vx)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for nb, no in ((6, 20), (3, 5), (6, 30)):
            say("exx_apply_static sizes", nb, no)
            kx.exx_apply_static(plan, psi[:no], occ[:no], psi[:nb], vx[:nb])
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        say("exx_apply_static oversize rejection", n_big)
        with pytest.raises(kx.KronxError) as err:
            kx.exx_apply_static(plan, psi, occ, psi[:1], vx[:1])
        assert "exx_apply_static" in str(err.value) and err.value.status == kx.KX_EINVAL
        assert torch.isfinite(vx).all()
    finally:
        plan.destroy()

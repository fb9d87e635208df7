"""The Python binding refuses tensors that do not fit a call (CPU only).

Every check runs before the library is called, so a wrong element type, a
short vector or a host tensor raises ValueError instead of handing the
kernels a pointer they would read or write out of bounds.  The plans here
carry no library handle: a check that let a tensor through would reach the
library with a NULL plan and come back as a KronxError, not a ValueError.
"""

import pytest

from paper_2501_16572_amd import kronx

torch = pytest.importorskip("torch")

N = 6 * 5 * 4


def _plan(prec="fp64", cplx=False):
    return kronx.Plan(None, (6, 5, 4), (0.3,) * 3, ("periodic",) * 3, 12, 0.0, (0.0, 0.0, 0.0), prec,
                      complex_=cplx)


def _good(plan, n_occ=3, n_b=4):
    dt = plan.dtype
    vdt = torch.complex128 if plan.complex else torch.float64
    return dict(psi=torch.zeros((n_occ, N), dtype=dt), occ=torch.ones(n_occ, dtype=torch.float64),
                phi=torch.zeros((n_b, N), dtype=dt), vx=torch.zeros((n_b, N), dtype=vdt),
                ex=torch.zeros(1, dtype=torch.float64), gphi=torch.ones(n_b, dtype=torch.float64))


def _exx(plan, a):
    return kronx.exx_apply(plan, a["psi"], a["occ"], a["phi"], a["vx"], ex=a["ex"], gphi=a["gphi"])


@pytest.mark.parametrize("prec,cplx", [("fp64", False), ("fp32", False), ("bf16x6", False),
                                       ("fp64", True), ("fp32", True)])
@pytest.mark.parametrize("what,bad,match", [
    ("vx", lambda a: torch.zeros(a["vx"].shape, dtype=torch.float32), "vx: dtype"),
    ("vx", lambda a: a["vx"][:3], "vx: 3 rows"),
    ("occ", lambda a: a["occ"].to(torch.float32), "occ: dtype"),
    ("occ", lambda a: a["occ"][:2], "occ: a contiguous"),
    ("occ", lambda a: torch.ones(6, dtype=torch.float64)[::2], "occ: a contiguous"),
    ("gphi", lambda a: a["gphi"][:3], "gphi: a contiguous"),
    ("gphi", lambda a: a["gphi"].to(torch.float32), "gphi: dtype"),
    ("ex", lambda a: a["ex"].to(torch.float32), "ex: dtype"),
    ("ex", lambda a: torch.zeros(0, dtype=torch.float64), "ex: a contiguous"),
    ("psi", lambda a: torch.zeros(a["psi"].shape,
                                  dtype=torch.complex64 if not a["psi"].is_complex() else torch.float32),
     "psi: dtype"),
    ("phi", lambda a: a["phi"][:, : N - 1], "phi: expected"),
])
def test_exx_apply_refuses_misfit_tensors(prec, cplx, what, bad, match):
    plan = _plan(prec, cplx)
    a = _good(plan)
    a[what] = bad(a)
    with pytest.raises(ValueError, match=match):
        _exx(plan, a)


def test_exx_apply_refuses_host_tensors():
    plan = _plan()
    with pytest.raises(ValueError, match="must be a GPU tensor"):
        _exx(plan, _good(plan))


def test_ex_needs_gphi():
    plan = _plan()
    a = _good(plan)
    a["gphi"] = None
    with pytest.raises(ValueError, match="gphi|GPU"):
        _exx(plan, a)


def test_batched_and_autotune_check_every_task():
    plan = _plan("fp32")
    a = _good(plan)
    bad = dict(a, plan=plan, occ=a["occ"].to(torch.float32))
    with pytest.raises(ValueError, match="occ: dtype"):
        kronx.exx_apply_batched([bad])
    with pytest.raises(ValueError, match="psi: dtype"):
        kronx.kx_autotune(plan, a["psi"].double(), a["occ"], a["phi"])


def test_kron_solve_checks_element_type_and_rows():
    plan = _plan("fp32")
    B = torch.zeros((3, N), dtype=torch.float32)
    with pytest.raises(ValueError, match="X: dtype"):
        kronx.kron_solve(plan, B, torch.zeros((3, N), dtype=torch.float64))
    with pytest.raises(ValueError, match="X: 2 rows"):
        kronx.kron_solve(plan, B, torch.zeros((2, N), dtype=torch.float32))
    with pytest.raises(ValueError, match="B: dtype"):
        kronx.kron_solve(plan, B.double())


def test_ace_wrappers_check_dtypes_and_work():
    psi = torch.zeros((4, N), dtype=torch.float64)
    with pytest.raises(ValueError, match="psi: expected a float64"):
        kronx.ace_construct(psi.float(), psi.float(), 0.1)
    with pytest.raises(ValueError, match="w: dtype"):
        kronx.ace_construct(psi, psi.to(torch.complex128), 0.1)
    with pytest.raises(ValueError, match="work: "):
        kronx.ace_construct(psi, psi, 0.1, work=torch.zeros(4, dtype=torch.float64))
    with pytest.raises(ValueError, match="vphi: 2 rows"):
        kronx.ace_apply(psi, psi, 0.1, psi[:2])

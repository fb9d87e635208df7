"""Batched exchange (exx_apply_batched): the work-queue form (one persistent
launch per call) and the grouped-round form (KX_BATCHED=rounds; split-BF16
plans always).

Both forms run the pass bodies of the single-batch kernels item by item, so
the batched results are compared with per-task exx_apply calls (FP64 to 1e-14
relative, FP32 / split-BF16 to 1e-6 of the FP64 scale) and with the FP64
oracle (1e-12 / 1e-6 on Vx, E_x relative 1e-12 or 1e-6 Ha per nominal atom).
The schedule shape (rounds, batches, launches, widest launch) is checked
through kx_batched_schedule so that the form that ran is known.  The queue's
bounded waits are checked by a tiny poll budget set from the host
(KX_QUEUE_SPIN): the launch ends early and kx_batched_check reports it.
"""

import numpy as np
import pytest

from oracle.exx import exchange_energy, vx_apply, vx_apply_kpoints
from oracle.kron import KronSolver
from paper_2501_16572_amd.workloads import fermi_occupations, random_orbitals

from gpu_util import rel_fro, say, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BCP = ("periodic",) * 3


@pytest.fixture(scope="module")
def kx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_16572_amd import kronx
    kronx.load_library()
    return kronx


def _eager(kx, task):
    vx = torch.zeros_like(task["vx"])
    ex = torch.zeros(1, dtype=torch.float64, device="cuda")
    kx.exx_apply(task["plan"], task["psi"], task["occ"], task["phi"], vx, ex=ex, gphi=task["gphi"])
    return vx, ex


def _rel(a, b):
    return float((a - b).norm() / max(float(b.norm()), 1e-300))


@pytest.mark.parametrize("form", ["queue", "rounds"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_kpoint_set_batched(kx, prec, form, monkeypatch):
    # 2 k-points x 2 q-points on one grid: four complex plans (one per k - q).
    # Tasks of one k write the same Vx, so the schedule has two rounds of two
    # batches: one queue launch for all of them, or per round one launch per
    # pass holding both batches.
    n, h = (16, 18, 14), (0.35, 0.35, 0.35)
    say("batched k-points", prec, form)
    monkeypatch.setenv("KX_BATCHED", form)
    L = [n[d] * h[d] for d in range(3)]
    kpts = [(2 * np.pi / L[0] * 0.25, 2 * np.pi / L[1] * 0.25, 0.0),
            (-2 * np.pi / L[0] * 0.25, 2 * np.pi / L[1] * 0.25, 0.0)]
    wk = [0.375, 0.625]
    psi = [random_orbitals(n, h, 5, seed=80 + i, kpt=k, decay=2.0) for i, k in enumerate(kpts)]
    g = [np.array([1.0, 0.85, 0.0, 0.0, 0.0]), np.array([1.0, 0.9, 0.45, 0.0, 0.0])]
    nocc = [2, 3]
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    if prec == "fp32":
        psi = [p.astype(np.complex64).astype(np.complex128) for p in psi]
    plans = []
    try:
        dev_psi = [to_dev(p, ct) for p in psi]
        vx = [torch.zeros((5, psi[0].shape[1]), dtype=torch.complex128, device="cuda") for _ in range(2)]
        ex = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(2)]
        tasks = []
        for ik in range(2):
            gphi = to_dev(g[ik] * wk[ik], torch.float64)
            for iq in range(2):
                kq = tuple(kpts[ik][d] - kpts[iq][d] for d in range(3))
                plan = kx.kron_setup(n, h, BCP, 12, 0.0, kq=kq, prec=prec, complex=True)
                plans.append(plan)
                occ = to_dev(wk[iq] * g[iq][:nocc[iq]], torch.float64)
                tasks.append(dict(plan=plan, psi=dev_psi[iq][:nocc[iq]], occ=occ, phi=dev_psi[ik], vx=vx[ik],
                                  ex=ex[ik], gphi=gphi))
        results = []
        for rep in range(2):
            for ik in range(2):
                vx[ik].zero_()
                ex[ik].zero_()
            kx.exx_apply_batched(tasks)
            torch.cuda.synchronize()
            results.append(([to_host(v) for v in vx], [float(to_host(e)[0]) for e in ex]))
        sched = kx.kx_batched_schedule()
        assert sched == ((2, 4, 1, 4) if form == "queue" else (2, 4, 6, 2)), sched
    finally:
        for p in plans:
            p.destroy()
    # replays are bitwise identical
    for ik in range(2):
        assert np.array_equal(results[0][0][ik], results[1][0][ik])
        assert results[0][1][ik] == results[1][1][ik]

    W = vx_apply_kpoints(psi, g, wk, kpts, lambda kq: KronSolver(n, h, BCP, 12, 0.0, kq))
    dV = float(np.prod(h))
    atoms = 2.0 * sum(wk[i] * g[i].sum() for i in range(2)) / 14.0
    out, exv = results[0]
    for ik in range(2):
        Eref = wk[ik] * exchange_energy(psi[ik], g[ik], W[ik], dV)
        if prec == "fp64":
            assert rel_fro(out[ik], W[ik]) < 1e-12, ik
            assert abs(exv[ik] - Eref) < 1e-12 * abs(Eref), (exv[ik], Eref)
        else:
            assert rel_fro(out[ik], W[ik]) < 1e-6, ik
            assert abs(exv[ik] - Eref) / atoms < 1e-6, (exv[ik], Eref)


# uneven Gamma systems: (grid, h, omega, bands, occupied, seed); the first two
# share the x1/x2 and x3 tile counts, the last two share the x1/x2 one
SYSTEMS = [((24, 24, 24), 0.3, 0.0, 6, 4, 91), ((22, 20, 24), 0.3, 0.106, 5, 4, 92),
           ((40, 36, 44), 0.28, 0.106, 4, 3, 93), ((36, 40, 30), 0.3, 0.0, 4, 3, 94)]


def _gamma_tasks(kx, prec, systems):
    dt = {"fp64": torch.float64}.get(prec, torch.float32)
    plans, tasks = [], []
    for n, h, omega, nb, no, seed in systems:
        psi = random_orbitals(n, (h,) * 3, nb, seed=seed)
        g = fermi_occupations(nb, no, 0.01, seed=seed)
        plan = kx.kron_setup(n, (h,) * 3, BCP, 12, omega, prec=prec)
        plans.append(plan)
        psid = to_dev(psi, dt)
        tasks.append(dict(plan=plan, psi=psid[:no], occ=to_dev(g[:no], torch.float64), phi=psid,
                          vx=torch.zeros(psid.shape, dtype=torch.float64, device="cuda"),
                          ex=torch.zeros(1, dtype=torch.float64, device="cuda"),
                          gphi=to_dev(g, torch.float64)))
    return plans, tasks


def _oracle_systems(prec, systems):
    """Vx and E_x of each system from the FP64 oracle, on the inputs as the
    device holds them (rounded to FP32 for the mixed-precision plans)."""
    out = []
    for n, h, omega, nb, no, seed in systems:
        psi = random_orbitals(n, (h,) * 3, nb, seed=seed)
        if prec != "fp64":
            psi = psi.astype(np.float32).astype(np.float64)
        g = fermi_occupations(nb, no, 0.01, seed=seed)
        S = KronSolver(n, (h,) * 3, BCP, 12, omega)
        W = vx_apply(psi[:no], g[:no], psi, S)
        out.append((W, exchange_energy(psi, g, W, S.dV), 2.0 * g.sum() / 14.0))
    return out


@pytest.mark.parametrize("prec,form", [("fp64", "queue"), ("fp64", "rounds"), ("fp32", "queue"),
                                       ("fp32", "rounds"), ("bf16x6", "rounds")])
def test_uneven_systems_ragged_batches(kx, prec, form, monkeypatch):
    # a small workspace cuts every task into several batches of uneven size,
    # so rounds hold batches of different systems and ragged last batches;
    # every replay against the FP64 oracle (FP64 1e-12, mixed 1e-6 on Vx and
    # 1e-6 Ha per nominal atom on E_x) and against per-task exx_apply calls
    say("batched uneven systems", prec, form)
    monkeypatch.setenv("KX_WORKSPACE_MB", "1")
    monkeypatch.setenv("KX_BATCHED", form)
    plans, tasks = _gamma_tasks(kx, prec, SYSTEMS)
    ora = _oracle_systems(prec, SYSTEMS)
    try:
        ref = [_eager(kx, t) for t in tasks]
        for rep in range(2):
            for t in tasks:
                t["vx"].zero_()
                t["ex"].zero_()
            kx.exx_apply_batched(tasks)
            torch.cuda.synchronize()
            tol = 1e-14 if prec == "fp64" else 1e-6
            for i, (t, (vx_e, ex_e), (W, E, atoms)) in enumerate(zip(tasks, ref, ora)):
                assert _rel(t["vx"], vx_e) < tol, (rep, i, _rel(t["vx"], vx_e))
                assert abs(float(t["ex"][0] - ex_e[0])) <= tol * abs(float(ex_e[0])), (rep, i)
                err = rel_fro(to_host(t["vx"]), W)
                dE = abs(float(t["ex"][0]) - E)
                if prec == "fp64":
                    assert err < 1e-12 and dE < 1e-12 * abs(E), (rep, i, err, dE)
                else:
                    assert err < 1e-6 and dE / atoms < 1e-6, (rep, i, err, dE / atoms)
        rounds, batches, launches, widest = kx.kx_batched_schedule()
        assert batches > len(SYSTEMS) and rounds >= 2
        if form == "queue":
            assert launches == 1 and widest == batches, (rounds, batches, launches, widest)
        else:
            assert widest >= 2 and launches < 3 * batches, (rounds, batches, launches, widest)
    finally:
        for p in plans:
            p.destroy()


def test_shared_plan_and_oracle(kx, monkeypatch):
    # one plan used by two tasks (its bands split in two) next to a second
    # system: the two halves never share a round (one workspace), and the
    # result matches the FP64 oracle
    say("batched shared plan")
    monkeypatch.setenv("KX_WORKSPACE_MB", "2")
    n, h, omega, nb, no, seed = (24, 24, 24), 0.3, 0.106, 6, 4, 95
    psi = random_orbitals(n, (h,) * 3, nb, seed=seed)
    g = fermi_occupations(nb, no, 0.01, seed=seed)
    plans, tasks2 = _gamma_tasks(kx, "fp64", [SYSTEMS[1]])
    plan = kx.kron_setup(n, (h,) * 3, BCP, 12, omega, prec="fp64")
    plans.append(plan)
    try:
        psid = to_dev(psi, torch.float64)
        occ = to_dev(g[:no], torch.float64)
        vx = torch.zeros_like(psid)
        ex = torch.zeros(1, dtype=torch.float64, device="cuda")
        gphi = to_dev(g, torch.float64)
        tasks = [dict(plan=plan, psi=psid[:no], occ=occ, phi=psid[:3], vx=vx[:3], ex=ex, gphi=gphi[:3]),
                 tasks2[0],
                 dict(plan=plan, psi=psid[:no], occ=occ, phi=psid[3:], vx=vx[3:], ex=ex, gphi=gphi[3:])]
        kx.exx_apply_batched(tasks)
        torch.cuda.synchronize()
        rounds, batches, launches, widest = kx.kx_batched_schedule()
        assert rounds >= 2 and widest >= 2, (rounds, batches, launches, widest)
        S = KronSolver(n, (h,) * 3, BCP, 12, omega)
        from oracle.exx import exchange_energy, vx_apply
        W = vx_apply(psi[:no], g[:no], psi, S)
        assert rel_fro(to_host(vx), W) < 1e-12
        E = exchange_energy(psi, g, W, S.dV)
        assert abs(float(to_host(ex)[0]) - E) < 1e-12 * abs(E)
        vx_e, ex_e = _eager(kx, tasks2[0])
        assert _rel(tasks2[0]["vx"], vx_e) < 1e-14
    finally:
        for p in plans:
            p.destroy()


def test_workspace_bytes_and_balanced_batches(kx, monkeypatch):
    # 1 MiB of workspace holds 2 targets x 4 occupied of a 24^3 FP64 grid:
    # 5 targets run as 3 balanced batches of 2, and kx_workspace_bytes states
    # the buffers exx_apply then holds
    say("workspace bytes")
    monkeypatch.setenv("KX_WORKSPACE_MB", "1")
    n, h, nb, no = (24, 24, 24), (0.3,) * 3, 5, 4
    N = n[0] * n[1] * n[2]
    psi = random_orbitals(n, h, nb, seed=96)
    g = fermi_occupations(nb, no, 0.01, seed=96)
    plan = kx.kron_setup(n, h, BCP, 12, 0.106, prec="fp64")
    try:
        assert kx.kx_workspace_bytes(plan, 0, no) == 0
        wb = kx.kx_workspace_bytes(plan, nb, no)
        assert wb == 2 * no * N * 8 + 2 * 64 * 8, wb
        psid = to_dev(psi, torch.float64)
        vx = torch.zeros_like(psid)
        kx.exx_apply(plan, psid[:no], to_dev(g[:no], torch.float64), psid, vx)
        torch.cuda.synchronize()
        assert plan.info()[7] == 2
        S = KronSolver(n, h, BCP, 12, 0.106)
        from oracle.exx import vx_apply
        assert rel_fro(to_host(vx), vx_apply(psi[:no], g[:no], psi, S)) < 1e-12
    finally:
        plan.destroy()


def test_graph_cache_bounded_and_retuned(kx, tmp_path, monkeypatch):
    # fresh output tensors on every call make every task list new: the cache
    # stays at its capacity, and every call still matches the eager result;
    # an unchanged list replays without a capture, and retuning the plan makes
    # the next call capture again
    say("graph cache")
    monkeypatch.setenv("KX_TUNE_CACHE", str(tmp_path / "tune.txt"))
    n, h, nb, no = (24, 24, 24), (0.3,) * 3, 3, 2
    psi = random_orbitals(n, h, nb, seed=98)
    g = fermi_occupations(nb, no, 0.01, seed=98)
    plan = kx.kron_setup(n, h, BCP, 12, 0.106, prec="fp64")
    try:
        psid = to_dev(psi, torch.float64)
        occ = to_dev(g[:no], torch.float64)
        vx_e = torch.zeros_like(psid)
        kx.exx_apply(plan, psid[:no], occ, psid, vx_e)
        torch.cuda.synchronize()
        held, cap, cap0 = kx.kx_graph_cache_info()
        outs = []
        for i in range(cap + 4):
            vx = torch.zeros_like(psid)
            outs.append(vx)
            kx.exx_apply_batched([dict(plan=plan, psi=psid[:no], occ=occ, phi=psid, vx=vx)])
            torch.cuda.synchronize()
            assert torch.equal(vx, vx_e), i
            held, cap_i, caps = kx.kx_graph_cache_info()
            assert cap_i == cap and held <= cap, (held, cap)
            assert caps == cap0 + i + 1
        assert held == cap
        task = [dict(plan=plan, psi=psid[:no], occ=occ, phi=psid, vx=outs[-1])]
        outs[-1].zero_()
        kx.exx_apply_batched(task)
        torch.cuda.synchronize()
        assert kx.kx_graph_cache_info()[2] == caps          # replayed
        assert torch.equal(outs[-1], vx_e)
        kx.kx_autotune(plan, psid[:no], occ, psid)
        outs[-1].zero_()
        kx.exx_apply_batched(task)
        torch.cuda.synchronize()
        assert kx.kx_graph_cache_info()[2] == caps + 1      # captured again
        assert rel_fro(to_host(outs[-1]), to_host(vx_e)) < 1e-13
    finally:
        plan.destroy()


def test_queue_matches_rounds_and_shares_plans(kx, monkeypatch):
    # one list through both forms: two Gamma systems, one of them split over
    # two tasks of one plan (its halves never overlap in the queue), small
    # workspace for several batches each; FP64 results of the two forms agree
    # to 1e-14 and both match the oracle
    say("queue vs rounds")
    monkeypatch.setenv("KX_WORKSPACE_MB", "1")
    systems = [SYSTEMS[0], SYSTEMS[2]]
    plans, tasks = _gamma_tasks(kx, "fp64", systems)
    ora = _oracle_systems("fp64", systems)
    try:
        t0 = tasks[0]
        half = t0["phi"].shape[0] // 2
        split = [dict(t0, phi=t0["phi"][:half], vx=t0["vx"][:half], gphi=t0["gphi"][:half]),
                 tasks[1],
                 dict(t0, phi=t0["phi"][half:], vx=t0["vx"][half:], gphi=t0["gphi"][half:])]
        out = {}
        for form in ("queue", "rounds"):
            monkeypatch.setenv("KX_BATCHED", form)
            for t in tasks:
                t["vx"].zero_()
                t["ex"].zero_()
            kx.exx_apply_batched(split)
            kx.kx_batched_check()
            torch.cuda.synchronize()
            sched = kx.kx_batched_schedule()
            assert (sched[2] == 1) == (form == "queue"), (form, sched)
            out[form] = [(t["vx"].clone(), t["ex"].clone()) for t in tasks]
        for (vq, eq), (vr, er), (W, E, _) in zip(out["queue"], out["rounds"], ora):
            assert _rel(vq, vr) < 1e-14
            assert abs(float(eq[0] - er[0])) <= 1e-14 * abs(float(er[0]))
            assert rel_fro(to_host(vq), W) < 1e-12
            assert abs(float(eq[0]) - E) < 1e-12 * abs(E)
    finally:
        for p in plans:
            p.destroy()


def test_queue_bounded_wait_reports_and_recovers(kx, monkeypatch):
    # a poll budget of no retries (KX_QUEUE_SPIN=0, set from the host): one
    # batch whose pass A has a ticket per block, so the first block to take a
    # pass-B ticket finds the other blocks' pass-A tickets still running; its
    # wait gives up, the error flag ends every block at its next ticket, the
    # launch returns and kx_batched_check raises, on every replay (each
    # replay resets the counters and the flag).  A list captured with the
    # default budget then runs to the oracle's result.
    say("queue bounded wait")
    monkeypatch.setenv("KX_BATCHED", "queue")
    systems = [((50, 50, 50), 0.3, 0.106, 16, 12, 97)]
    monkeypatch.setenv("KX_QUEUE_SPIN", "0")
    plans, tasks = _gamma_tasks(kx, "fp64", systems)
    try:
        gave_up = 0
        for rep in range(3):
            kx.exx_apply_batched(tasks)
            try:
                kx.kx_batched_check()
            except kx.KronxError as e:
                assert "gave up" in str(e)
                gave_up += 1
        assert gave_up == 3
    finally:
        for p in plans:
            p.destroy()
    monkeypatch.delenv("KX_QUEUE_SPIN")
    ora = _oracle_systems("fp64", systems)
    plans, tasks = _gamma_tasks(kx, "fp64", systems)
    try:
        kx.exx_apply_batched(tasks)
        kx.kx_batched_check()
        torch.cuda.synchronize()
        assert kx.kx_batched_schedule()[2] == 1
        for t, (W, E, _) in zip(tasks, ora):
            assert rel_fro(to_host(t["vx"]), W) < 1e-12
            assert abs(float(t["ex"][0]) - E) < 1e-12 * abs(E)
    finally:
        for p in plans:
            p.destroy()

"""Host-side logic of bench.py (no GPU): the flop counts behind the roofline
and the rule that a committed traffic record counts only while the library
sources hash to the value it was taken on."""

import json
import os

import pytest

import bench


def test_pass_flops_sum_to_the_solver_count():
    # forward + inverse modes 1, 2 in passes A and C (2 N n_d each), both
    # mode-3 products in pass B: together 4 N (n1 + n2 + n3) per real solve
    n = (72, 80, 96)
    N = n[0] * n[1] * n[2]
    f = bench.pass_flops(n, 10)
    assert f["exx_fused_passA"] == f["exx_fused_passC"] == 2.0 * N * (n[0] + n[1]) * 10
    assert f["exx_fused_passB"] == 4.0 * N * n[2] * 10
    assert sum(f.values()) == 4.0 * N * sum(n) * 10


def test_sources_hash_is_stable():
    h = bench.kernel_sources_sha256()
    assert len(h) == 64 and h == bench.kernel_sources_sha256()


def _write_record(root, sha, bytes_):
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    rec = {"workload": "w", "form": "fp64:fused", "sources_sha256": sha,
           "kernels": {"fp64:fused/exx_fused_passC": {"hbm_bytes_per_launch": bytes_}}}
    with open(os.path.join(root, "profiles", "traffic_w.json"), "w") as f:
        json.dump(rec, f)


def test_traffic_counts_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    sha = bench.kernel_sources_sha256()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # kernel_sources_sha256 reads ROOT too: pin it to the real sources' hash
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: sha)
    assert bench.measured_traffic("w", "fp64:fused", "exx_fused_passC") is None  # no record
    _write_record(str(tmp_path), sha, 1.5e11)
    assert bench.measured_traffic("w", "fp64:fused", "exx_fused_passC") == pytest.approx(1.5e11)
    assert bench.measured_traffic("w", "fp64:fused", "exx_fused_passA") is None  # other kernel
    _write_record(str(tmp_path), "0" * 64, 1.5e11)  # sources changed since
    assert bench.measured_traffic("w", "fp64:fused", "exx_fused_passC") is None


def test_committed_traffic_records_name_their_commands():
    for wl in ("hse120", "hse72", "batch5"):
        path = os.path.join(bench.ROOT, "profiles", f"traffic_{wl}.json")
        with open(path) as f:
            rec = json.load(f)
        assert rec["workload"] == wl
        assert "rocprofv3 --pmc FETCH_SIZE" in rec["command"]
        assert rec["fetch_scale"] > 0 and rec["write_scale"] > 0
        for k in rec["kernels"].values():
            assert k["hbm_bytes_per_launch"] == pytest.approx(k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"])

"""The plan's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).

plan_host.cpp (FD weights, 1D eigenpairs for every boundary condition and
Bloch vector, the f table) is compiled with g++ for the host with both
sanitizers and driven over the edge cases of its inputs (axis lengths 1 ... 160,
orders 2, 12, 16, Bloch vectors, Dirichlet); any invalid access, overflow or
undefined operation aborts the run with a report.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_16572_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_plan_host_clean_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "plan_host_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", CSRC, os.path.join(CSRC, "plan_host.cpp"),
           os.path.join(ROOT, "tests", "host", "plan_host_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    # the environment may preload a library of its own ahead of the ASan
    # runtime; that does not change what ASan instruments in this program
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_queue_tickets_order_and_dependencies(tmp_path):
    # The batched work queue's ticket order and dependency counters
    # (queue_plan.h) on random task lists: every wait is on earlier tickets,
    # simulated runs with random block counts and timings always finish, and
    # the orders the passes, workspaces, outputs and E_x need hold in each run.
    exe = str(tmp_path / "queue_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", CSRC, os.path.join(ROOT, "tests", "host", "queue_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "OK" in r.stdout

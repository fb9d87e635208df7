"""Shared helpers for the GPU parity tests (inputs come from the workload
generators; expected values from the oracle only)."""

import sys

import numpy as np


def say(*a):
    """Name the case before each GPU step, flushed, so a failing run shows it."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel_fro(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.linalg.norm((x - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def to_dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def to_host(t):
    return t.detach().cpu().numpy()

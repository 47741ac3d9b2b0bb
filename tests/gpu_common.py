"""Shared helpers of the GPU parity tests (inputs come from `workloads`,
expected values from `oracle`; the HIP path is reached through the C ABI)."""
import sys

import numpy as np


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def to_dev(x, device=0):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to(f"cuda:{device}")


def to_host(t):
    return t.detach().cpu().numpy()


def rel_err(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    scale = max(np.abs(ref).max(), 1e-300)
    return float(np.abs(got - ref).max() / scale)

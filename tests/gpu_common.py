"""Shared helpers of the GPU parity tests: device upload of inputs and oracle runs."""
import sys

import numpy as np


def say(*a):
    """Print and flush the case name before a GPU step (so a fault names its case)."""
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / den)

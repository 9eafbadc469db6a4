"""Helpers shared by the GPU tests (device transfer, relative errors)."""
import sys

import numpy as np


def dev(x, dtype=None):
    import torch
    dtype = dtype or torch.float64
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def say(*args):
    """Flushed progress line naming the case before GPU work starts."""
    print(*args, file=sys.stderr, flush=True)

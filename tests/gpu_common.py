"""Shared helpers of the GPU parity tests."""
import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def context(dims, eps, seed, kappa, unit=False):
    import torch  # noqa: F401
    from paper_1903_06986_amd import Context
    from synth import random_su3_links, unit_links
    U = unit_links(dims) if unit else random_su3_links(dims, eps, seed)
    return Context(dims, U, kappa), U


def to_gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*args):
    """Print and flush a line naming the case before a GPU step."""
    print(*args, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))

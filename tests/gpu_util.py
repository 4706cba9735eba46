"""Helpers shared by the GPU tests (device transfers only)."""
import sys

import numpy as np


def cuda(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()

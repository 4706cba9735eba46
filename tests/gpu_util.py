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


def parity_error(p, got, ref):
    """Error of a solution against the oracle's for the parity tests: the
    larger of the relative 2-norm error and the relative max-norm error
    max|g(got) - g(ref)| / max|g(ref)| (g: gauge normalisation for singular
    problems), so a test bounds both the error as a whole and at every
    unknown."""
    import oracle as O
    return max(O.relative_error(p, got, ref), O.relative_error(p, got, ref, norm="max"))

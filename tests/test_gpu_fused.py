"""Fused x fast transform + y GEMM of FP64 solves (opt-in: the x transform
applied in the y GEMM's operand loads): solves against the CPU oracle and
against the separate passes of the same problem, several right-hand sides,
unaligned fields (which take the separate passes), and which plans fuse."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import cuda, host, say, parity_error

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def _T():
    import paper_2603_09528_amd as T
    return T


def _prob(nx, ny, nz, bcx, kind="poisson", loc=("C", "C", "C"), bcz=W.NN):
    # x uniform (fast transform), y and z stretched (y by GEMM)
    return W.make_problem((nx, ny, nz), (0.0, 2.0, 1.5), (bcx, W.NN, bcz), loc=loc, kind=kind,
                          alpha=1e-3 if kind == "helmholtz" else 0.0)


# (nx, ny, nz, bc x, kind, expected x transform): both row lengths, the three
# x transforms, two y tile rows, Poisson (pinned null line) and Helmholtz
CASES = [
    (128, 128, 3, W.PP, "poisson", "fft"),
    (256, 128, 2, W.PP, "helmholtz", "fft"),
    (128, 256, 2, W.NN, "poisson", "dct"),
    (256, 128, 3, W.DD, "poisson", "dst"),
    (256, 256, 2, W.NN, "helmholtz", "dct"),
    (128, 128, 4, W.DD, "helmholtz", "dst"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}-{c[5]}-{c[4]}")
def test_fused_matches_oracle_and_separate(case):
    import torch
    T = _T()
    nx, ny, nz, bcx, kind, xf = case
    p = _prob(nx, ny, nz, bcx, kind)
    f = W.rhs(p, 51)
    say("fused", p.n, xf, kind)
    plan = T.Plan.from_problem(p, fuse_xy=True)
    assert plan.fused and plan.transforms == (xf, "gemm")
    got = host(plan.solve(cuda(f)))
    sep = T.Plan.from_problem(p)
    assert not sep.fused
    ref_sep = host(sep.solve(cuda(f)))
    torch.cuda.synchronize()
    err = parity_error(p, got, O.solve(p, f))
    d = float(np.linalg.norm(got - ref_sep) / np.linalg.norm(ref_sep))
    say("  err vs oracle", err, "vs separate", d)
    assert err <= FP64_TOL, err
    assert d <= 1e-13, d


def test_fused_several_rhs():
    import torch
    T = _T()
    p = _prob(256, 128, 3, W.PP)
    fs = np.stack([W.rhs(p, 52), W.rhs(p, 53)])
    plan = T.Plan.from_problem(p, nrhs=2, fuse_xy=True)
    assert plan.fused
    got = host(plan.solve(cuda(fs)))
    torch.cuda.synchronize()
    for r in range(2):
        err = parity_error(p, got[r], O.solve(p, fs[r]))
        assert err <= FP64_TOL, (r, err)


def test_fused_unaligned_fields_take_separate_passes():
    """rhs and out 8 bytes off a 16-byte boundary: same result as aligned."""
    import torch
    T = _T()
    p = _prob(128, 128, 3, W.PP)
    f = W.rhs(p, 54)
    plan = T.Plan.from_problem(p, fuse_xy=True)
    aligned = host(plan.solve(cuda(f)))
    n = f.size
    base_in = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    base_out = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    rin = base_in[1:].view(f.shape)
    rin.copy_(cuda(f))
    rout = base_out[1:].view(f.shape)
    assert rin.data_ptr() % 16 == 8 and rout.data_ptr() % 16 == 8
    plan.solve(rin, rout)
    torch.cuda.synchronize()
    d = float(np.linalg.norm(host(rout) - aligned) / np.linalg.norm(aligned))
    assert d <= 1e-13, d


def test_which_plans_fuse():
    T = _T()
    ok = _prob(256, 128, 2, W.PP)
    F = dict(fuse_xy=True)
    assert T.Plan.from_problem(ok, **F).fused
    assert not T.Plan.from_problem(ok).fused                           # opt-in
    assert not T.Plan.from_problem(ok, precision="fp32", **F).fused
    assert not T.Plan.from_problem(ok, dense_x=True, **F).fused
    assert not T.Plan.from_problem(_prob(64, 128, 2, W.PP), **F).fused  # row length
    assert not T.Plan.from_problem(_prob(256, 96, 2, W.PP), **F).fused  # y tile rows
    uni_y = W.make_problem((256, 128, 2), (0.0, 0.0, 1.5), (W.PP, W.NN, W.NN))
    assert T.Plan.from_problem(uni_y, **F).transforms[1] != "gemm"
    assert not T.Plan.from_problem(uni_y, **F).fused                   # y by fast transform
    assert not T.Plan.from_problem(ok, host_only=True, **F).fused

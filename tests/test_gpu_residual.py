"""The FP64 residual of the refinement (r = f - A x, §2.2.2 operator, §4.1),
through tpt_residual, element by element against the oracle's residual.

Both kernel forms are covered: the paired-column form (even Nx, 16-byte
aligned x and f) and the scalar form (odd Nx, or x one element off a 16-byte
boundary).  Bound per element: the FP32 store rounds to within half an FP32
ulp, and the FP64 sums, formed in another order, can move the value across
one FP32 rounding boundary: |r - r_oracle| <= 2^-23 |r_oracle| + 16 eps64
(|f| + |A| |x|), with |A| |x| the operator of absolute coefficients applied
to |x|."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.operator import _apply_1d, _ops, implicit_dirs
from tests.gpu_util import cuda, host, say

pytestmark = pytest.mark.gpu

CASES = [
    # n, beta, bc, loc, kind, alpha, implicit
    ((48, 40, 36), (0.0, 2.0, 1.5), (W.PP, W.NN, W.NN), ("C", "C", "C"), "poisson", 0.0, "xyz"),
    ((37, 29, 23), (1.5, 2.0, 1.0), (W.DD, W.NN, W.DD), ("C", "C", "C"), "poisson", 0.0, "xyz"),
    ((32, 24, 20), (1.0, 0.0, 0.0), (W.NN, W.PP, W.PP), ("C", "C", "C"), "poisson", 0.0, "xyz"),
    ((64, 48, 40), (0.0, 2.0, 2.0), (W.PP, W.DD, W.DD), ("F", "C", "F"), "helmholtz", 2e-3, "xyz"),
    ((40, 36, 30), (1.0, 1.5, 2.0), (W.NN, W.NN, W.NN), ("C", "C", "C"), "helmholtz", 2e-3, "yz"),
    ((40, 36, 30), (1.0, 1.5, 2.0), (W.NN, W.NN, W.NN), ("C", "C", "C"), "helmholtz", 2e-3, "z"),
    ((34, 30, 33), (2.0, 1.0, 2.5), (("N", "D"), W.DD, W.NN), ("C", "F", "C"), "poisson", 0.0, "xyz"),
    ((2, 3, 5), (0.0, 1.0, 1.0), (W.NN, W.NN, W.NN), ("C", "C", "C"), "poisson", 0.0, "xyz"),
    ((600, 2, 3), (1.0, 0.0, 0.0), (W.PP, W.PP, W.NN), ("C", "C", "C"), "poisson", 0.0, "xyz"),
]


def _problem(c):
    n, beta, bc, loc, kind, alpha, implicit = c
    return W.make_problem(n, beta, bc, loc=loc, kind=kind, alpha=alpha, implicit=implicit)


def _abs_apply(p, x):
    """|A| |x|: the operator with absolute coefficients on |x|."""
    ax = np.abs(x)
    lap = np.zeros_like(ax)
    ops = _ops(p)
    for d, axis in ((0, 2), (1, 1), (2, 0)):
        if d not in implicit_dirs(p):
            continue
        a, b, c, _, per = ops[d]
        lap += _apply_1d(ax, np.abs(a), np.abs(b), np.abs(c), per, axis)
    return ax + abs(p.alpha) * lap if p.kind == "helmholtz" else lap


def _check(p, x, f, got):
    ref = O.residual(p, f, x)
    bound = 2.0 ** -23 * np.abs(ref) + 16 * np.finfo(float).eps * (np.abs(f) + _abs_apply(p, x))
    err = np.abs(got.astype(np.float64) - ref)
    assert (err <= bound).all(), float((err / bound).max())


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"{c[0][0]}x{c[0][1]}x{c[0][2]}-{c[4][0]}{c[6]}")
def test_residual_matches_oracle(c):
    import torch
    T = pytest.importorskip("paper_2603_09528_amd")
    p = _problem(c)
    plan = T.Plan.from_problem(p)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(p.shape)
    f = W.rhs(p, 12)
    say("residual", p.n, p.bc, p.loc, p.kind, getattr(p, "implicit", "xyz"))
    got = host(plan.residual(cuda(x), cuda(f)))
    torch.cuda.synchronize()
    _check(p, x, f, got)
    # x one element off a 16-byte boundary: the scalar form
    buf = torch.zeros(x.size + 1, dtype=torch.float64, device="cuda")
    xm = buf[1:].view(p.shape)
    xm.copy_(cuda(x))
    assert xm.data_ptr() % 16 == 8
    got2 = host(plan.residual(xm, cuda(f)))
    _check(p, x, f, got2)
    # the two forms round the same FP64 sums to FP32: at most one FP32 ulp apart
    assert (np.abs(got2.astype(np.float64) - got) <= 2.0 ** -23 * np.abs(got.astype(np.float64)) + 1e-30
            + 16 * np.finfo(float).eps * (np.abs(f) + _abs_apply(p, x))).all()


def test_residual_of_fp64_solution_is_roundoff():
    """§4.1: the residual of an FP64 solve sits at round-off of the operator
    applied to the solution."""
    import torch
    T = pytest.importorskip("paper_2603_09528_amd")
    p = _problem(CASES[0])
    plan = T.Plan.from_problem(p)
    f = W.rhs(p, 13)
    fd = cuda(f)
    x = plan.solve(fd)
    r = host(plan.residual(x, fd)).astype(np.float64)
    torch.cuda.synchronize()
    scale = np.abs(f) + _abs_apply(p, host(x))
    assert (np.abs(r) <= 64 * np.finfo(float).eps * scale.max()).all()


def test_residual_nrhs_and_rejections():
    import torch
    T = pytest.importorskip("paper_2603_09528_amd")
    p = _problem(CASES[3])
    plan = T.Plan.from_problem(p, nrhs=2)
    rng = np.random.default_rng(14)
    xs = rng.standard_normal((2,) + p.shape)
    fs = np.stack([W.rhs(p, 15), W.rhs(p, 16)])
    got = host(plan.residual(cuda(xs), cuda(fs)))
    torch.cuda.synchronize()
    for q in range(2):
        _check(p, xs[q], fs[q], got[q])
    with pytest.raises(T.TptError) as ei:
        T._check(T.lib().tpt_residual(plan.handle, None, None, None, None))
    assert ei.value.code == -1

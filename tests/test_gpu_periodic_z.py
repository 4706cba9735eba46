"""Periodic z: cyclic Thomas lines (kernel level, against the oracle's dense
per-line solve) and whole solves with a periodic z against the oracle, in
FP64, in the refined mixed modes (the FP64 residual wraps around in z) and
inside batches."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import cuda, host, say, parity_error

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-10


def _T():
    import paper_2603_09528_amd as T
    return T


@pytest.mark.parametrize("nx,ny,nz,nsys", [(37, 5, 11, 1), (64, 4, 33, 2), (5, 3, 2, 1), (9, 2, 3, 1),
                                           (70, 3, 64, 1), (8, 8, 100, 1)])
@pytest.mark.parametrize("sigma,tau", [(0.0, 1.0), (1.0, -3e-3)])
def test_cyclic_thomas_matches_oracle(nx, ny, nz, nsys, sigma, tau):
    import torch
    T = _T()
    say("cyclic thomas", nx, ny, nz, nsys, sigma, tau)
    rng = np.random.default_rng(nx * 1000 + ny * 10 + nz)
    faces = np.cumsum(np.concatenate([[0.0], rng.uniform(0.5, 1.5, nz)]))
    az, bz, cz, _ = O.operator_1d(faces, W.PP, "C")
    lamx = -rng.uniform(0.5, 50.0, nx)
    lamy = -rng.uniform(0.5, 50.0, ny)
    f = rng.standard_normal((nsys, nz, ny, nx))
    lam = lamy[:, None] + lamx[None, :]
    ref = np.stack([O.solver.cyclic_lines(az, bz, cz, lam, sigma, tau, f[s]) for s in range(nsys)])
    x = torch.empty(f.shape, dtype=torch.float64, device="cuda")
    scratch = torch.empty((4,) + f.shape, dtype=torch.float64, device="cuda")
    T.thomas(nx, ny, nz, nsys, cuda(lamx), cuda(lamy), cuda(az), cuda(bz), cuda(cz), sigma, tau, -1,
             cuda(f), x, scratch, periodic_z=True)
    torch.cuda.synchronize()
    got = host(x)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    with pytest.raises(T.TptError):  # the partitioned kernels take non-cyclic lines only
        T.thomas(nx, ny, nz, nsys, cuda(lamx), cuda(lamy), cuda(az), cuda(bz), cuda(cz), sigma, tau, -1,
                 cuda(f), x, scratch, periodic_z=True, variant=5)


@pytest.mark.parametrize("nz", [2, 17, 40])
def test_cyclic_thomas_pinned_line_in_place(nz):
    import torch
    T = _T()
    nx, ny = 9, 4
    rng = np.random.default_rng(6 + nz)
    faces = np.cumsum(np.concatenate([[0.0], rng.uniform(0.5, 1.5, nz)]))
    az, bz, cz, vol = O.operator_1d(faces, W.PP, "C")
    lamx = -rng.uniform(1.0, 20.0, nx)
    lamy = -rng.uniform(1.0, 20.0, ny)
    lamx[3] = 0.0
    lamy[2] = 0.0
    f = rng.standard_normal((nz, ny, nx))
    f[:, 2, 3] -= (vol * f[:, 2, 3]).sum() / vol.sum()  # compatible singular line
    lam = lamy[:, None] + lamx[None, :]
    ref = O.solver.cyclic_lines(az, bz, cz, lam, 0.0, 1.0, f, pin=(2, 3))
    xf = cuda(f)
    scratch = torch.empty((4, nz, ny, nx), dtype=torch.float64, device="cuda")
    T.thomas(nx, ny, nz, 1, cuda(lamx), cuda(lamy), cuda(az), cuda(bz), cuda(cz), 0.0, 1.0, 3 + nx * 2,
             xf, xf, scratch, periodic_z=True)
    torch.cuda.synchronize()
    got = host(xf)
    assert got[-1, 2, 3] == 0.0
    assert np.isfinite(got).all()
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


CASES = [
    ((24, 20, 16), (1.5, 2.0, 0.0), (W.NN, W.NN, W.PP), ("C", "C", "C"), "poisson"),
    ((32, 16, 12), (0.0, 0.0, 0.0), (W.PP, W.PP, W.PP), ("C", "C", "C"), "poisson"),
    ((19, 32, 40), (2.0, 0.0, 0.0), (W.DD, W.PP, W.PP), ("C", "C", "F"), "helmholtz"),
    ((33, 17, 2), (1.0, 1.0, 0.0), (("N", "D"), W.NN, W.PP), ("C", "C", "C"), "poisson"),
    ((64, 48, 35), (0.0, 1.5, 0.0), (W.PP, W.DD, W.PP), ("C", "F", "C"), "helmholtz"),
]


def _prob(case):
    n, beta, bc, loc, kind = case
    return W.make_problem(n, beta, bc, loc=loc, kind=kind, alpha=1e-3 if kind == "helmholtz" else 0.0)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0][0]}x{c[0][1]}x{c[0][2]}-{c[4]}")
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_periodic_z_solve_matches_oracle(case, prec):
    import torch
    T = _T()
    p = _prob(case)
    f = W.rhs(p, 91)
    say("periodic z", prec, p.n, p.bc, p.loc, p.kind)
    kw = {} if prec == "fp64" else dict(precision=prec, rtol=1e-13, max_refine=12)
    plan = T.Plan.from_problem(p, **kw)
    got = host(plan.solve(cuda(f)))
    torch.cuda.synchronize()
    err = parity_error(p, got, O.solve(p, f))
    say("  err", err, "iters", plan.info().iters)
    assert err <= (FP64_TOL if prec == "fp64" else MIXED_TOL), err


def test_periodic_z_in_batch():
    import torch
    T = _T()
    probs = [_prob(c) for c in CASES] + [W.make_problem((20, 18, 16), (1.0, 1.0, 1.0), (W.NN, W.DD, W.NN))]
    plans = [T.Plan.from_problem(p) for p in probs]
    fs = [W.rhs(p, 95 + i) for i, p in enumerate(probs)]
    rhs = [cuda(f) for f in fs]
    outs = [torch.empty_like(r) for r in rhs]
    batch = T.Batch(plans)
    for use_graph in (False, True):
        for o in outs:
            o.zero_()
        batch.solve(rhs, outs, use_graph=use_graph)
        torch.cuda.synchronize()
        for i, p in enumerate(probs):
            single = host(plans[i].solve(rhs[i]))
            assert np.array_equal(host(outs[i]), single), (i, use_graph)
            assert parity_error(p, single, O.solve(p, fs[i])) <= FP64_TOL, i

"""Fast transforms of uniform directions (real Fourier, DCT-II, DST-II along x
and along y, power-of-two N): solves through them against the CPU oracle,
against the dense-GEMM passes of the same plan, inside batches next to GEMM
plans, and the selection rule itself."""
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


def _prob(nx, ny, nz, kind="poisson", loc=("C", "C", "C"), bcy=W.NN, bcz=W.NN, beta=(0.0, 2.0, 1.5)):
    return W.make_problem((nx, ny, nz), beta, (W.PP, bcy, bcz), loc=loc, kind=kind,
                          alpha=1e-3 if kind == "helmholtz" else 0.0)


def _stretched_x(p, beta=1.2):
    """p with its periodic x faces tanh-stretched (a non-uniform periodic
    direction: dense cyclic eigenbasis, no fast transform)."""
    import dataclasses
    return dataclasses.replace(p, faces=(W.tanh_faces(p.n[0], beta, 1.0),) + tuple(p.faces[1:]))


def _solve(p, f, **kw):
    import torch
    T = _T()
    plan = T.Plan.from_problem(p, **kw)
    out = plan.solve(cuda(f))
    torch.cuda.synchronize()
    return host(out), plan


# (nx, ny, nz, kind, loc, bc y, bc z): every power-of-two block shape of the
# kernel (4, 2, 1 lines per block), odd line counts (ragged last block)
ORACLE_CASES = [
    (8, 5, 3, "poisson", ("C", "C", "C"), W.NN, W.NN),
    (16, 7, 9, "helmholtz", ("F", "C", "C"), W.DD, W.DD),
    (64, 13, 11, "poisson", ("C", "C", "C"), W.DD, W.NN),
    (128, 9, 7, "poisson", ("C", "C", "C"), W.NN, W.NN),
    (256, 11, 5, "helmholtz", ("C", "F", "C"), W.DD, W.DD),
    (512, 6, 5, "poisson", ("C", "C", "C"), W.NN, ("D", "N")),
]


@pytest.mark.parametrize("case", ORACLE_CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}-{c[3]}")
def test_fft_solve_matches_oracle(case):
    nx, ny, nz, kind, loc, bcy, bcz = case
    p = _prob(nx, ny, nz, kind, loc, bcy, bcz)
    f = W.rhs(p, 41)
    say("fft fp64", p.n, kind, loc)
    got, plan = _solve(p, f)
    assert plan.x_fft
    ref = O.solve(p, f)
    err = parity_error(p, got, ref)
    assert err <= FP64_TOL, err


@pytest.mark.parametrize("case", ORACLE_CASES[::2], ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}-{c[3]}")
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fft_mixed_matches_oracle(case, prec):
    nx, ny, nz, kind, loc, bcy, bcz = case
    p = _prob(nx, ny, nz, kind, loc, bcy, bcz)
    f = W.rhs(p, 42)
    say("fft mixed", prec, p.n)
    got, plan = _solve(p, f, precision=prec, rtol=1e-13, max_refine=12)
    assert plan.x_fft
    err = parity_error(p, got, O.solve(p, f))
    say("  iters", plan.info().iters, "err", err)
    assert err <= MIXED_TOL, err


def _norm_inf_bound(p):
    """Upper bound of ||A||_inf from the 1-D operators' absolute row sums."""
    from oracle.operator import operator_1d
    s = 0.0
    for d in range(3):
        a, b, c, _ = operator_1d(p.faces[d], p.bc[d], p.loc[d])
        s += float(np.max(np.abs(a) + np.abs(b) + np.abs(c)))
    return 1.0 + p.alpha * s if p.kind == "helmholtz" else s


@pytest.mark.parametrize("nx", [1024, 2048])
def test_fft_long_lines_match_dense_x(nx):
    # the oracle's eigensolver is slow at these N: compare with the dense x
    # pass of the same (analytic) basis, and bound the normwise backward
    # error ||r|| / (||A|| ||x|| + ||f||) of the FFT solve (inf-norms)
    p = _prob(nx, 6, 5, "helmholtz", bcy=W.DD, bcz=W.DD)
    f = W.rhs(p, 43)
    say("fft vs dense", p.n)
    a, pa = _solve(p, f)
    b, pb = _solve(p, f, dense_x=True)
    assert pa.x_fft and not pb.x_fft
    assert np.linalg.norm(a - b) / np.linalg.norm(b) <= FP64_TOL
    r = O.residual(p, f, a)
    eta = np.abs(r).max() / (_norm_inf_bound(p) * np.abs(a).max() + np.abs(f).max())
    say("  backward error", eta)
    assert eta <= 5e-14, eta


def test_fft_selection_rule():
    T = _T()
    assert T.Plan.from_problem(_prob(32, 4, 4)).x_fft
    assert not T.Plan.from_problem(_prob(32, 4, 4), dense_x=True).x_fft
    assert not T.Plan.from_problem(_prob(48, 4, 4)).x_fft          # not a power of two
    assert not T.Plan.from_problem(_prob(4, 4, 4)).x_fft           # below 8
    assert not T.Plan.from_problem(_prob(4096, 2, 2)).x_fft        # above 2048
    assert not T.Plan.from_problem(_stretched_x(_prob(32, 4, 4))).x_fft           # stretched
    q = W.make_problem((32, 4, 4), (1.0, 0.0, 0.0), (W.NN, W.PP, W.DD))
    assert T.Plan.from_problem(q).transforms == ("gemm", "gemm")     # stretched NN x; y below 8
    q = W.make_problem((32, 16, 4), (0.0, 0.0, 0.0), (("N", "D"), W.DD, W.DD))
    assert T.Plan.from_problem(q).transforms == ("gemm", "dst")      # mixed N/D x: no fast form
    assert T.Plan.from_problem(q, dense_y=True).transforms == ("gemm", "gemm")


def test_fft_nrhs_and_repeat():
    import torch
    T = _T()
    p = _prob(64, 10, 7, "helmholtz", bcy=W.DD, bcz=W.DD)
    fs = np.stack([W.rhs(p, 51), W.rhs(p, 52), W.rhs(p, 53)])
    plan3 = T.Plan.from_problem(p, nrhs=3)
    o3 = host(plan3.solve(cuda(fs)))
    o3b = host(plan3.solve(cuda(fs)))
    assert np.array_equal(o3, o3b)
    for i in range(3):
        assert parity_error(p, o3[i], O.solve(p, fs[i])) <= FP64_TOL
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec,fixed", [("fp64", -1), ("bf16x3", 4)])
def test_batch_mixing_fft_and_gemm_plans(prec, fixed):
    import torch
    T = _T()
    probs = [_prob(64, 9, 6), _prob(48, 7, 5), _prob(128, 5, 4, "poisson", bcy=W.DD),
             _stretched_x(_prob(64, 9, 6)), _prob(256, 3, 3, "helmholtz", bcy=W.DD, bcz=W.DD)]
    kw = dict(precision=prec, fixed_refine=fixed) if prec != "fp64" else {}
    plans = [T.Plan.from_problem(p, **kw) for p in probs]
    assert [pl.x_fft for pl in plans] == [True, False, True, False, True]
    fs = [W.rhs(p, 60 + i) for i, p in enumerate(probs)]
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
            err = parity_error(p, single, O.solve(p, fs[i]))
            assert err <= (FP64_TOL if prec == "fp64" else MIXED_TOL), (i, err)


# (cells, bc, loc, kind, beta, expected (x, y) transforms)
KIND_CASES = [
    ((64, 32, 9), (W.PP, W.NN, W.NN), ("C", "C", "C"), "poisson", (0, 0, 1.5), ("fft", "dct")),
    ((32, 64, 7), (W.NN, W.DD, W.DD), ("C", "C", "C"), "poisson", (0, 0, 1.5), ("dct", "dst")),
    ((16, 128, 5), (W.DD, W.PP, ("D", "N")), ("C", "C", "C"), "helmholtz", (0, 0, 2.0), ("dst", "fft")),
    ((128, 16, 6), (W.DD, W.NN, W.NN), ("C", "C", "C"), "helmholtz", (0, 0, 1.0), ("dst", "dct")),
    ((8, 256, 3), (W.NN, W.PP, W.DD), ("C", "C", "F"), "poisson", (0, 0, 1.0), ("dct", "fft")),
    ((32, 32, 8), (W.NN, W.NN, W.NN), ("C", "C", "C"), "poisson", (0, 0, 0.0), ("dct", "dct")),
    ((64, 16, 10), (W.PP, W.PP, W.NN), ("C", "C", "C"), "poisson", (0, 0, 2.5), ("fft", "fft")),
    ((48, 64, 5), (W.NN, W.NN, W.DD), ("C", "C", "C"), "poisson", (0, 0, 1.5), ("gemm", "dct")),
    ((64, 33, 5), (W.NN, W.DD, W.NN), ("C", "F", "C"), "helmholtz", (0, 0, 1.5), ("dct", "gemm")),
    ((512, 8, 4), (W.NN, W.DD, W.NN), ("C", "C", "C"), "poisson", (0, 0, 1.5), ("dct", "dst")),
    ((8, 512, 4), (W.DD, W.NN, W.NN), ("C", "C", "C"), "helmholtz", (0, 0, 1.5), ("dst", "dct")),
]


def _kind_problem(case):
    n, bc, loc, kind, beta, _ = case
    return W.make_problem(n, beta, bc, loc=loc, kind=kind, alpha=1e-3 if kind == "helmholtz" else 0.0)


def _kid(c):
    return f"{c[0][0]}x{c[0][1]}x{c[0][2]}-{c[5][0]}-{c[5][1]}"


@pytest.mark.parametrize("case", KIND_CASES, ids=_kid)
def test_transform_kinds_match_oracle(case):
    p = _kind_problem(case)
    f = W.rhs(p, 71)
    say("kinds fp64", p.n, p.bc, p.loc, case[5])
    got, plan = _solve(p, f)
    assert plan.transforms == case[5]
    ref = O.solve(p, f)
    err = parity_error(p, got, ref)
    assert err <= FP64_TOL, err


@pytest.mark.parametrize("case", KIND_CASES[:4], ids=_kid)
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_transform_kinds_mixed_match_oracle(case, prec):
    p = _kind_problem(case)
    f = W.rhs(p, 72)
    say("kinds mixed", prec, p.n, case[5])
    got, plan = _solve(p, f, precision=prec, rtol=1e-13, max_refine=12)
    assert plan.transforms == case[5]
    err = parity_error(p, got, O.solve(p, f))
    say("  iters", plan.info().iters, "err", err)
    assert err <= MIXED_TOL, err


@pytest.mark.parametrize("ny,bcy,want", [(1024, W.NN, "dct"), (2048, W.DD, "dst"), (1024, W.PP, "fft")])
def test_long_y_lines_match_dense_y(ny, bcy, want):
    p = W.make_problem((12, ny, 4), (0, 0, 1.5), (W.DD, bcy, W.DD), kind="helmholtz", alpha=1e-3)
    f = W.rhs(p, 73)
    say("y fast vs dense", p.n, want)
    a, pa = _solve(p, f)
    b, pb = _solve(p, f, dense_y=True)
    assert pa.transforms[1] == want and pb.transforms[1] == "gemm"
    assert np.linalg.norm(a - b) / np.linalg.norm(b) <= FP64_TOL
    r = O.residual(p, f, a)
    eta = np.abs(r).max() / (_norm_inf_bound(p) * np.abs(a).max() + np.abs(f).max())
    say("  backward error", eta)
    assert eta <= 5e-14, eta


@pytest.mark.parametrize("prec,fixed", [("fp64", -1), ("fp32", 3)])
def test_batch_mixing_all_transform_kinds(prec, fixed):
    import torch
    T = _T()
    probs = [_kind_problem(c) for c in KIND_CASES[:9]]
    kw = dict(precision=prec, fixed_refine=fixed) if prec != "fp64" else {}
    plans = [T.Plan.from_problem(p, **kw) for p in probs]
    assert [pl.transforms for pl in plans] == [c[5] for c in KIND_CASES[:9]]
    fs = [W.rhs(p, 80 + i) for i, p in enumerate(probs)]
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
            err = parity_error(p, single, O.solve(p, fs[i]))
            assert err <= (FP64_TOL if prec == "fp64" else MIXED_TOL), (i, err)

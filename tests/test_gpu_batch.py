"""Multi-problem batches on the GPU: one launch per stage (and tile variant)
for many uneven problems, eager and hipGraph-replayed, against the oracle and
bitwise against the single-problem path."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import cuda, host, say, parity_error

pytestmark = pytest.mark.gpu


def _T():
    import paper_2603_09528_amd as T
    return T


def _problems(count, lo, hi, seed):
    rng = np.random.default_rng(seed)
    return [(W.random_problem(rng, lo, hi), 100 + i) for i in range(count)]


@pytest.mark.parametrize("prec,fixed", [("fp64", -1), ("fp32", 4), ("bf16x3", 5)])
def test_batch_matches_single_and_oracle(prec, fixed):
    import torch
    T = _T()
    probs = _problems(7, 9, 40, seed=11)
    say("batch", prec, [p.n for p, _ in probs])
    plans = [T.Plan.from_problem(p, precision=prec, fixed_refine=fixed) for p, _ in probs]
    rhs = [cuda(W.rhs(p, s)) for p, s in probs]
    singles = [host(pl.solve(r)) for pl, r in zip(plans, rhs)]
    b = T.Batch(plans)
    outs = [torch.empty_like(r) for r in rhs]
    b.solve(rhs, outs, use_graph=False)
    torch.cuda.synchronize()
    eager = [host(o) for o in outs]
    for i, (p, s) in enumerate(probs):
        assert np.array_equal(eager[i], singles[i]), f"problem {i} differs from the single-problem path"
        ref = O.solve(p, W.rhs(p, s))
        tol = 1e-12 if prec == "fp64" else 1e-10
        assert parity_error(p, eager[i], ref) <= tol
    # graph capture, replayed with eager work and synchronisation in between
    for rep in range(3):
        for o in outs:
            o.zero_()
        b.solve(rhs, outs, use_graph=True)
        torch.cuda.synchronize()
        _ = (rhs[0] * 2.0).sum().item()
        for i in range(len(outs)):
            assert np.array_equal(host(outs[i]), singles[i]), f"graph replay {rep}, problem {i}"


@pytest.mark.parametrize("prec,fixed", [("fp64", -1), ("fp32", 2)])
def test_small_batch_of_interior_problems_matches_single(prec, fixed):
    """Up to four problems whose GEMMs take a persistent tile run one launch per
    problem instead of one work list; results stay bitwise those of the single
    solves."""
    import torch
    T = _T()
    probs = [(W.make_problem((128, 128, 12), (1.5, 2.0, 1.0), (W.NN, W.DD, W.NN)), 41),
             (W.make_problem((128, 256, 10), (2.0, 1.0, 1.5), (W.DD, W.NN, W.DD), kind="helmholtz", alpha=1e-3), 42),
             (W.make_problem((256, 128, 9), (1.0, 1.5, 2.0), (W.NN, W.NN, W.NN)), 43)]
    plans = [T.Plan.from_problem(p, precision=prec, fixed_refine=fixed, dense_x=True) for p, _ in probs]
    rhs = [cuda(W.rhs(p, s)) for p, s in probs]
    singles = [host(pl.solve(r)) for pl, r in zip(plans, rhs)]
    b = T.Batch(plans)
    outs = [torch.empty_like(r) for r in rhs]
    for use_graph in (False, True):
        b.solve(rhs, outs, use_graph=use_graph)
        torch.cuda.synchronize()
        for i, (p, s) in enumerate(probs):
            assert np.array_equal(host(outs[i]), singles[i]), (i, use_graph)
    for i, (p, s) in enumerate(probs):
        err = parity_error(p, singles[i], O.solve(p, W.rhs(p, s)))
        assert err <= (1e-12 if prec == "fp64" else 1e-10), (i, err)


def test_batch_rejects_mixed_precisions_and_nrhs():
    T = _T()
    (p, _), (q, _) = _problems(2, 8, 12, seed=3)
    with pytest.raises(T.TptError):
        T.Batch([T.Plan.from_problem(p), T.Plan.from_problem(q, precision="fp32", fixed_refine=2)])
    with pytest.raises(T.TptError):
        T.Batch([T.Plan.from_problem(p, nrhs=2)])
    with pytest.raises(T.TptError):
        T.Batch([T.Plan.from_problem(p, precision="fp32")])  # adaptive refinement


@pytest.mark.slow
def test_batch64_uneven_fp64_with_autotune():
    import torch
    T = _T()
    probs = W.batch64()
    say("batch64 plans")
    plans = [T.Plan.from_problem(p) for p, _ in probs]
    T.autotune(plans)
    rhs = [cuda(W.rhs(p, s)) for p, s in probs]
    outs = [torch.empty_like(r) for r in rhs]
    b = T.Batch(plans)
    b.solve(rhs, outs, use_graph=True)
    torch.cuda.synchronize()
    for i in range(0, 64, 9):
        p, s = probs[i]
        say("oracle", i, p.n, p.bc)
        ref = O.solve(p, W.rhs(p, s))
        assert parity_error(p, host(outs[i]), ref) <= 1e-12


@pytest.mark.slow
def test_batch64_uneven_fp32_matches_oracle():
    """The 64-problem batch in FP32-mixed mode (two corrections, one launch
    per stage from a graph): every eighth problem against the oracle at
    1e-10 (2-norm and max-norm)."""
    import torch
    T = _T()
    probs = W.batch64()
    plans = [T.Plan.from_problem(p, precision="fp32", fixed_refine=2) for p, _ in probs]
    rhs = [cuda(W.rhs(p, s)) for p, s in probs]
    outs = [torch.empty_like(r) for r in rhs]
    b = T.Batch(plans)
    b.solve(rhs, outs, use_graph=True)
    torch.cuda.synchronize()
    for i in range(3, 64, 8):
        p, s = probs[i]
        ref = O.solve(p, W.rhs(p, s))
        err = parity_error(p, host(outs[i]), ref)
        say("fp32 batch", i, p.n, p.bc, f"{err:.3e}")
        assert err <= 1e-10, (i, err)

"""Helmholtz plans with y and z implicit (yz: no x transforms) or z only (z:
the Thomas solve alone), §2.1 and §3, on the GPU against the oracle (FP64,
2-norm and max-norm at 1e-12), alone, in batches mixed with full (xyz)
plans and served."""
import time

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import cuda, host, say, parity_error

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12

CASES = [
    # n, beta, bc, loc
    ((37, 29, 23), (1.5, 2.0, 1.0), (W.DD, W.NN, W.DD), ("C", "C", "C")),
    ((48, 64, 17), (0.0, 0.0, 2.0), (W.PP, W.NN, W.DD), ("C", "C", "C")),       # y by DCT
    ((32, 128, 16), (0.0, 0.0, 2.0), (W.PP, W.DD, W.DD), ("F", "C", "F")),      # y by DST, staggered
    ((24, 20, 19), (2.0, 1.5, 0.0), (("N", "D"), W.DD, W.PP), ("C", "F", "C")), # periodic z (cyclic lines)
    ((64, 48, 300), (1.0, 1.5, 2.0), (W.NN, W.NN, W.NN), ("C", "C", "C")),      # long z lines
]


def _T():
    import paper_2603_09528_amd as T
    return T


def _problem(case, implicit, alpha=2e-3):
    n, beta, bc, loc = case
    return W.make_problem(n, beta, bc, loc=loc, kind="helmholtz", alpha=alpha, implicit=implicit)


@pytest.mark.parametrize("implicit", ["yz", "z"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0][0]}x{c[0][1]}x{c[0][2]}")
def test_implicit_matches_oracle(case, implicit):
    import torch
    T = _T()
    p = _problem(case, implicit)
    f = W.rhs(p, 21)
    plan = T.Plan.from_problem(p)
    tr = plan.transforms
    assert tr[0] == "none" and (tr[1] == "none") == (implicit == "z")
    say("implicit", implicit, p.n, p.bc, p.loc, tr)
    got = host(plan.solve(cuda(f)))
    torch.cuda.synchronize()
    err = parity_error(p, got, O.solve(p, f))
    assert err <= FP64_TOL, err
    inf = plan.info()
    assert inf.nonfinite == 0 and inf.compat_defect == 0.0 and inf.null_line == -1


@pytest.mark.parametrize("seq", [False, True])
def test_implicit_nrhs_and_sequential_thomas(seq):
    import torch
    T = _T()
    p = _problem(CASES[0], "yz")
    fs = np.stack([W.rhs(p, 30 + r) for r in range(3)])
    plan = T.Plan.from_problem(p, nrhs=3, seq_thomas=seq)
    got = host(plan.solve(cuda(fs)))
    torch.cuda.synchronize()
    for r in range(3):
        assert parity_error(p, got[r], O.solve(p, fs[r])) <= FP64_TOL, r


def test_batch_mixes_implicit_options():
    """One batch holding xyz, yz and z plans (FP64): each result bitwise the
    single solve's, and each against the oracle."""
    import torch
    T = _T()
    probs = [_problem(CASES[0], "xyz"), _problem(CASES[1], "yz"), _problem(CASES[3], "z"),
             _problem(CASES[2], "yz"), _problem(CASES[4], "z"),
             W.make_problem((40, 36, 30), (1.5, 2.0, 1.0), (W.NN, W.NN, W.NN))]
    plans = [T.Plan.from_problem(p) for p in probs]
    fs = [W.rhs(p, 50 + i) for i, p in enumerate(probs)]
    rhs = [cuda(f) for f in fs]
    singles = [host(pl.solve(r)) for pl, r in zip(plans, rhs)]
    b = T.Batch(plans)
    outs = [torch.empty_like(r) for r in rhs]
    for use_graph in (False, True):
        for o in outs:
            o.fill_(np.nan)
        b.solve(rhs, outs, use_graph=use_graph)
        torch.cuda.synchronize()
        for i in range(len(probs)):
            assert np.array_equal(host(outs[i]), singles[i]), (i, use_graph)
    for i, p in enumerate(probs):
        assert parity_error(p, singles[i], O.solve(p, fs[i])) <= FP64_TOL, i


def test_server_serves_implicit_options():
    import torch
    T = _T()
    probs = [_problem(CASES[0], "yz"), _problem(CASES[1], "z"), _problem(CASES[0], "xyz")]
    plans = [T.Plan.from_problem(p) for p in probs]
    rhs = [cuda(W.rhs(p, 60 + i)) for i, p in enumerate(probs)]
    outs = [torch.empty_like(r) for r in rhs]
    srv = T.Server(hbm_budget_bytes=0, max_slots=2)
    tickets = [srv.submit(pl, r, o) for pl, r, o in zip(plans, rhs, outs)]
    done = set()
    t0 = time.time()
    while len(done) < len(tickets) and time.time() - t0 < 60:
        for t in tickets:
            if t not in done and srv.poll(t) is not None:
                done.add(t)
        time.sleep(0.0005)
    srv.drain()
    del srv
    assert len(done) == len(tickets)
    for i, p in enumerate(probs):
        assert np.array_equal(host(outs[i]), host(plans[i].solve(rhs[i]))), i


def test_implicit_option_rejections():
    T = _T()
    pois = W.make_problem((16, 16, 16), (1.0, 1.0, 1.0), (W.NN, W.NN, W.NN))
    with pytest.raises(T.TptError) as ei:
        T.Plan.from_problem(pois, implicit="yz")
    assert ei.value.code == -1
    helm = _problem(CASES[0], "yz")
    for prec in ("fp32", "bf16x3"):
        with pytest.raises(T.TptError) as ei:
            T.Plan.from_problem(helm, precision=prec, fixed_refine=2)
        assert ei.value.code == -2

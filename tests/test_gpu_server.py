"""Serving loop on the GPU: continuous batching with memory admission.  Each
result is bitwise the same served in a mix as solved alone."""
import time

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import cuda, host, say, parity_error

pytestmark = pytest.mark.gpu


def _T():
    import paper_2603_09528_amd as T
    return T


def _wait(srv, tickets, timeout=60.0):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for t in tickets:
            if t in done:
                continue
            r = srv.poll(t)
            if r is not None:
                done[t] = r
        if time.time() - t0 > timeout:
            raise TimeoutError("requests did not finish")
        time.sleep(0.0005)
    return done


@pytest.mark.parametrize("prec,fixed", [("fp64", -1), ("bf16x3", 5)])
def test_server_mix_equals_alone(prec, fixed):
    import torch
    T = _T()
    fams = W.serving_families(seed=5, sizes=(16, 24, 32, 40, 48))
    plans = [T.Plan.from_problem(p, precision=prec, fixed_refine=fixed) for p in fams]
    reqs = []
    rng = np.random.default_rng(9)
    for k in range(20):
        i = int(rng.integers(len(fams)))
        reqs.append((i, 500 + k))
    rhs = [cuda(W.rhs(fams[i], s)) for i, s in reqs]
    alone = [host(plans[i].solve(r)) for (i, _), r in zip(reqs, rhs)]
    srv = T.Server(hbm_budget_bytes=0, max_slots=3)
    outs = [torch.empty_like(r) for r in rhs]
    tickets = [srv.submit(plans[i], r, o) for (i, _), r, o in zip(reqs, rhs, outs)]
    done = _wait(srv, tickets)
    srv.drain()
    for k, t in enumerate(tickets):
        info, ts, t0, t1 = done[t]
        assert ts <= t0 <= t1
        assert np.array_equal(host(outs[k]), alone[k]), f"request {k} differs from its solve alone"
    i, s = reqs[0]
    ref = O.solve(fams[i], W.rhs(fams[i], s))
    assert parity_error(fams[i], host(outs[0]), ref) <= (1e-12 if prec == "fp64" else 1e-10)
    del srv


def test_server_memory_admission_and_oversize_rejection():
    import torch
    T = _T()
    small = W.make_problem((20, 20, 20), (1.0, 1.0, 1.0), (W.NN, W.NN, W.NN))
    big = W.make_problem((64, 64, 64), (1.0, 1.0, 1.0), (W.DD, W.DD, W.DD))
    ps = T.Plan.from_problem(small)
    pb = T.Plan.from_problem(big)
    budget = int(ps.workspace_bytes() * 1.6) + 4096   # one small request at a time
    srv = T.Server(hbm_budget_bytes=budget, max_slots=4)
    rhs = [cuda(W.rhs(small, 40 + k)) for k in range(6)]
    outs = [torch.empty_like(r) for r in rhs]
    tickets = [srv.submit(ps, r, o) for r, o in zip(rhs, outs)]
    done = _wait(srv, tickets)
    # with room for one request, the admissions are serialised
    spans = sorted((done[t][2], done[t][3]) for t in tickets)
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert b0 >= a1 - 1e-3
    for k, o in enumerate(outs):
        assert np.array_equal(host(o), host(ps.solve(rhs[k])))
    rb = cuda(W.rhs(big, 1))
    ob = torch.empty_like(rb)
    t = srv.submit(pb, rb, ob)
    with pytest.raises(T.TptError) as ei:
        _wait(srv, [t])
    assert ei.value.code == -3
    del srv
    say("admission ok")


@pytest.mark.slow
@pytest.mark.parametrize("prec,fixed", [("fp64", -1), ("bf16x3", 3)])
def test_served_full_size_families_match_oracle(prec, fixed):
    """Requests of the 64^3, 256^3 and 512^3 serving families, served
    together, each against the oracle (FP64 at 1e-12, refined BF16x3 at
    1e-10, 2-norm and max-norm)."""
    import torch
    T = _T()
    fams = W.serving_families()
    pick = [fams[0], fams[5], fams[9]]
    assert [p.n[0] for p in pick] == [64, 256, 512]
    plans = [T.Plan.from_problem(p, precision=prec, fixed_refine=fixed) for p in pick]
    rhs = [cuda(W.rhs(p, 700 + k)) for k, p in enumerate(pick)]
    outs = [torch.empty_like(r) for r in rhs]
    srv = T.Server(hbm_budget_bytes=0, max_slots=3)
    tickets = [srv.submit(pl, r, o) for pl, r, o in zip(plans, rhs, outs)]
    done = _wait(srv, tickets, timeout=120.0)
    srv.drain()
    del srv
    for k, (p, t) in enumerate(zip(pick, tickets)):
        info = done[t][0]
        assert info.nonfinite == 0
        say("oracle", p.name, p.bc)
        ref = O.solve(p, W.rhs(p, 700 + k))
        err = parity_error(p, host(outs[k]), ref)
        say(f"  {prec}: {err:.3e}")
        assert err <= (1e-12 if prec == "fp64" else 1e-10), (p.name, err)

"""Right-hand-side checks of a solve (tpt_info.compat_defect, .nonfinite) on
the GPU, for single solves, batches and served requests.

compat_defect of a singular Poisson problem is |sum dV f| / sum dV |f|: the
left null vector of the operator is the control-volume field dV (§2.2.1, D T
symmetric), so sum dV f = 0 is the solvability condition and the pin of §3
absorbs whatever of f violates it.  The expected values are computed here
from the right-hand side and the control volumes of the workload generator."""
import time

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import cuda, host, say

pytestmark = pytest.mark.gpu


def _T():
    import paper_2603_09528_amd as T
    return T


def _defect(p, f):
    dv = p.volumes()
    return abs(float((dv * f).sum())) / float((dv * np.abs(f)).sum())


SINGULAR = W.make_problem((24, 20, 16), (1.5, 2.0, 1.0), (W.NN, W.NN, W.NN))
PERIODIC = W.make_problem((32, 16, 12), (0.0, 2.0, 1.5), (W.PP, W.NN, W.NN))
REGULAR = W.make_problem((20, 18, 14), (1.0, 1.5, 2.0), (W.DD, W.NN, ("N", "D")))
# x by FFT with whole blocks of x lines per right-hand side: the check rides
# in the loads of the x forward transform
PERIODIC_F = W.make_problem((64, 32, 16), (0.0, 2.0, 1.5), (W.PP, W.NN, W.NN))
REGULAR_F = W.make_problem((64, 32, 16), (0.0, 2.0, 1.5), (W.PP, W.NN, W.DD))
# long x lines (a block holds fewer threads than pairs per line)
PERIODIC_L1 = W.make_problem((1024, 8, 4), (0.0, 1.5, 1.0), (W.PP, W.NN, W.NN))
PERIODIC_L2 = W.make_problem((2048, 4, 3), (0.0, 1.5, 1.0), (W.PP, W.NN, W.NN))


@pytest.mark.parametrize("prec,fixed", [("fp64", -1), ("fp32", 2), ("bf16x3", -1)])
@pytest.mark.parametrize("p", [SINGULAR, PERIODIC, PERIODIC_F, PERIODIC_L1, PERIODIC_L2],
                         ids=["nnn", "pnn", "pnn-fused", "pnn-fused-1024", "pnn-fused-2048"])
def test_compat_defect_of_incompatible_rhs(p, prec, fixed):
    import torch
    T = _T()
    f = W.rhs(p, 3)                    # compatibility-projected
    g = f + 0.25                       # a constant breaks sum dV f = 0
    plan = T.Plan.from_problem(p, precision=prec, fixed_refine=fixed, rtol=1e-12)
    say("compat", p.bc, prec)
    plan.solve(cuda(f))
    torch.cuda.synchronize()
    inf = plan.info()
    assert inf.nonfinite == 0
    assert inf.compat_defect <= 1e-13, inf.compat_defect
    plan.solve(cuda(g))
    torch.cuda.synchronize()
    inf = plan.info()
    want = _defect(p, g)
    assert want > 1e-3
    assert abs(inf.compat_defect - want) <= 1e-12 * want + 1e-15, (inf.compat_defect, want)
    assert inf.null_line >= 0


@pytest.mark.parametrize("prec,fixed", [("fp64", -1), ("fp32", 1), ("bf16x3", 2)])
def test_regular_problem_reports_no_defect(prec, fixed):
    import torch
    T = _T()
    f = W.rhs(REGULAR, 4) + 1.0
    plan = T.Plan.from_problem(REGULAR, precision=prec, fixed_refine=fixed)
    plan.solve(cuda(f))
    torch.cuda.synchronize()
    inf = plan.info()
    assert inf.null_line == -1
    assert inf.compat_defect == 0.0 and inf.nonfinite == 0


@pytest.mark.parametrize("prec,fixed", [("fp64", -1), ("fp32", 2), ("bf16x3", 2)])
@pytest.mark.parametrize("p", [REGULAR, REGULAR_F], ids=["gemm-x", "fused"])
def test_nonfinite_rhs_is_counted(p, prec, fixed):
    import torch
    T = _T()
    f = W.rhs(p, 5)
    f[3, 4, 5] = np.nan
    f[0, 0, 0] = np.inf
    f[-1, -1, -1] = -np.inf
    plan = T.Plan.from_problem(p, precision=prec, fixed_refine=fixed)
    say("nonfinite", prec)
    plan.solve(cuda(f))
    torch.cuda.synchronize()
    assert plan.info().nonfinite == 3
    # the next finite solve clears it
    plan.solve(cuda(W.rhs(p, 6)))
    torch.cuda.synchronize()
    assert plan.info().nonfinite == 0


def test_nonfinite_rhs_stops_adaptive_refinement():
    import torch
    T = _T()
    f = W.rhs(REGULAR, 7)
    f[1, 2, 3] = np.nan
    plan = T.Plan.from_problem(REGULAR, precision="fp32")
    with pytest.raises(T.TptError) as ei:
        plan.solve(cuda(f))
    torch.cuda.synchronize()
    assert ei.value.code == -5 and "non-finite" in str(ei.value)
    assert plan.info().nonfinite == 1


@pytest.mark.parametrize("p", [SINGULAR, PERIODIC_F], ids=["gemm-x", "fused"])
def test_nrhs_checks_report_the_worst_rhs(p):
    import torch
    T = _T()
    fs = np.stack([W.rhs(p, 10), W.rhs(p, 11) + 0.1, W.rhs(p, 12)])
    fs[2, 1, 1, 1] = np.nan
    plan = T.Plan.from_problem(p, nrhs=3)
    plan.solve(cuda(fs))
    torch.cuda.synchronize()
    inf = plan.info()
    want = _defect(p, fs[1])
    assert abs(inf.compat_defect - want) <= 1e-12 * want
    assert inf.nonfinite == 1


def test_checks_off():
    import torch
    T = _T()
    f = W.rhs(SINGULAR, 13)
    f[0, 0, 1] = np.nan
    plan = T.Plan.from_problem(SINGULAR, check=False)
    plan.solve(cuda(f))
    torch.cuda.synchronize()
    inf = plan.info()
    assert inf.compat_defect == -1.0 and inf.nonfinite == -1


@pytest.mark.parametrize("prec,fixed", [("fp64", -1), ("fp32", 2)])
def test_batch_info(prec, fixed):
    import torch
    T = _T()
    probs = [SINGULAR, PERIODIC, REGULAR]
    fs = [W.rhs(SINGULAR, 20) + 0.5, W.rhs(PERIODIC, 21), W.rhs(REGULAR, 22)]
    fs[2][2, 2, 2] = np.inf
    plans = [T.Plan.from_problem(p, precision=prec, fixed_refine=fixed) for p in probs]
    b = T.Batch(plans)
    with pytest.raises(T.TptError):
        b.info(0)                      # not solved yet
    rhs = [cuda(f) for f in fs]
    outs = [torch.empty_like(r) for r in rhs]
    for use_graph in (False, True):
        b.solve(rhs, outs, use_graph=use_graph)
        torch.cuda.synchronize()
        i0, i1, i2 = b.info(0), b.info(1), b.info(2)
        assert abs(i0.compat_defect - _defect(SINGULAR, fs[0])) <= 1e-12 * _defect(SINGULAR, fs[0])
        assert i1.compat_defect <= 1e-13 and i1.nonfinite == 0
        assert i2.compat_defect == 0.0 and i2.nonfinite == 1
        assert i0.iters == (0 if prec == "fp64" else fixed)
        if prec != "fp64":
            # the last correction of a converged refinement is small
            assert 0.0 < i1.rel_correction <= 1e-8 and 0.0 < i1.rel_residual <= 1e-6
    with pytest.raises(T.TptError):
        b.info(3)


def test_server_info():
    import torch
    T = _T()
    plan = T.Plan.from_problem(SINGULAR)
    good, bad = W.rhs(SINGULAR, 30), W.rhs(SINGULAR, 31) + 1.0
    srv = T.Server(hbm_budget_bytes=0, max_slots=2)
    rg, rb = cuda(good), cuda(bad)
    og, ob = torch.empty_like(rg), torch.empty_like(rb)
    tg, tb = srv.submit(plan, rg, og), srv.submit(plan, rb, ob)
    done = {}
    t0 = time.time()
    while len(done) < 2 and time.time() - t0 < 60:
        for t in (tg, tb):
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        time.sleep(0.0005)
    assert len(done) == 2
    assert done[tg][0].compat_defect <= 1e-13
    want = _defect(SINGULAR, bad)
    assert abs(done[tb][0].compat_defect - want) <= 1e-12 * want
    assert done[tb][0].nonfinite == 0
    # the solve is unaffected by the check: bitwise the plan's own result
    assert np.array_equal(host(og), host(plan.solve(rg)))
    del srv


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_incompatible_rhs_solution_matches_oracle(prec):
    """The pin of §3 absorbs the incompatible part of f in every mode: the
    refined mixed solves reach the oracle's pinned solution too (their
    residuals drop that part, so the corrections converge to it)."""
    import torch
    import oracle as O
    from tests.gpu_util import parity_error
    T = _T()
    p = SINGULAR
    g = W.rhs(p, 40) + 0.3
    ref = O.solve(p, g)
    plan = T.Plan.from_problem(p, precision=prec, rtol=1e-13, max_refine=12)
    got = host(plan.solve(cuda(g)))
    torch.cuda.synchronize()
    err = parity_error(p, got, ref)
    say("incompatible", prec, err, plan.info().iters)
    assert err <= (1e-12 if prec == "fp64" else 1e-10), err

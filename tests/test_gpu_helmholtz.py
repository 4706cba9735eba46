"""The implicit-diffusion Helmholtz workload at full size on the GPU:
(I - alpha L) u = f, alpha = 1e-4, 1024 x 768 x 512 cells, x periodic uniform,
y and z Dirichlet walls with tanh beta = 2, the three staggered velocity
components (u on x-faces, v on y-faces, w on z-faces) solved as one batch of
three plans, in FP64 and with split-BF16x3 transforms and FP64 refinement.

Every component is compared element by element with the oracle's solution
at 1024 seeded positions per field (corners included), stored with the whole
oracle field's 2-norm and max-norm in golden/helmholtz1024_samples.txt by
golden/make_helmholtz_samples.py (oracle only; a full oracle solve takes
minutes).  The tolerance is relative to the field's max-norm.  A whole-field
check goes with it: with A = I - alpha L self-adjoint in the
volume-weighted inner product and A >= I,
||e||_D / ||x||_D <= kappa_D ||f - A x||_D / ||f||_D, where
kappa_D <= 1 + alpha * sum_d (Gershgorin bound of the symmetrised T_d) and
the residual is computed by the oracle's stencil in FP64."""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import cuda, host, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "helmholtz1024_samples.txt")


def _golden():
    fields = {}
    cur = None
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            if t[0] == "field":
                cur = {"shape": (int(t[2]), int(t[3]), int(t[4])), "norm2": float(t[5]), "maxabs": float(t[6]),
                       "idx": [], "val": []}
                fields[t[1]] = cur
            else:
                cur["idx"].append(int(t[0]))
                cur["val"].append(float(t[1]))
    for f in fields.values():
        f["idx"] = np.array(f["idx"], dtype=np.int64)
        f["val"] = np.array(f["val"])
    return fields


def _kappa_bound(p):
    g = 0.0
    for d in range(3):
        a, b, c, vol = O.operator_1d(p.faces[d], p.bc[d], p.loc[d])
        n = len(b)
        s = np.sqrt(vol)
        sub = np.zeros(n)
        sup = np.zeros(n)
        sub[1:] = np.abs(a[1:]) * s[1:] / s[:-1]
        sup[:-1] = np.abs(c[:-1]) * s[:-1] / s[1:]
        if p.bc[d][0] == "P":
            sub[0] = abs(a[0]) * s[0] / s[-1]
            sup[-1] = abs(c[-1]) * s[-1] / s[0]
        g += float((np.abs(b) + sub + sup).max())
    return 1.0 + p.alpha * g


def _dnorm(p, x):
    return float(np.sqrt((p.volumes() * x * x).sum()))


def _solve_batch(prec, fixed):
    import torch
    import paper_2603_09528_amd as T
    comps = W.helmholtz3()
    say("plans", prec)
    plans = [T.Plan.from_problem(p, precision=prec, fixed_refine=fixed) for p, _ in comps]
    rhs = [cuda(W.rhs(p, s)) for p, s in comps]
    outs = [torch.empty_like(r) for r in rhs]
    b = T.Batch(plans)
    say("batch solve", prec)
    b.solve(rhs, outs, use_graph=False)
    torch.cuda.synchronize()
    infos = [b.info(i) for i in range(3)]
    xs = [host(o) for o in outs]
    del outs, rhs, b
    torch.cuda.empty_cache()
    return comps, xs, infos


def _compare_samples(comps, xs, tol):
    gold = _golden()
    for (p, _), x in zip(comps, xs):
        g = gold[p.name]
        assert g["shape"] == p.shape
        xf = x.reshape(-1)
        err = float(np.abs(xf[g["idx"]] - g["val"]).max()) / g["maxabs"]
        nerr = abs(float(np.linalg.norm(xf)) - g["norm2"]) / g["norm2"]
        merr = abs(float(np.abs(xf).max()) - g["maxabs"]) / g["maxabs"]
        say(f"  {p.name}: sampled max-norm error {err:.3e}, 2-norm {nerr:.3e}, max {merr:.3e}")
        assert err <= tol and nerr <= tol and merr <= tol, (p.name, err, nerr, merr)


def test_helmholtz_staggered_three_rhs_fp64():
    comps, xs, infos = _solve_batch("fp64", -1)
    for inf in infos:
        assert inf.nonfinite == 0 and inf.compat_defect == 0.0
    _compare_samples(comps, xs, 1e-12)


def test_helmholtz_staggered_three_rhs_bf16x3():
    # two corrections: the count the benchmark times (one leaves ~1e-10)
    comps, xs, infos = _solve_batch("bf16x3", 2)
    for inf in infos:
        assert inf.iters == 2 and inf.nonfinite == 0
    _compare_samples(comps, xs, 1e-10)
    for (p, s), x in zip(comps, xs):
        say("residual", p.name)
        f = W.rhs(p, s)
        r = O.residual(p, f, x)
        bound = _kappa_bound(p) * _dnorm(p, r) / _dnorm(p, f)
        spread = np.sqrt(p.volumes().max() / p.volumes().min())
        say("  kappa bound", _kappa_bound(p), "error bound", bound * spread)
        assert bound * spread <= 1e-10

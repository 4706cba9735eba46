"""The implicit-diffusion Helmholtz workload at full size on the GPU:
(I - alpha L) u = f, alpha = 1e-4, 1024 x 768 x 512 cells, x periodic uniform,
y and z Dirichlet walls with tanh beta = 2, the three staggered velocity
components (u on x-faces, v on y-faces, w on z-faces) solved as one batch of
three plans with split-BF16x3 transforms and FP64 refinement.

The u component is compared element by element with the oracle.  For v and
w (a full oracle solve of each takes minutes) the check is a bound that holds
at any size: with A = I - alpha L self-adjoint in the volume-weighted inner
product and A >= I, ||e||_D / ||x||_D <= kappa_D ||f - A x||_D / ||f||_D, with
kappa_D <= 1 + alpha * sum_d (Gershgorin bound of the symmetrised T_d) and the
residual computed by the oracle's stencil in FP64."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import cuda, host, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _kappa_bound(p):
    g = 0.0
    for d in range(3):
        a, b, c, vol = O.operator_1d(p.faces[d], p.bc[d], p.loc[d])
        n = len(b)
        off = np.zeros(n + 1)
        s = np.sqrt(vol)
        sub = np.zeros(n)
        sup = np.zeros(n)
        sub[1:] = np.abs(a[1:]) * s[1:] / s[:-1]
        sup[:-1] = np.abs(c[:-1]) * s[:-1] / s[1:]
        if p.bc[d][0] == "P":
            sub[0] = abs(a[0]) * s[0] / s[-1]
            sup[-1] = abs(c[-1]) * s[-1] / s[0]
        g += float((np.abs(b) + sub + sup).max())
        del off
    return 1.0 + p.alpha * g


def _dnorm(p, x):
    return float(np.sqrt((p.volumes() * x * x).sum()))


def test_helmholtz_staggered_three_rhs_bf16x3():
    import torch
    import paper_2603_09528_amd as T
    comps = W.helmholtz3()
    say("plans")
    plans = [T.Plan.from_problem(p, precision="bf16x3", fixed_refine=4) for p, _ in comps]
    rhs = [cuda(W.rhs(p, s)) for p, s in comps]
    outs = [torch.empty_like(r) for r in rhs]
    b = T.Batch(plans)
    say("batch solve")
    b.solve(rhs, outs, use_graph=False)
    torch.cuda.synchronize()
    xs = [host(o) for o in outs]
    del outs, b
    # v and w: residual bound
    for (p, s), x in list(zip(comps, xs))[1:]:
        say("residual", p.name)
        f = W.rhs(p, s)
        r = O.residual(p, f, x)
        bound = _kappa_bound(p) * _dnorm(p, r) / _dnorm(p, f)
        spread = np.sqrt(p.volumes().max() / p.volumes().min())
        say("  kappa bound", _kappa_bound(p), "error bound", bound * spread)
        assert bound * spread <= 1e-10
    # u: element-wise against the oracle
    p, s = comps[0]
    say("oracle", p.name)
    f = W.rhs(p, s)
    ref = O.solve(p, f)
    err = O.relative_error(p, xs[0], ref)
    say("  rel err", err)
    assert err <= 1e-10

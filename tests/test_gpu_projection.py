"""Projection step on the GPU (§2.1 staggered grid, §4.1 divergence test):
the divergence and gradient-update kernels element by element against the
oracle's, and the projection of a white-noise velocity through the C-ABI,
whose divergence must vanish to round-off, against the oracle's projection."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import projection as P
from tests.gpu_util import cuda, host, say

pytestmark = pytest.mark.gpu

GRIDS = [
    # pressure grids: n, beta, bc (P or N per direction: periodic or walls)
    ((48, 40, 36), (0.0, 2.0, 1.5), (W.PP, W.NN, W.NN)),     # channel
    ((33, 29, 27), (1.5, 2.0, 1.0), (W.NN, W.NN, W.NN)),     # cavity
    ((40, 32, 24), (0.0, 0.0, 2.0), (W.PP, W.PP, W.NN)),     # x, y by fast transforms
    ((20, 24, 18), (1.0, 0.0, 0.0), (W.NN, W.PP, W.PP)),     # periodic z (cyclic lines)
    ((257, 3, 300), (2.0, 1.0, 2.0), (W.NN, W.NN, W.NN)),    # ragged columns, long lines
]


def _T():
    import paper_2603_09528_amd as T
    return T


def _grid(g):
    n, beta, bc = g
    return W.make_problem(n, beta, bc)


@pytest.mark.parametrize("g", GRIDS, ids=lambda g: "".join(b[0] for b in g[2]) + f"-{g[0][0]}")
def test_divergence_and_gradient_match_oracle(g):
    import torch
    T = _T()
    p = _grid(g)
    plan = T.Plan.from_problem(p)
    u, v, w = W.white_noise_velocity(p, 7)
    assert plan.velocity_shapes() == tuple(a.shape for a in (u, v, w))
    du = host(plan.divergence(cuda(u), cuda(v), cuda(w)))
    ref = P.divergence(p, u, v, w)
    assert np.abs(du - ref).max() <= 1e-14 * P.divergence_flux_bound(p, u, v, w)
    phi = np.random.default_rng(8).standard_normal(p.shape)
    gu, gv, gw = cuda(u), cuda(v), cuda(w)
    plan.gradient_update(cuda(phi), gu, gv, gw)
    torch.cuda.synchronize()
    gx, gy, gz = P.gradient(p, phi)
    # rounding: the centre distance dx_{m+1/2} of a small cell near a wall
    # carries a relative error up to eps |x| / dx_{m+1/2} in either
    # formulation (difference of two centres, or half the sum of two widths)
    eps = np.finfo(float).eps
    for d, (got, comp, g, name) in enumerate(((gu, u, gx, "u"), (gv, v, gy, "v"), (gw, w, gz, "w"))):
        dc = P._dir(p, d)[2][: g.shape[2 - d]]
        shape = [1, 1, 1]
        shape[2 - d] = -1
        cond = 1.0 + np.abs(p.faces[d]).max() / dc.reshape(shape)
        bound = 8 * eps * (np.abs(comp) + np.abs(g) * cond)
        err = np.abs(host(got) - (comp - g))
        assert (err <= bound).all(), (name, float((err / bound).max()))


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("g", GRIDS, ids=lambda g: "".join(b[0] for b in g[2]) + f"-{g[0][0]}")
def test_projected_white_noise_is_divergence_free(g, prec):
    import torch
    T = _T()
    p = _grid(g)
    kw = {} if prec == "fp64" else {"precision": prec, "rtol": 1e-13, "max_refine": 12}
    plan = T.Plan.from_problem(p, **kw)
    u, v, w = W.white_noise_velocity(p, 9)
    du, dv, dw = cuda(u), cuda(v), cuda(w)
    d0 = np.abs(P.divergence(p, u, v, w)).max()
    phi = host(plan.project(du, dv, dw))
    pu, pv, pw = host(du), host(dv), host(dw)
    # the projected field's divergence by the oracle's stencil and by the kernel
    d1 = np.abs(P.divergence(p, pu, pv, pw)).max()
    d1k = np.abs(host(plan.divergence(du, dv, dw))).max()
    bound = P.divergence_flux_bound(p, pu, pv, pw)
    say(f"{prec} {p.n}: max|D u*| {d0:.3e}, max|D u| {d1:.3e} (kernel {d1k:.3e}), flux bound {bound:.3e}")
    assert d1 <= 1e-13 * d0 and d1k <= 1e-13 * d0
    assert d1 <= 256 * np.finfo(float).eps * bound
    # against the oracle's projection: the velocity is unique, phi up to a constant
    ou, ov, ow, ophi = P.project(p, u, v, w)
    tol = 1e-12 if prec == "fp64" else 1e-10
    for got, want in ((pu, ou), (pv, ov), (pw, ow)):
        assert np.abs(got - want).max() <= tol * np.abs(want).max()
    assert O.relative_error(p, phi, ophi, norm="max") <= tol
    assert plan.info().compat_defect <= 1e-13


def test_projection_rejects_non_pressure_plans():
    T = _T()
    bad = [W.make_problem((16, 16, 16), (1.0, 1.0, 1.0), (W.DD, W.NN, W.NN)),
           W.make_problem((16, 16, 16), (0.0, 1.0, 1.0), (W.PP, W.DD, W.DD), loc=("F", "C", "C"),
                          kind="helmholtz", alpha=1e-3)]
    for p in bad:
        plan = T.Plan.from_problem(p)
        z = cuda(np.zeros(p.shape))
        with pytest.raises(T.TptError) as ei:
            T._check(T.lib().tpt_divergence(plan.handle, z.data_ptr(), z.data_ptr(), z.data_ptr(),
                                            z.data_ptr(), None))
        assert ei.value.code == -1

"""Closed-form incompressible flows advanced by the GPU time stepper over many
steps, against the exact solutions of the Navier--Stokes equations (§2.1),
independently of the oracle:

* the Taylor--Green vortex on a doubly periodic domain, u = sin 2pi x
  cos 2pi y, v = -cos 2pi x sin 2pi y, decaying as exp(-8 pi^2 nu t), with
  pressure (cos 4pi x + cos 4pi y) / 4 exp(-16 pi^2 nu t);
* a decaying shear mode between no-slip walls on a stretched grid,
  u = sin pi y sin pi z (advection vanishes), decaying as exp(-2 pi^2 nu t).

The errors at the final time must be small and fall at second order when the
grid and the time step are refined (ratio >= 3.5 for a halved spacing): a
validation of the discretised solver as a whole -- advection, diffusion,
the implicit and explicit splits, projection and pressure update -- across
hundreds of substeps."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import cuda, host, say

pytestmark = pytest.mark.gpu


def _positions(p, c):
    """Coordinates (X, Y, Z) of the unknowns of velocity component c."""
    coords = []
    for e in range(3):
        f = p.faces[e]
        if e == c:
            coords.append(f[1:] if p.bc[e][0] == "P" else f[1:-1])
        else:
            coords.append(0.5 * (f[:-1] + f[1:]))
    Z, Y, X = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    return X, Y, Z


def _advance(p, vel, nu, dt, nsteps, implicit):
    import torch
    import paper_2603_09528_amd as T
    plan = T.Plan.from_problem(p)
    ns = T.NavierStokes(plan, nu, dt, implicit)
    du, dv, dw = (cuda(a) for a in vel)
    dP = torch.zeros(plan.shape, dtype=torch.float64, device="cuda")
    for _ in range(nsteps):
        ns.step(du, dv, dw, dP)
    torch.cuda.synchronize()
    return host(du), host(dv), host(dw), host(dP)


def _taylor_green(n, implicit, T=0.125, nu=0.01):
    p = W.make_problem((n, n, 4), (0.0, 0.0, 0.0), (W.PP, W.PP, W.PP))
    X, Y, _ = _positions(p, 0)
    u = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    X, Y, _ = _positions(p, 1)
    v = -np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    w = np.zeros(W.velocity_shapes(p)[2])
    nsteps = 10 * n // 16
    say("taylor-green", n, implicit, nsteps, "steps")
    gu, gv, gw, gP = _advance(p, (u, v, w), nu, T / nsteps, nsteps, implicit)
    F = np.exp(-8 * np.pi ** 2 * nu * T)
    xc = 0.5 * (p.faces[0][:-1] + p.faces[0][1:])
    Xc, Yc = np.meshgrid(xc, xc, indexing="xy")
    pex = np.broadcast_to((np.cos(4 * np.pi * Xc) + np.cos(4 * np.pi * Yc)) / 4 * F * F, p.shape)
    eu = max(np.abs(gu - u * F).max(), np.abs(gv - v * F).max())
    ep = np.abs((gP - gP.mean()) - (pex - pex.mean())).max()
    assert np.abs(gw).max() < 1e-12
    return eu, ep


@pytest.mark.parametrize("implicit", ["none", "xyz"])
def test_taylor_green_vortex_second_order(implicit):
    eu16, ep16 = _taylor_green(16, implicit)
    eu32, ep32 = _taylor_green(32, implicit)
    say("taylor-green errors", implicit, eu16, eu32, ep16, ep32)
    assert eu16 < 1.5e-3 and ep16 < 1.6e-2, (eu16, ep16)
    assert eu16 / eu32 > 3.5 and ep16 / ep32 > 3.5, (eu16 / eu32, ep16 / ep32)


def _shear_mode(n, implicit, nsteps, T=0.5, nu=0.05):
    p = W.make_problem((8, n, n), (0.0, 1.5, 1.5), (W.PP, W.NN, W.NN))
    shp = W.velocity_shapes(p)
    _, Y, Z = _positions(p, 0)
    u = np.sin(np.pi * Y) * np.sin(np.pi * Z)
    say("shear mode", n, implicit, nsteps, "steps")
    gu, gv, gw, _ = _advance(p, (u, np.zeros(shp[1]), np.zeros(shp[2])), nu, T / nsteps, nsteps, implicit)
    assert np.abs(gv).max() < 1e-12 and np.abs(gw).max() < 1e-12
    return np.abs(gu - u * np.exp(-2 * np.pi ** 2 * nu * T)).max()


@pytest.mark.parametrize("implicit,nsteps", [("xyz", 20), ("none", 200)])
def test_wall_bounded_mode_second_order_on_stretched_grid(implicit, nsteps):
    e16 = _shear_mode(16, implicit, nsteps)
    e32 = _shear_mode(32, implicit, nsteps)
    say("shear mode errors", implicit, e16, e32)
    assert e16 < 3e-3, e16
    assert e16 / e32 > 3.5, e16 / e32

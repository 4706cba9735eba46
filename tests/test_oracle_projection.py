"""Pins of the oracle's projection step (§2.1 staggered grid; §4.1
divergence test).

* D G = L: the divergence of the gradient is the pressure operator of
  Eq. poisson-fd2 with its Neumann / periodic rows (itself pinned by closed
  forms in test_oracle_operator.py);
* discrete integration by parts: sum_cells dV phi (D u) = -sum_faces
  dV_face u (G phi), so G = -D^T in the volume-weighted inner products;
* second-order convergence of D and G to the continuous divergence and
  gradient on stretched grids;
* the projection of a white-noise velocity is divergence-free to round-off
  and projecting twice changes nothing.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import projection as P

BCS = [(W.PP, W.NN, W.NN), (W.NN, W.NN, W.NN), (W.PP, W.PP, W.NN), (W.NN, W.PP, W.PP), (W.PP, W.PP, W.PP)]


def _prob(bc, n=(9, 7, 8), beta=(1.5, 2.0, 1.0)):
    return W.make_problem(n, beta, bc)


@pytest.mark.parametrize("bc", BCS, ids=lambda b: "".join(x[0] + x[1] for x in b))
def test_divergence_of_gradient_is_the_operator(bc):
    p = _prob(bc)
    phi = np.random.default_rng(1).standard_normal(p.shape)
    lap = O.apply_operator(p, phi)
    dg = P.divergence(p, *P.gradient(p, phi))
    assert np.abs(dg - lap).max() <= 1e-13 * np.abs(lap).max()


@pytest.mark.parametrize("bc", BCS, ids=lambda b: "".join(x[0] + x[1] for x in b))
def test_gradient_is_minus_divergence_adjoint(bc):
    p = _prob(bc)
    rng = np.random.default_rng(2)
    phi = rng.standard_normal(p.shape)
    u, v, w = W.white_noise_velocity(p, 3)
    lhs = float((p.volumes() * phi * P.divergence(p, u, v, w)).sum())
    gx, gy, gz = P.gradient(p, phi)
    # face control volumes: centre distance along the face normal times the
    # cell widths of the other two directions
    wx, wy, wz = (np.diff(p.faces[d]) for d in range(3))
    dcs = [P._dir(p, d)[2] for d in range(3)]
    rhs = (float((gx * u * dcs[0][None, None, :] * wy[None, :, None] * wz[:, None, None]).sum())
           + float((gy * v * wx[None, None, :] * dcs[1][None, :, None] * wz[:, None, None]).sum())
           + float((gz * w * wx[None, None, :] * wy[None, :, None] * dcs[2][:, None, None]).sum()))
    assert abs(lhs + rhs) <= 1e-13 * (abs(lhs) + abs(rhs))


def test_total_flux_vanishes():
    """Walls carry no flux and periodic faces cancel: sum dV (D u) = 0."""
    for bc in BCS:
        p = _prob(bc)
        u, v, w = W.white_noise_velocity(p, 4)
        d = P.divergence(p, u, v, w)
        assert abs(float((p.volumes() * d).sum())) <= 1e-14 * float((p.volumes() * np.abs(d)).sum())


def _fields(p):
    """Smooth velocity and pressure for the convergence tests (x periodic,
    y and z walls): u = sin(2 pi x) y(1-y) cos(pi z), v = cos(2 pi x) sin(pi y) z^2,
    w = (1 + sin(2 pi x)) cos(pi y) sin(pi z), with zero
    normal velocity on the walls, and their divergence / the pressure
    gradient at the unknowns."""
    fx = [np.asarray(p.faces[d]) for d in range(3)]
    cx = [0.5 * (f[:-1] + f[1:]) for f in fx]
    ux = fx[0][1:]                     # x faces of the periodic direction
    vy = fx[1][1:-1]                   # interior y faces
    wz = fx[2][1:-1]                   # interior z faces
    X, Y, Z = cx[0][None, None, :], cx[1][None, :, None], cx[2][:, None, None]
    u = np.sin(2 * np.pi * ux)[None, None, :] * (Y * (1 - Y)) * np.cos(np.pi * Z)
    v = np.cos(2 * np.pi * X) * np.sin(np.pi * vy)[None, :, None] * Z ** 2
    w = (1 + np.sin(2 * np.pi * X)) * np.cos(np.pi * Y) * np.sin(np.pi * wz)[:, None, None]
    div = (2 * np.pi * np.cos(2 * np.pi * X) * (Y * (1 - Y)) * np.cos(np.pi * Z)
           + np.cos(2 * np.pi * X) * np.pi * np.cos(np.pi * Y) * Z ** 2
           + (1 + np.sin(2 * np.pi * X)) * np.cos(np.pi * Y) * np.pi * np.cos(np.pi * Z))
    pres = np.cos(2 * np.pi * X) * np.cos(np.pi * Y) * np.cos(np.pi * Z)
    gx = -2 * np.pi * np.sin(2 * np.pi * ux)[None, None, :] * np.cos(np.pi * Y) * np.cos(np.pi * Z)
    gy = -np.pi * np.cos(2 * np.pi * X) * np.sin(np.pi * vy)[None, :, None] * np.cos(np.pi * Z)
    gz = -np.pi * np.cos(2 * np.pi * X) * np.cos(np.pi * Y) * np.sin(np.pi * wz)[:, None, None]
    return (u, v, w), div, pres, (gx, gy, gz)


def test_divergence_and_gradient_second_order():
    ed, eg = [], []
    for n in (16, 32, 64):
        p = W.channel_pressure((n, n, n), beta=1.5)
        (u, v, w), div, pres, g = _fields(p)
        ed.append(np.abs(P.divergence(p, u, v, w) - div).max())
        gg = P.gradient(p, pres)
        eg.append(max(np.abs(a - b).max() for a, b in zip(gg, g)))
    od = np.log2(np.array(ed[:-1]) / np.array(ed[1:]))
    og = np.log2(np.array(eg[:-1]) / np.array(eg[1:]))
    assert od[-1] >= 1.8, od
    assert og[-1] >= 1.8, og


@pytest.mark.parametrize("bc", BCS, ids=lambda b: "".join(x[0] + x[1] for x in b))
def test_projection_of_white_noise_is_divergence_free(bc):
    p = _prob(bc, n=(12, 10, 9))
    u, v, w = W.white_noise_velocity(p, 5)
    pu, pv, pw, phi = P.project(p, u, v, w)
    d0 = np.abs(P.divergence(p, u, v, w)).max()
    d1 = np.abs(P.divergence(p, pu, pv, pw)).max()
    assert d1 <= 1e-13 * d0, (d1, d0)
    assert d1 <= 64 * np.finfo(float).eps * P.divergence_flux_bound(p, pu, pv, pw)
    # a divergence-free field is its own projection
    qu, qv, qw, _ = P.project(p, pu, pv, pw)
    for a, b in ((qu, pu), (qv, pv), (qw, pw)):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()

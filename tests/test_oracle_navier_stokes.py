"""Pins of the Navier--Stokes substep oracle (§2.1, Eq. rk3) against closed
forms and invariants that do not retype its arithmetic:

* advection of a constant field is zero;
* advection conserves kinetic energy for a discretely divergence-free field
  on stretched grids with walls (the symmetry-preserving property the paper
  claims for its discretisation): a wrong interpolation weight, index or
  sign breaks it;
* advection converges at second order to -div(u (x) u) of smooth fields,
  derivatives taken by complex step (exact to rounding);
* on a discrete eigenmode of the diffusion operator (advection and pressure
  vanish there) one full step multiplies the mode by the amplification
  factor of the scheme: 1 + z + z^2/2 + z^3/6 (a three-stage third-order
  Runge--Kutta method on y' = lambda y) when diffusion is explicit,
  prod_k (1 + gamma_k z/2) / (1 - gamma_k z/2) (Crank--Nicolson substeps)
  when it is implicit;
* the updated velocity is discretely divergence-free;
* for the Taylor--Green vortex (an Euler steady state whose advection is a
  pure gradient) the pressure after one substep is the exact pressure
  (cos 4 pi x + cos 4 pi y) / 4 up to the discretisation error.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import navier_stokes as NS
from oracle.operator import dense_1d, operator_1d

GRIDS = [
    ((12, 10, 9), (0.0, 2.0, 1.5), (W.PP, W.NN, W.NN)),
    ((9, 11, 10), (1.5, 2.0, 1.0), (W.NN, W.NN, W.NN)),
    ((10, 8, 12), (0.0, 0.0, 2.0), (W.PP, W.PP, W.NN)),
]


def _grid(g):
    return W.make_problem(*g)


def _solenoidal(p, seed):
    u, v, w = W.white_noise_velocity(p, seed)
    u, v, w, _ = O.projection.project(p, u, v, w)
    return u, v, w


def test_advection_of_constant_field_is_zero():
    p = _grid(((8, 6, 5), (0.0, 0.0, 0.0), (W.PP, W.PP, W.PP)))
    shp = W.velocity_shapes(p)
    u, v, w = (np.full(s, c) for s, c in zip(shp, (1.3, -0.7, 0.4)))
    for a in NS.advection(p, u, v, w):
        assert np.abs(a).max() < 1e-13
    # channel: a uniform streamwise velocity between the walls
    p = _grid(GRIDS[0])
    shp = W.velocity_shapes(p)
    u = np.full(shp[0], 2.0)
    for a in NS.advection(p, u, np.zeros(shp[1]), np.zeros(shp[2])):
        assert np.abs(a).max() < 1e-12


@pytest.mark.parametrize("g", GRIDS, ids=lambda g: "".join(b[0] for b in g[2]))
def test_advection_conserves_kinetic_energy(g):
    p = _grid(g)
    u, v, w = _solenoidal(p, 3)
    assert np.abs(O.projection.divergence(p, u, v, w)).max() < 1e-9
    adv = NS.advection(p, u, v, w)
    for c, (q, a) in enumerate(zip((u, v, w), adv)):
        vol = NS.velocity_volumes(p, c)
        terms = vol * q * a
        scale = np.abs(terms).sum()
        assert scale > 1e-3
        assert abs(terms.sum()) < 1e-12 * scale, (c, terms.sum() / scale)
    # a field that is not divergence-free does produce energy: the invariant
    # above is not trivially satisfied
    u2, v2, w2 = W.white_noise_velocity(p, 4)
    tot = sum(abs((NS.velocity_volumes(p, c) * q * a).sum()) / np.abs(NS.velocity_volumes(p, c) * q * a).sum()
              for c, (q, a) in enumerate(zip((u2, v2, w2), NS.advection(p, u2, v2, w2))))
    assert tot > 1e-3


def _fields(X, Y, Z):
    """Smooth velocity with zero normal velocity on the walls y = 0, 1 and
    z = 0, 1; periodic in x."""
    tp = 2 * np.pi
    u = np.cos(tp * X) * np.cos(np.pi * Y) * (1.0 + 0.5 * np.cos(np.pi * Z))
    v = (0.5 + np.sin(tp * X)) * np.sin(np.pi * Y) * np.cos(np.pi * Z)
    w = np.cos(tp * X) * np.cos(np.pi * Y) * np.sin(np.pi * Z) * (1.0 + Y)
    return u, v, w


def _exact_advection(c, X, Y, Z):
    """-(d/dx (q_c u) + d/dy (q_c v) + d/dz (q_c w)) by complex-step derivatives."""
    h = 1e-30
    out = 0.0
    for e, (dx, dy, dz) in enumerate(((h, 0, 0), (0, h, 0), (0, 0, h))):
        f = _fields(X + 1j * dx, Y + 1j * dy, Z + 1j * dz)
        out = out - np.imag(f[c] * f[e]) / h
    return out


def _positions(p, c):
    """Coordinates (X, Y, Z) of the unknowns of component c."""
    coords = []
    for e in range(3):
        f = p.faces[e]
        if e == c:
            x = f[1:] if p.bc[e][0] == "P" else f[1:-1]
        else:
            x = 0.5 * (f[:-1] + f[1:])
        coords.append(x)
    Z, Y, X = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    return X, Y, Z


def test_advection_is_second_order():
    errs = []
    for n in (16, 32, 64):
        p = W.make_problem((n, n, n), (0.0, 2.0, 1.5), (W.PP, W.NN, W.NN))
        vel = []
        for c in range(3):
            vel.append(_fields(*_positions(p, c))[c])
        adv = NS.advection(p, *vel)
        errs.append(max(np.abs(adv[c] - _exact_advection(c, *_positions(p, c))).max() for c in range(3)))
    assert errs[0] / errs[1] > 3.4 and errs[1] / errs[2] > 3.7, errs


def _mode(p, c):
    """A discrete eigenmode of the diffusion operator of component c that is
    constant along x (periodic): q(j, k) = s_y(j) s_z(k), s_d the eigenvector
    of the third-smallest |eigenvalue| of the dense 1-D operator along d (a
    library eigensolver); returns q and (lambda_y, lambda_z)."""
    pc = NS.velocity_problem(p, c)
    vecs, lams = [], []
    for d in (1, 2):
        a, b, cc, _ = operator_1d(pc.faces[d], pc.bc[d], pc.loc[d])
        lam, vec = np.linalg.eig(dense_1d(a, b, cc, pc.bc[d][0] == "P"))
        i = np.argsort(np.abs(lam.real))[2]
        vecs.append(vec[:, i].real)
        lams.append(lam[i].real)
    q = np.zeros(pc.shape)
    q[:] = (vecs[1][:, None] * vecs[0][None, :])[:, :, None]
    return q, lams


@pytest.mark.parametrize("implicit", ["none", "z", "yz", "xyz"])
def test_full_step_amplification_of_eigenmode(implicit):
    p = _grid(GRIDS[0])
    shp = W.velocity_shapes(p)
    q, (ly, lz) = _mode(p, 0)
    nu = 0.01
    dt = 0.3 / (nu * abs(ly + lz))                 # nu dt (lambda_y + lambda_z) = -0.3
    vel, P = NS.rk3_step(p, dt, nu, implicit, q, np.zeros(shp[1]), np.zeros(shp[2]), np.zeros(p.shape))
    z = nu * dt * (ly + lz)
    if implicit == "none":
        R = 1 + z + z * z / 2 + z ** 3 / 6
    elif implicit in ("yz", "xyz"):                # the mode is constant along x: L_E q = 0
        R = np.prod([(1 + g * z / 2) / (1 - g * z / 2) for g in (8 / 15, 2 / 15, 1 / 3)])
    else:
        R = None
    ratio = np.vdot(q.ravel(), vel[0].ravel()) / np.vdot(q.ravel(), q.ravel())
    # the result is a multiple of the mode
    assert np.allclose(vel[0], ratio * q, rtol=0, atol=1e-13 * np.abs(q).max())
    if R is not None:
        assert abs(ratio - R) < 1e-13, (ratio, R)
    else:
        # explicit y, implicit z: second order in time, so within |z|^3 of
        # the exact decay exp(z)
        assert abs(ratio - np.exp(z)) < abs(z) ** 3, (ratio, np.exp(z))
    assert np.abs(vel[1]).max() < 1e-13 and np.abs(vel[2]).max() < 1e-13
    assert np.abs(P).max() < 1e-10


def test_rk3_coefficients_sum_to_one():
    """Consistency of Eq. rk3: the weights of the explicit terms over a step
    sum to one, and gamma_k sums to one (the pressure time level)."""
    a = sum(NS.RK3_ALPHA) + sum(NS.RK3_BETA)
    g = sum(NS.rk3_coefficients(k)[2] for k in (1, 2, 3))
    assert abs(a - 1) < 1e-15 and abs(g - 1) < 1e-15


@pytest.mark.parametrize("implicit", ["none", "z", "yz", "xyz"])
@pytest.mark.parametrize("g", GRIDS[:2], ids=lambda g: "".join(b[0] for b in g[2]))
def test_substep_leaves_divergence_free_velocity(g, implicit):
    p = _grid(g)
    u, v, w = _solenoidal(p, 5)
    rng = np.random.default_rng(6)
    e = tuple(rng.standard_normal(s) for s in W.velocity_shapes(p))
    P = rng.standard_normal(p.shape)
    for k in (1, 2, 3):
        (u2, v2, w2), e2, P2, phi = NS.rk3_substep(p, k, 1e-3, 0.05, implicit, u, v, w, e, P)
        div = O.projection.divergence(p, u2, v2, w2)
        assert np.abs(div).max() < 1e-10 * O.projection.divergence_flux_bound(p, u2, v2, w2)
        assert np.isfinite(P2).all()


def test_taylor_green_pressure():
    n = 32
    p = W.make_problem((n, n, 2), (0.0, 0.0, 0.0), (W.PP, W.PP, W.PP))
    X, Y, Z = _positions(p, 0)
    u = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    X, Y, Z = _positions(p, 1)
    v = -np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    w = np.zeros(W.velocity_shapes(p)[2])
    dt = 1e-4
    (u2, v2, _), _, P, phi = NS.rk3_substep(p, 1, dt, 0.0, "none", u, v, w, (None,) * 3, np.zeros(p.shape))
    xc = 0.5 * (p.faces[0][:-1] + p.faces[0][1:])
    Xc, Yc = np.meshgrid(xc, xc, indexing="xy")
    exact = np.broadcast_to((np.cos(4 * np.pi * Xc) + np.cos(4 * np.pi * Yc)) / 4, p.shape)
    err = (P - P.mean()) - (exact - exact.mean())
    assert np.abs(err).max() < 0.02 * np.abs(exact).max(), np.abs(err).max()
    # the steady Euler solution barely moves: far less than dt |A u|
    assert np.abs(u2 - u).max() < 0.05 * dt * (2 * np.pi)


@pytest.mark.parametrize("implicit", ["z", "yz", "xyz"])
def test_substep_satisfies_crank_nicolson_momentum_with_updated_pressure(implicit):
    """On a uniform periodic grid L_I and G commute, and the fractional step
    with the pressure update P^{k+1/2} = P^{k-1/2} + Phi - c L_I Phi is the
    Crank--Nicolson momentum equation
        u^{k+1} - u^k = dt (alpha E^k + beta E^{k-1}) - gamma dt G P^{k+1/2}
                        + gamma nu dt L_I (u^k + u^{k+1}) / 2
    exactly; a wrong pressure update leaves gamma dt G (2 c L_I Phi)."""
    p = W.make_problem((8, 10, 12), (0.0, 0.0, 0.0), (W.PP, W.PP, W.PP), length=(1.0, 2.0, 1.5))
    rng = np.random.default_rng(8)
    shp = W.velocity_shapes(p)
    u, v, w = (rng.standard_normal(s) for s in shp)
    e_prev = tuple(rng.standard_normal(s) for s in shp)
    P = rng.standard_normal(p.shape)
    nu, dt = 0.3, 0.02
    dirs = NS.IMPLICIT[implicit]
    for k in (1, 2, 3):
        a, b, g = NS.rk3_coefficients(k)
        (u2, v2, w2), e, P2, phi = NS.rk3_substep(p, k, dt, nu, implicit, u, v, w, e_prev, P)
        gp = O.projection.gradient(p, P2)
        for c, (q0, q1) in enumerate(zip((u, v, w), (u2, v2, w2))):
            pc = NS.velocity_problem(p, c)
            lhs = q1 - q0
            rhs = (dt * (a * e[c] + b * e_prev[c]) - g * dt * gp[c]
                   + g * nu * dt * NS.laplacian_dirs(pc, q0 + q1, dirs) / 2)
            assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(lhs).max(), (k, c)
        u, v, w, e_prev, P = u2, v2, w2, e, P2

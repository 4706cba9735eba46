"""Pins of the oracle's tensor-product--Thomas solve.

* Thomas lines against a dense solve of each line (brute force), and the
  gauge pin of §3 on a singular line (also for the cyclic lines of a
  periodic z);
* the whole solve against the plain definition x = A^{-1} f (dense LU of the
  assembled operator, bordered for singular problems) on grids up to 12^3,
  over boundary conditions, staggering, stretching and Poisson/Helmholtz;
* the algebraic residual at round-off (§4.1);
* second-order convergence to manufactured solutions (the discretisation of
  Eq. poisson-fd2 is second order);
* the gauge implied by the final-pivot pin: zero area-weighted mean of the
  last z plane.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def test_thomas_lines_brute_force():
    rng = np.random.default_rng(1)
    nz = 9
    faces = W.tanh_faces(nz, 2.0)
    for bc in (W.DD, W.NN, ("N", "D")):
        az, bz, cz, _ = O.operator_1d(faces, bc, "C")
        lam = -rng.uniform(0.5, 50.0, size=(3, 4))
        rhs = rng.standard_normal((nz, 3, 4))
        for sigma, tau in ((0.0, 1.0), (1.0, -1e-2)):
            x, _ = O.thomas_lines(az, bz, cz, lam, sigma, tau, rhs)
            Tz = O.dense_1d(az, bz, cz, False)
            for j in range(3):
                for i in range(4):
                    M = sigma * np.eye(nz) + tau * (lam[j, i] * np.eye(nz) + Tz)
                    ref = np.linalg.solve(M, rhs[:, j, i])
                    assert np.abs(x[:, j, i] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_thomas_pinned_singular_line():
    nz = 11
    az, bz, cz, _ = O.operator_1d(W.tanh_faces(nz, 1.5), W.NN, "C")
    rhs = np.random.default_rng(2).standard_normal((nz, 1))
    lam = np.zeros(1)
    x, piv = O.thomas_lines(az, bz, cz, lam, 0.0, 1.0, rhs, pin=(0,))
    Tz = O.dense_1d(az, bz, cz, False)
    assert abs(piv[0]) <= 64 * nz * np.finfo(float).eps * np.abs(bz).max()
    assert x[-1, 0] == 0.0
    r = Tz @ x[:, 0] - rhs[:, 0]
    assert np.abs(r[:-1]).max() <= 1e-12 * np.abs(rhs).max()   # all but the dropped last equation


BCS = [
    (W.NN, W.NN, W.NN),
    (W.PP, W.NN, W.NN),
    (W.PP, W.PP, W.DD),
    (W.DD, ("N", "D"), ("D", "N")),
    (("N", "D"), W.PP, W.NN),
    (W.NN, W.DD, W.PP),
    (W.PP, W.PP, W.PP),
]


@pytest.mark.parametrize("bc", BCS, ids=lambda b: "".join(x[0] + x[1] for x in b))
@pytest.mark.parametrize("kind,alpha", [("poisson", 0.0), ("helmholtz", 2e-3)])
@pytest.mark.parametrize("n,beta", [((6, 5, 7), (1.5, 1.5, 1.5)), ((12, 12, 12), (2.5, 0.5, 2.0)),
                                    ((2, 3, 2), (1.0, 1.0, 1.0))])
def test_solve_matches_dense_lu(bc, kind, alpha, n, beta):
    p = W.make_problem(n, beta, bc, kind=kind, alpha=alpha)
    f = W.rhs(p, 7)
    x = O.solve(p, f)
    ref = O.solve_dense(p, f)
    assert O.relative_error(p, x, ref) <= 5e-14


def test_cyclic_lines_pinned_singular_line():
    # periodic z, zero shift: the cyclic T_z is singular; the pinned line has
    # its last unknown zero and satisfies every equation but the last
    nz = 10
    az, bz, cz, _ = O.operator_1d(W.tanh_faces(nz, 0.0), W.PP, "C")
    rng = np.random.default_rng(3)
    rhs = rng.standard_normal((nz, 1, 2))
    rhs[:, 0, 0] -= rhs[:, 0, 0].mean()
    lam = np.array([[0.0, -3.0]])
    x = O.solver.cyclic_lines(az, bz, cz, lam, 0.0, 1.0, rhs, pin=(0, 0))
    Tz = O.dense_1d(az, bz, cz, True)
    assert x[-1, 0, 0] == 0.0
    r = Tz @ x[:, 0, 0] - rhs[:, 0, 0]
    assert np.abs(r[:-1]).max() <= 1e-12 * np.abs(rhs).max()
    # a compatible right-hand side satisfies the dropped equation too
    assert abs(r[-1]) <= 1e-12 * np.abs(rhs).max()
    r2 = (Tz - 3.0 * np.eye(nz)) @ x[:, 0, 1] - rhs[:, 0, 1]
    assert np.abs(r2).max() <= 1e-12 * np.abs(rhs).max()


@pytest.mark.parametrize("loc", [("F", "C", "C"), ("C", "F", "C"), ("C", "C", "F"), ("F", "F", "F")])
def test_staggered_helmholtz_matches_dense_lu(loc):
    p = W.make_problem((9, 8, 10), (0.0, 2.0, 2.0), (W.PP, W.DD, W.DD), loc=loc,
                       kind="helmholtz", alpha=1e-3)
    f = W.rhs(p, 3)
    assert O.relative_error(p, O.solve(p, f), O.solve_dense(p, f)) <= 5e-14


def test_residual_roundoff_cavity32():
    p = W.cavity32()
    f = W.rhs(p, 1, "uniform")
    x = O.solve(p, f)
    r = O.residual(p, f, x)
    assert np.linalg.norm(r) / np.linalg.norm(f) <= 1e-12
    # residual scaled by the operator size, pointwise (round-off at every point)
    assert np.abs(r).max() <= 1e-9 * np.abs(f).max()


def test_gauge_last_plane_area_weighted_mean_is_zero():
    p = W.make_problem((10, 9, 8), (1.5, 2.0, 1.0), (W.NN, W.PP, W.NN))
    x = O.solve(p, W.rhs(p, 4))
    wx = W.control_volumes(p.faces[0], p.bc[0], "C")
    wy = W.control_volumes(p.faces[1], p.bc[1], "C")
    last = x[-1]
    assert abs((wy[:, None] * wx[None, :] * last).sum()) <= 1e-13 * np.abs(last).max()


def _mms_errors(make, sizes):
    errs = []
    for n in sizes:
        p, f, u = make(n)
        x = O.solve(p, f)
        dv = p.volumes()
        e = O.gauge_normalise(p, x) - O.gauge_normalise(p, u)
        errs.append((np.sqrt((dv * e * e).sum() / dv.sum()), np.abs(e).max()))
    return np.array(errs)


def _mk_nn(n):
    p = W.make_problem((n, n, n), (1.5, 1.5, 1.5), (W.NN, W.NN, W.NN))
    f, u = W.mms_cos(p)
    return p, f, u


def _mk_dd_helm(n):
    # u = sin(pi x) sin(pi y) sin(pi z), (I - a L) u = (1 + 3 a pi^2) u
    alpha = 1e-2
    p = W.make_problem((n, n, n), (2.0, 1.0, 2.0), (W.DD, W.DD, W.DD), kind="helmholtz", alpha=alpha)
    xs = [W.centres(p.faces[d], p.bc[d], "C") for d in range(3)]
    sx, sy, sz = (np.sin(np.pi * x) for x in xs)
    u = sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    return p, (1 + 3 * alpha * np.pi ** 2) * u, u


def _mk_pnn(n):
    # u = cos(2 pi x) cos(pi y) cos(pi z), x periodic
    p = W.make_problem((n, n, n), (0.0, 2.0, 2.0), (W.PP, W.NN, W.NN))
    xs = [W.centres(p.faces[d], p.bc[d], "C") for d in range(3)]
    u = (np.cos(np.pi * xs[2])[:, None, None] * np.cos(np.pi * xs[1])[None, :, None]
         * np.cos(2 * np.pi * xs[0])[None, None, :])
    return p, -(4 + 1 + 1) * np.pi ** 2 * u, u


def _mk_nnp(n):
    # u = cos(pi x) cos(pi y) sin(2 pi z), z periodic (x, y stretched)
    p = W.make_problem((n, n, n), (1.5, 2.0, 0.0), (W.NN, W.NN, W.PP))
    xs = [W.centres(p.faces[d], p.bc[d], "C") for d in range(3)]
    u = (np.sin(2 * np.pi * xs[2])[:, None, None] * np.cos(np.pi * xs[1])[None, :, None]
         * np.cos(np.pi * xs[0])[None, None, :])
    return p, -(1 + 1 + 4) * np.pi ** 2 * u, u


@pytest.mark.parametrize("make", [_mk_nn, _mk_dd_helm, _mk_pnn, _mk_nnp], ids=["nnn", "ddd_helm", "pnn", "nnp"])
def test_mms_second_order(make):
    e = _mms_errors(make, [16, 32, 64])
    order_l2 = np.log2(e[:-1, 0] / e[1:, 0])
    order_max = np.log2(e[:-1, 1] / e[1:, 1])
    assert order_l2[-1] >= 1.9, order_l2
    assert order_max[-1] >= 1.75, order_max


# ---- implicit directions of the Helmholtz step (§2.1 L_I; §3) ---------------

IMPLICIT_CASES = [
    ((6, 5, 7), (1.5, 1.5, 1.5), (W.DD, W.NN, W.DD), ("C", "C", "C")),
    ((7, 6, 5), (0.0, 2.0, 2.0), (W.PP, W.DD, W.DD), ("F", "C", "F")),
    ((5, 8, 6), (2.0, 0.0, 1.0), (("N", "D"), W.PP, W.NN), ("C", "C", "C")),
    ((6, 6, 8), (1.0, 1.5, 0.0), (W.NN, W.NN, W.PP), ("C", "C", "C")),
]


@pytest.mark.parametrize("implicit", ["yz", "z"])
@pytest.mark.parametrize("case", IMPLICIT_CASES, ids=lambda c: "".join(x[0] + x[1] for x in c[2]) + "".join(c[3]))
def test_implicit_options_match_dense_lu(case, implicit):
    n, beta, bc, loc = case
    p = W.make_problem(n, beta, bc, loc=loc, kind="helmholtz", alpha=0.05, implicit=implicit)
    f = W.rhs(p, 17)
    assert O.relative_error(p, O.solve(p, f), O.solve_dense(p, f), norm="max") <= 5e-14


def test_z_only_lines_match_banded_solver():
    """I - alpha T_z on every (i, j) line, against LAPACK's banded solver
    (scipy.linalg.solve_banded) line by line."""
    from scipy.linalg import solve_banded
    p = W.make_problem((5, 4, 11), (1.0, 1.0, 2.0), (W.DD, W.NN, ("N", "D")), kind="helmholtz",
                       alpha=0.3, implicit="z")
    f = W.rhs(p, 5)
    x = O.solve(p, f)
    az, bz, cz, _ = O.operator_1d(p.faces[2], p.bc[2], p.loc[2])
    ab = np.zeros((3, len(bz)))
    ab[0, 1:] = -p.alpha * cz[:-1]
    ab[1] = 1.0 - p.alpha * bz
    ab[2, :-1] = -p.alpha * az[1:]
    for j in range(p.shape[1]):
        for i in range(p.shape[2]):
            ref = solve_banded((1, 1), ab, f[:, j, i])
            assert np.abs(x[:, j, i] - ref).max() <= 1e-14 * np.abs(ref).max()


def test_yz_solve_does_not_couple_x():
    """With x explicit, a right-hand side g(x) h(y, z) has the solution
    g(x) times the solution for h: every x index is its own 2-D problem."""
    p = W.make_problem((7, 6, 5), (1.5, 2.0, 1.0), (W.NN, W.DD, W.NN), kind="helmholtz", alpha=0.1,
                       implicit="yz")
    rng = np.random.default_rng(8)
    g = rng.standard_normal(p.shape[2])
    h = rng.standard_normal(p.shape[:2])
    x = O.solve(p, h[:, :, None] * g[None, None, :])
    xh = O.solve(p, np.repeat(h[:, :, None], p.shape[2], axis=2))[:, :, 0]
    assert np.abs(x - xh[:, :, None] * g[None, None, :]).max() <= 1e-13 * np.abs(x).max()


def _mk_yz_helm(n):
    # u = g(x) sin(pi y) sin(pi z) with an arbitrary g: x is not differentiated,
    # (I - a (d_yy + d_zz)) u = (1 + 2 a pi^2) u
    alpha = 0.1
    p = W.make_problem((n, n, n), (1.5, 1.0, 2.0), (W.NN, W.DD, W.DD), kind="helmholtz", alpha=alpha,
                       implicit="yz")
    xs = [W.centres(p.faces[d], p.bc[d], "C") for d in range(3)]
    g = 1.0 + xs[0] ** 3 - np.cos(5 * xs[0])
    u = np.sin(np.pi * xs[2])[:, None, None] * np.sin(np.pi * xs[1])[None, :, None] * g[None, None, :]
    return p, (1 + 2 * alpha * np.pi ** 2) * u, u


def _mk_z_helm(n):
    # u = g(x, y) sin(pi z), (I - a d_zz) u = (1 + a pi^2) u
    alpha = 0.1
    p = W.make_problem((n, n, n), (1.5, 1.0, 2.0), (W.PP, W.NN, W.DD), kind="helmholtz", alpha=alpha,
                       implicit="z")
    xs = [W.centres(p.faces[d], p.bc[d], "C") for d in range(3)]
    g = np.exp(xs[1])[:, None] * (2.0 + np.sin(2 * np.pi * xs[0]))[None, :]
    u = np.sin(np.pi * xs[2])[:, None, None] * g[None, :, :]
    return p, (1 + alpha * np.pi ** 2) * u, u


@pytest.mark.parametrize("make", [_mk_yz_helm, _mk_z_helm], ids=["yz_helm", "z_helm"])
def test_implicit_mms_second_order(make):
    e = _mms_errors(make, [16, 32, 64])
    order_l2 = np.log2(e[:-1, 0] / e[1:, 0])
    order_max = np.log2(e[:-1, 1] / e[1:, 1])
    assert order_l2[-1] >= 1.9, order_l2
    assert order_max[-1] >= 1.75, order_max

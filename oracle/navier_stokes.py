"""One Runge--Kutta substep of the incompressible Navier--Stokes solver on the
staggered grid (oracle; test infrastructure only).

§2.1, Eq. rk3: substep k of Wray's three-stage scheme with coefficients
alpha_k = (8/15, 5/12, 3/4), beta_k = (0, -17/60, -5/12), gamma_k = alpha_k +
beta_k advances the face velocity u^k and the pressure P^{k-1/2}:

    u**        = u^k + dt [alpha_k E^k + beta_k E^{k-1}
                           + gamma_k (-G P^{k-1/2} + nu L_I u^k)],
                 E^k = A u^k + nu L_E u^k    (explicit terms, kept for k+1)
    (I - c L_I) u* = u** - c L_I u^k,        c = gamma_k nu dt / 2
    L Phi      = D u* / (gamma_k dt)
    u^{k+1}    = u* - gamma_k dt G Phi
    P^{k+1/2}  = P^{k-1/2} + Phi - c L_I Phi

L = L_E + L_I splits the discrete Laplacian by direction: L_I holds none,
z, y and z, or all three directions (implicit 'none', 'z', 'yz', 'xyz').
For 'none' the Helmholtz step is the identity, u* = u**.

Grid and layouts are those of ``projection``: the pressure problem p is the
cell-centred Poisson problem (periodic or Neumann = wall boundaries); u, v, w
live on the faces normal to them, N face unknowns in a periodic direction
(face m between cells m and m+1, the last wrapping) or N - 1 between walls.
Velocity boundary conditions at walls: no penetration (the wall face carries
no normal velocity) and no slip (the tangential components vanish on the
wall: Dirichlet rows of the cell-centred operator, the mirrored-ghost row
of ``operator``).  The diffusion operator of a component is the
one-dimensional operator of §2.2.1 in each direction, face-located (loc F)
along the component's own direction.

The advection term A u = -div(u (x) u) (§2.1; the paper gives no stencil,
only that the discretisation is second order and conserves kinetic energy
semi-discretely) is taken in the symmetry-preserving finite-volume form:
the control volume of a face unknown is the half cells on both sides of
the face; the mass flux through each of its faces is the one that makes the
discrete continuity of that control volume the half-sum of the continuities
of the two cells (the mean of the two normal face velocities along the
component's own direction, the cell-width weighted mean of the two
transverse face velocities in the other directions), and the transported
velocity on it is the plain mean of the two neighbouring unknowns.  The
resulting operator is skew-symmetric in the volume-weighted inner product
for a discretely divergence-free field, so sum(vol u A u) = 0 per component
(kinetic energy is conserved by advection), which the tests pin.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .operator import _apply_1d, operator_1d
from .projection import _check, _dir, divergence, gradient
from .solver import solve

RK3_ALPHA = (8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0)
RK3_BETA = (0.0, -17.0 / 60.0, -5.0 / 12.0)
IMPLICIT = {"none": (), "z": (2,), "yz": (1, 2), "xyz": (0, 1, 2)}


def _axis(d):
    """Array axis of direction d (arrays are (Nz, Ny, Nx), x fastest)."""
    return 2 - d


def _take(q, axis, idx, n, periodic):
    """q at positions idx along axis; indices outside 0..n-1 wrap if the
    direction is periodic and read zero otherwise (a wall)."""
    idx = np.asarray(idx)
    if periodic:
        return np.take(q, idx % n, axis=axis)
    ok = ((idx >= 0) & (idx < n)).astype(np.float64)
    out = np.take(q, np.clip(idx, 0, n - 1), axis=axis)
    shape = [1] * q.ndim
    shape[axis] = idx.shape[0]
    return out * ok.reshape(shape)


def _along(vec, axis):
    shape = [1, 1, 1]
    shape[axis] = vec.shape[0]
    return vec.reshape(shape)


def velocity_problem(p, c, alpha=0.0, implicit="xyz"):
    """The problem of velocity component c (0 = u, 1 = v, 2 = w) on the
    pressure grid p: face-located along c, cell-centred elsewhere; periodic
    stays periodic, a wall direction gets zero (Dirichlet) velocity.  kind
    'helmholtz' with coefficient alpha and implicit directions, or 'poisson'
    (the plain Laplacian) for alpha = 0."""
    _check(p)
    bc = tuple(("P", "P") if p.bc[e][0] == "P" else ("D", "D") for e in range(3))
    loc = tuple("F" if e == c else "C" for e in range(3))
    if alpha == 0.0:
        return dataclasses.replace(p, bc=bc, loc=loc, kind="poisson", alpha=0.0, implicit="xyz")
    return dataclasses.replace(p, bc=bc, loc=loc, kind="helmholtz", alpha=float(alpha), implicit=implicit)


def laplacian_dirs(p, q, dirs):
    """Sum over directions in dirs of the one-dimensional operators of
    problem p applied to q (L_E or L_I of §2.1)."""
    out = np.zeros_like(q)
    for d in dirs:
        a, b, c, _ = operator_1d(p.faces[d], p.bc[d], p.loc[d])
        out += _apply_1d(q, a, b, c, p.bc[d][0] == "P", _axis(d))
    return out


def velocity_volumes(p, c):
    """Control volume of each unknown of component c (for the energy norm)."""
    vols = []
    for e in range(3):
        per, wdt, dc = _dir(p, e)
        vols.append(dc if e == c else wdt)
    return vols[2][:, None, None] * vols[1][None, :, None] * vols[0][None, None, :]


def advection(p, u, v, w):
    """(A u, A v, A w): -div(u (x) u) on the face unknowns of each component,
    in the symmetry-preserving flux form described above."""
    _check(p)
    q = tuple(np.asarray(x, dtype=np.float64) for x in (u, v, w))
    ncell = [len(p.faces[d]) - 1 for d in range(3)]
    info = [_dir(p, d) for d in range(3)]         # (periodic, cell widths, face spacings)
    out = []
    for c in range(3):
        Q = q[c]
        per_c, wc, hc = info[c]
        ac = _axis(c)
        nf = hc.shape[0]                             # face unknowns along c
        m = np.arange(nf)
        # along c: the fluxes through the cell centres on both sides of face m
        u_lo = 0.5 * (_take(Q, ac, m - 1, nf, per_c) + Q)
        u_hi = 0.5 * (Q + _take(Q, ac, m + 1, nf, per_c))
        res = -(u_hi * u_hi - u_lo * u_lo) / _along(hc, ac)
        for e in range(3):
            if e == c:
                continue
            per_e, we, he = info[e]
            ae = _axis(e)
            Qe = q[e]                                 # face-located along e, centred along c
            nfe = he.shape[0]
            # mass flux through the e-faces of the control volume of face m:
            # both cells' transverse velocities weighted by their widths
            c0 = np.take(Qe, m, axis=ac)
            c1 = np.take(Qe, (m + 1) % ncell[c], axis=ac)
            flux = 0.5 * (_along(wc[m], ac) * c0 + _along(wc[(m + 1) % ncell[c]], ac) * c1)
            j = np.arange(ncell[e])
            f_hi = _take(flux, ae, j, nfe, per_e)    # e-face j above cell j
            f_lo = _take(flux, ae, j - 1, nfe, per_e)
            t_hi = 0.5 * (Q + _take(Q, ae, j + 1, ncell[e], per_e))
            t_lo = 0.5 * (Q + _take(Q, ae, j - 1, ncell[e], per_e))
            res = res - (f_hi * t_hi - f_lo * t_lo) / (_along(hc, ac) * _along(we, ae))
        out.append(res)
    return tuple(out)


def rk3_coefficients(k):
    """(alpha_k, beta_k, gamma_k) of substep k = 1, 2, 3."""
    a, b = RK3_ALPHA[k - 1], RK3_BETA[k - 1]
    return a, b, a + b


def rk3_substep(p, k, dt, nu, implicit, u, v, w, e_prev, P):
    """Substep k of Eq. rk3.  e_prev: the explicit terms E^{k-1} per
    component (unused for k = 1).  Returns (u^{k+1}, v^{k+1}, w^{k+1}),
    E^k, P^{k+1/2} and Phi."""
    _check(p)
    if k not in (1, 2, 3):
        raise ValueError("substep k must be 1, 2 or 3")
    if implicit not in IMPLICIT:
        raise ValueError(f"unknown implicit directions {implicit!r}")
    a, b, g = rk3_coefficients(k)
    dirs_i = IMPLICIT[implicit]
    dirs_e = tuple(d for d in range(3) if d not in dirs_i)
    cn = g * nu * dt / 2.0
    q = (u, v, w)
    adv = advection(p, u, v, w)
    gp = gradient(p, P)
    e_new, ustar = [], []
    for c in range(3):
        pc = velocity_problem(p, c)
        e_c = adv[c] + nu * laplacian_dirs(pc, q[c], dirs_e)
        li = laplacian_dirs(pc, q[c], dirs_i)
        udd = q[c] + dt * (a * e_c + g * (-gp[c] + nu * li))
        if b != 0.0:
            udd = udd + dt * b * e_prev[c]
        if dirs_i:
            us = solve(velocity_problem(p, c, cn, implicit), udd - cn * li)
        else:
            us = udd
        e_new.append(e_c)
        ustar.append(us)
    phi = solve(p, divergence(p, *ustar) / (g * dt))
    gphi = gradient(p, phi)
    unew = tuple(ustar[c] - g * dt * gphi[c] for c in range(3))
    pnew = P + phi - cn * laplacian_dirs(p, phi, dirs_i)
    return unew, tuple(e_new), pnew, phi


def rk3_step(p, dt, nu, implicit, u, v, w, P):
    """A full time step: substeps 1, 2, 3 (u^1 = u^n, u^4 = u^{n+1})."""
    e = (None, None, None)
    vel = (u, v, w)
    for k in (1, 2, 3):
        vel, e, P, _ = rk3_substep(p, k, dt, nu, implicit, *vel, e, P)
    return vel, P

"""Projection step on the staggered grid (oracle; test infrastructure only).

§2.1: the velocity components live on the cell faces normal to them and the
pressure at the cell centres; the intermediate velocity u* is projected onto
the discretely divergence-free fields by solving the Poisson equation for the
pressure correction and subtracting its gradient:

    L phi = D u*,    u = u* - G phi,    so that  D u = D u* - D G phi = 0

because the finite-volume divergence D and gradient G compose to the
Laplacian of Eq. poisson-fd2: (D G phi)_i = (1/dx_i) [(phi_{i+1} - phi_i) /
dx_{i+1/2} - (phi_i - phi_{i-1}) / dx_{i-1/2}].  §4.1 checks that the
projected field of a white-noise velocity is divergence-free to machine
precision.

Boundaries per direction: periodic, or walls with no penetration (the
normal velocity on a wall face is zero and not an unknown; the pressure
operator then has the Neumann rows).  Component layouts (x fastest):
u (Nz, Ny, Nux), v (Nz, Nvy, Nx), w (Nwz, Ny, Nx), where the face count of
a direction is N (periodic: face m between cells m and m+1, the last one
wrapping) or N - 1 (walls: the interior faces).  The pressure problem is the
cell-centred Poisson problem with the same faces and P / N boundaries.
"""
from __future__ import annotations

import numpy as np

from .solver import solve


def _dir(p, d):
    """(periodic, cell widths, centre distances of the face unknowns) of
    direction d of the pressure problem p."""
    faces = np.asarray(p.faces[d], dtype=np.float64)
    wdt = np.diff(faces)
    per = p.bc[d][0] == "P"
    xc = 0.5 * (faces[:-1] + faces[1:])
    dc = np.diff(xc)                           # between cells m and m+1, m < N-1
    if per:
        dc = np.concatenate([dc, [0.5 * (wdt[0] + wdt[-1])]])
    return per, wdt, dc


def face_shapes(p):
    """Array shapes of u, v, w for the pressure problem p."""
    nz, ny, nx = p.shape
    nf = [n if p.bc[d][0] == "P" else n - 1 for d, n in enumerate((nx, ny, nz))]
    return (nz, ny, nf[0]), (nz, nf[1], nx), (nf[2], ny, nx)


def _check(p):
    if p.kind != "poisson" or any(l != "C" for l in p.loc):
        raise ValueError("the projection needs the cell-centred pressure Poisson problem")
    for d in range(3):
        if p.bc[d] not in (("P", "P"), ("N", "N")):
            raise ValueError("pressure boundaries must be periodic or Neumann (walls)")


def divergence(p, u, v, w):
    """(D u)_{ijk}: the net flux out of cell (i, j, k) per unit volume."""
    _check(p)
    out = np.zeros(p.shape)
    for d, (comp, axis) in enumerate(((u, 2), (v, 1), (w, 0))):
        per, wdt, _ = _dir(p, d)
        q = np.moveaxis(np.asarray(comp, dtype=np.float64), axis, -1)
        n = wdt.shape[0]
        # face values on both sides of every cell: upper face m, lower face m-1
        if per:
            hi = q
            lo = np.roll(q, 1, axis=-1)
        else:
            z = np.zeros(q.shape[:-1] + (1,))
            hi = np.concatenate([q, z], axis=-1)     # upper wall face: zero
            lo = np.concatenate([z, q], axis=-1)     # lower wall face: zero
        out += np.moveaxis((hi - lo) / wdt.reshape((1,) * (q.ndim - 1) + (n,)), -1, axis)
    return out


def gradient(p, phi):
    """(G phi) on the face unknowns: (phi_{m+1} - phi_m) / dx_{m+1/2} for the
    face between cells m and m+1; returns (gx, gy, gz) in the u, v, w layouts."""
    _check(p)
    phi = np.asarray(phi, dtype=np.float64)
    out = []
    for d, axis in ((0, 2), (1, 1), (2, 0)):
        per, _, dc = _dir(p, d)
        q = np.moveaxis(phi, axis, -1)
        if per:
            g = (np.roll(q, -1, axis=-1) - q) / dc
        else:
            g = (q[..., 1:] - q[..., :-1]) / dc
        out.append(np.moveaxis(g, -1, axis))
    return tuple(out)


def project(p, u, v, w):
    """Return (u, v, w, phi): the projected velocity and the pressure
    correction solving L phi = D u* (gauge of the tensor-product solve)."""
    rhs = divergence(p, u, v, w)
    phi = solve(p, rhs)
    gx, gy, gz = gradient(p, phi)
    return u - gx, v - gy, w - gz, phi


def divergence_flux_bound(p, u, v, w):
    """sum over directions of max|face value| / min(cell width): the size of
    the divergence that rounding errors of the face values can leave."""
    s = 0.0
    for d, comp in enumerate((u, v, w)):
        _, wdt, _ = _dir(p, d)
        s += np.abs(comp).max() / wdt.min()
    return s

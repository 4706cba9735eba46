"""One-dimensional and three-dimensional discrete Laplacians (oracle; test
infrastructure only).

§2.2.1, Eq. poisson-fd2: at unknown i,
    (1/dx_i) [ (phi_{i+1} - phi_i)/dx_{i+1/2} - (phi_i - phi_{i-1})/dx_{i-1/2} ] = f_i,
with dx_i the control-volume width of unknown i and dx_{i+1/2} the distance
between unknowns i and i+1, so that (Eq. tridiagonal-coefficients)
    a_i = 1/(dx_i dx_{i-1/2}),  c_i = 1/(dx_i dx_{i+1/2}),  b_i = -(a_i + c_i).
The paper only says the first and last rows are modified by the boundary
conditions and that periodic boundaries add cyclic corner entries; the rows
used here are the ghost-cell rows (a reading of the paper, not its text):

* cell-centred unknowns, Neumann wall: zero flux through the wall face, the
  wall coupling is dropped and b_1 = -c_1;
* cell-centred unknowns, Dirichlet wall: mirrored ghost phi_0 = -phi_1 at
  distance dx_{1/2} = dx_1, so b_1 = -c_1 - 2/dx_1^2;
* periodic: dx_{1/2} = dx_{N+1/2} = (dx_1 + dx_N)/2, corner entries
  T[1,N] = a_1 and T[N,1] = c_N;
* face-located unknowns (velocities) between Dirichlet walls: the N-1
  interior faces, control volume = distance between the adjacent cell centres,
  neighbour distances = cell widths, zero wall values (coupling dropped);
  periodic face unknowns wrap the same way.

§2.2.2: T = T_x (x) I_y (x) I_z + I_x (x) T_y (x) I_z + I_x (x) I_y (x) T_z.
Arrays here are (Nz, Ny, Nx) with x fastest.

§2.1: the implicit diffusion operator L_I of the Helmholtz step may hold all
three directions (xyz), only y and z (yz) or only z (z); the terms of the
other directions are dropped from the Kronecker sum.
"""
from __future__ import annotations

import numpy as np


def has_null(bc, loc="C") -> bool:
    """True if the 1-D operator has a constant null mode (periodic, or
    Neumann at both ends of a cell-centred direction)."""
    if bc[0] == "P":
        return True
    return loc == "C" and bc[0] == "N" and bc[1] == "N"


def operator_1d(faces, bc, loc="C"):
    """Return (a, b, c, vol) for one direction.

    Row i of T reads a[i] phi[i-1] + b[i] phi[i] + c[i] phi[i+1]; for a
    periodic direction a[0] multiplies phi[N-1] and c[N-1] multiplies phi[0]
    (the cyclic corners); otherwise a[0] = c[N-1] = 0.  vol[i] is the
    control-volume width dx_i (the diagonal of D).
    """
    faces = np.asarray(faces, dtype=np.float64)
    w = np.diff(faces)                      # cell widths
    if np.any(w <= 0):
        raise ValueError("faces must be strictly increasing")
    periodic = bc[0] == "P"
    if periodic != (bc[1] == "P"):
        raise ValueError("periodic boundaries must be paired")
    if loc == "C":
        n = len(w)
        vol = w.copy()
        xc = 0.5 * (faces[:-1] + faces[1:])
        dc = np.diff(xc)                    # dx_{i+1/2}, i = 1..N-1
        if periodic:
            dlo = dhi = 0.5 * (w[0] + w[-1])
        else:
            dlo, dhi = w[0], w[-1]          # mirrored ghost centre
        dm = np.concatenate([[dlo], dc])    # dx_{i-1/2}
        dp = np.concatenate([dc, [dhi]])    # dx_{i+1/2}
        a = 1.0 / (vol * dm)
        c = 1.0 / (vol * dp)
        b = -(a + c)
        if not periodic:
            for side, coef in ((0, a), (n - 1, c)):
                kind = bc[0] if side == 0 else bc[1]
                if kind == "N":
                    b[side] += coef[side]
                elif kind == "D":
                    b[side] -= coef[side]
                else:
                    raise ValueError(f"unknown boundary condition {kind!r}")
                coef[side] = 0.0
        return a, b, c, vol
    if loc == "F":
        if periodic:
            n = len(w)                      # unknown m sits on face x_{m+1}; x_N == x_0
            wn = np.roll(w, -1)             # width of the cell above face m
            vol = 0.5 * (w + wn)
            a = 1.0 / (vol * w)
            c = 1.0 / (vol * wn)
            b = -(a + c)
            return a, b, c, vol
        if bc[0] == "D" and bc[1] == "D":
            vol = 0.5 * (w[:-1] + w[1:])    # N-1 interior faces
            a = 1.0 / (vol * w[:-1])
            c = 1.0 / (vol * w[1:])
            b = -(a + c)
            a[0] = 0.0                      # wall value is zero
            c[-1] = 0.0
            return a, b, c, vol
        raise ValueError("face-located unknowns need periodic or Dirichlet-Dirichlet walls")
    raise ValueError(f"unknown location {loc!r}")


def dense_1d(a, b, c, periodic: bool) -> np.ndarray:
    """The N x N matrix T of a one-dimensional operator."""
    n = len(b)
    T = np.zeros((n, n))
    for i in range(n):
        T[i, i] += b[i]
        if i > 0:
            T[i, i - 1] += a[i]
        if i < n - 1:
            T[i, i + 1] += c[i]
    if periodic and n > 1:
        T[0, n - 1] += a[0]
        T[n - 1, 0] += c[n - 1]
    return T


def _ops(p):
    out = []
    for d in range(3):
        a, b, c, vol = operator_1d(p.faces[d], p.bc[d], p.loc[d])
        out.append((a, b, c, vol, p.bc[d][0] == "P"))
    return out


def _apply_1d(x, a, b, c, periodic, axis):
    """Apply a tridiagonal (optionally cyclic) operator along `axis`."""
    x = np.moveaxis(x, axis, -1)
    y = b * x
    y[..., 1:] += a[1:] * x[..., :-1]
    y[..., :-1] += c[:-1] * x[..., 1:]
    if periodic and x.shape[-1] > 1:
        y[..., 0] += a[0] * x[..., -1]
        y[..., -1] += c[-1] * x[..., 0]
    return np.moveaxis(y, -1, axis)


def implicit_dirs(p):
    """Directions (0 = x, 1 = y, 2 = z) in the operator of problem p."""
    return {"xyz": (0, 1, 2), "yz": (1, 2), "z": (2,)}[getattr(p, "implicit", "xyz")]


def apply_operator(p, phi: np.ndarray) -> np.ndarray:
    """A phi for problem p: the Kronecker-sum Laplacian of §2.2.2, or
    (I - alpha L_I) phi for a Helmholtz problem."""
    ops = _ops(p)
    lap = np.zeros_like(phi)
    for d, axis in ((0, 2), (1, 1), (2, 0)):
        if d not in implicit_dirs(p):
            continue
        a, b, c, _, per = ops[d]
        lap += _apply_1d(phi, a, b, c, per, axis)
    if p.kind == "helmholtz":
        return phi - p.alpha * lap
    return lap


def residual(p, f: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """f - A phi (the algebraic residual checked in §4.1)."""
    return f - apply_operator(p, phi)


def assemble_3d(p) -> np.ndarray:
    """Dense matrix of the three-dimensional operator with unknowns ordered
    (k, j, i), i fastest: T = I_z (x) I_y (x) T_x + I_z (x) T_y (x) I_x +
    T_z (x) I_y (x) I_x (the Kronecker sum of §2.2.2 in this ordering)."""
    ops = _ops(p)
    Ts = [dense_1d(a, b, c, per) for (a, b, c, _, per) in ops]
    Ix, Iy, Iz = (np.eye(T.shape[0]) for T in Ts)
    # a direction outside L_I contributes nothing to the sum
    Ts = [T if d in implicit_dirs(p) else np.zeros_like(T) for d, T in enumerate(Ts)]
    T = (np.kron(Iz, np.kron(Iy, Ts[0])) + np.kron(Iz, np.kron(Ts[1], Ix))
         + np.kron(Ts[2], np.kron(Iy, Ix)))
    if p.kind == "helmholtz":
        return np.eye(T.shape[0]) - p.alpha * T
    return T

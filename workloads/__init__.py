"""Seeded synthetic inputs shared by the tests, ``bench.py`` and ``smoke()``.

This module generates grids (tanh-stretched face coordinates, Eq. tanh_stretching
of §4.1), boundary-condition draws and right-hand sides with the shapes of the
paper's workloads.  It holds none of the solver's arithmetic: both the HIP
library and the CPU oracle receive the face coordinates and right-hand sides
produced here as plain inputs.

Boundary conditions are encoded per direction as a pair ``(lower, upper)`` of
``'P'`` (periodic, must be paired), ``'N'`` (homogeneous Neumann) or ``'D'``
(homogeneous Dirichlet).  The unknown location per direction is ``'C'``
(cell centre, pressure-like) or ``'F'`` (face, velocity-like; with Dirichlet
walls a face direction of ``n`` cells carries ``n - 1`` interior unknowns).
Fields are ``numpy`` arrays of shape ``(Nz, Ny, Nx)`` (x fastest).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Sequence, Tuple

import numpy as np

BC = Tuple[str, str]


def tanh_faces(n: int, beta: float, length: float = 1.0) -> np.ndarray:
    """Face coordinates x_0..x_n of an n-cell direction on [0, length].

    Eq. tanh_stretching (§4.1): x(xi) = L/2 (1 + tanh(b (xi - 1/2)) / tanh(b/2))
    with xi = k/n, clustered at both ends; b -> 0 gives the uniform grid.
    (The paper calls the stretching parameter alpha; here it is beta, because
    alpha is the Helmholtz coefficient.)
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    xi = np.arange(n + 1, dtype=np.float64) / n
    if beta == 0.0:
        x = length * xi
    else:
        x = 0.5 * length * (1.0 + np.tanh(beta * (xi - 0.5)) / np.tanh(0.5 * beta))
    x[0] = 0.0
    x[-1] = length
    return x


def n_unknowns(n_cells: int, bc: BC, loc: str) -> int:
    """Unknowns along one direction: n cells, or n-1 interior faces for a
    face-located direction between two Dirichlet walls."""
    if loc == "F" and bc[0] == "D" and bc[1] == "D":
        return n_cells - 1
    return n_cells


def control_volumes(faces: np.ndarray, bc: BC, loc: str) -> np.ndarray:
    """Control-volume width of each unknown along one direction: the cell
    width for a cell-centred direction, the distance between the two adjacent
    cell centres for a face-located one (periodic: wrapped)."""
    w = np.diff(faces)
    if loc == "C":
        return w.copy()
    if bc[0] == "P":
        return 0.5 * (w + np.roll(w, -1))  # face i+1/2 between cells i and i+1 (wrapped)
    return 0.5 * (w[:-1] + w[1:])


@dataclass
class Problem:
    """One constant-coefficient Poisson or Helmholtz problem on a stretched grid.

    kind 'poisson': L phi = f.  kind 'helmholtz': (I - alpha L_I) u = f, with
    L_I the Laplacian restricted to the directions treated implicitly:
    implicit 'xyz' (L), 'yz' (L_y + L_z) or 'z' (L_z).
    """

    n: Tuple[int, int, int]
    faces: Tuple[np.ndarray, np.ndarray, np.ndarray]
    bc: Tuple[BC, BC, BC]
    loc: Tuple[str, str, str] = ("C", "C", "C")
    kind: str = "poisson"
    alpha: float = 0.0
    name: str = ""
    implicit: str = "xyz"

    @property
    def shape(self) -> Tuple[int, int, int]:
        """Array shape (Nz, Ny, Nx) of the unknowns."""
        nx, ny, nz = (n_unknowns(self.n[d], self.bc[d], self.loc[d]) for d in range(3))
        return (nz, ny, nx)

    @property
    def dof(self) -> int:
        s = self.shape
        return s[0] * s[1] * s[2]

    def volumes(self) -> np.ndarray:
        """Control volumes dV(k, j, i) = vx_i * vy_j * vz_k, shape (Nz, Ny, Nx)."""
        vx, vy, vz = (control_volumes(self.faces[d], self.bc[d], self.loc[d]) for d in range(3))
        return vz[:, None, None] * vy[None, :, None] * vx[None, None, :]

    @property
    def singular(self) -> bool:
        """Poisson with a constant null mode: periodic or Neumann-Neumann in all
        three directions (a face-located Dirichlet direction has no null mode)."""
        if self.kind != "poisson":
            return False
        return all(self.bc[d] in (("P", "P"), ("N", "N")) for d in range(3))


def make_problem(n, beta, bc, loc=("C", "C", "C"), kind="poisson", alpha=0.0,
                 length=(1.0, 1.0, 1.0), name="", implicit="xyz") -> Problem:
    """Build a Problem from per-direction cell counts and stretching; a
    periodic direction is always uniform."""
    if implicit not in ("xyz", "yz", "z"):
        raise ValueError(f"unknown implicit directions {implicit!r}")
    if implicit != "xyz" and kind != "helmholtz":
        raise ValueError("only a Helmholtz problem can leave directions explicit")
    faces = []
    for d in range(3):
        b = 0.0 if bc[d][0] == "P" else float(beta[d])
        faces.append(tanh_faces(int(n[d]), b, float(length[d])))
    return Problem(tuple(int(v) for v in n), tuple(faces), tuple(tuple(b) for b in bc),
                   tuple(loc), kind, float(alpha), name, implicit)


def project_compatible(p: Problem, f: np.ndarray) -> np.ndarray:
    """Remove the volume-weighted mean sum(dV f)/sum(dV) of a right-hand side
    of a singular problem (the left null vector of the operator is dV)."""
    if not p.singular:
        return f
    dv = p.volumes()
    return f - (dv * f).sum() / dv.sum()


def rhs(p: Problem, seed: int, dist: str = "normal") -> np.ndarray:
    """Seeded right-hand side of shape p.shape: 'normal' N(0,1) or 'uniform'
    U[-1, 1]; compatibility-projected for singular problems."""
    rng = np.random.default_rng(seed)
    if dist == "normal":
        f = rng.standard_normal(p.shape)
    elif dist == "uniform":
        f = rng.uniform(-1.0, 1.0, p.shape)
    else:
        raise ValueError(dist)
    return np.ascontiguousarray(project_compatible(p, f))


def centres(faces: np.ndarray, bc: BC, loc: str) -> np.ndarray:
    """Coordinates of the unknowns along one direction (cell centres, or the
    faces carrying unknowns)."""
    if loc == "C":
        return 0.5 * (faces[:-1] + faces[1:])
    if bc[0] == "P":
        return faces[1:].copy()
    return faces[1:-1].copy()


# ---------------------------------------------------------------------------
# The workloads: small verification case, channel-like Poisson, implicit
# diffusion Helmholtz, batched uneven problems and the serving families.
# ---------------------------------------------------------------------------

NN = ("N", "N")
DD = ("D", "D")
PP = ("P", "P")


def cavity32() -> Problem:
    """32^3 Poisson, Neumann walls in x, y, z, tanh beta = 1.5, [0,1]^3."""
    return make_problem((32, 32, 32), (1.5, 1.5, 1.5), (NN, NN, NN), name="cavity32_nnn_b1.5")


def cavity32_mms() -> Tuple[Problem, np.ndarray, np.ndarray]:
    """Manufactured case on cavity32: u = cos(pi x) cos(pi y) cos(pi z),
    f = -3 pi^2 u at the unknowns; returns (problem, f, u)."""
    p = cavity32()
    return (p,) + mms_cos(p)


def mms_cos(p: Problem):
    """Neumann-compatible manufactured solution u = prod cos(pi x_d / L_d) and its
    continuous Laplacian f at the unknowns (f projected to zero weighted mean)."""
    xs = [centres(p.faces[d], p.bc[d], p.loc[d]) for d in range(3)]
    L = [p.faces[d][-1] for d in range(3)]
    cx, cy, cz = (np.cos(np.pi * xs[d] / L[d]) for d in range(3))
    u = cz[:, None, None] * cy[None, :, None] * cx[None, None, :]
    lap = -sum((np.pi / L[d]) ** 2 for d in range(3)) * u
    return project_compatible(p, lap), u


def channel256() -> Problem:
    """256^3 channel-like Poisson: x uniform periodic, y and z Neumann walls
    with tanh beta = 2.0."""
    return make_problem((256, 256, 256), (0.0, 2.0, 2.0), (PP, NN, NN), name="channel256_pnn_b2")


def helmholtz_velocity(component: str, n=(1024, 768, 512), beta=2.0, alpha=1e-4) -> Problem:
    """Implicit-diffusion Helmholtz (I - alpha L) u = f for one staggered
    velocity component on the 1024x768x512 channel (x periodic uniform, y and z
    Dirichlet walls stretched with tanh beta): 'u' lives on x-faces, 'v' on
    y-faces (n_y - 1 unknowns), 'w' on z-faces (n_z - 1 unknowns)."""
    loc = {"u": ("F", "C", "C"), "v": ("C", "F", "C"), "w": ("C", "C", "F")}[component]
    return make_problem(n, (0.0, beta, beta), (PP, DD, DD), loc=loc, kind="helmholtz",
                        alpha=alpha, name=f"helmholtz_{component}_{n[0]}x{n[1]}x{n[2]}")


def helmholtz3(n=(1024, 768, 512)):
    """The three velocity components of the implicit-diffusion workload, with
    right-hand-side seeds 31, 32, 33."""
    return [(helmholtz_velocity(c, n), 31 + i) for i, c in enumerate("uvw")]


XY_BCS = (PP, NN, DD, ("N", "D"))
Z_BCS = (NN, DD, ("N", "D"))


def random_problem(rng: np.random.Generator, lo: int, hi: int, beta_max=2.5,
                   kind="poisson", alpha=0.0, name="") -> Problem:
    """One randomly drawn problem: each dimension uniform in [lo, hi], one beta
    in U[0, beta_max] for every non-periodic direction, BC per direction from
    {P, NN, DD, ND} in x, y and {NN, DD, ND} in z (z is the Thomas direction)."""
    n = tuple(int(v) for v in rng.integers(lo, hi + 1, size=3))
    beta = float(rng.uniform(0.0, beta_max))
    bcx = XY_BCS[int(rng.integers(len(XY_BCS)))]
    bcy = XY_BCS[int(rng.integers(len(XY_BCS)))]
    bcz = Z_BCS[int(rng.integers(len(Z_BCS)))]
    return make_problem(n, (beta, beta, beta), (bcx, bcy, bcz), kind=kind, alpha=alpha, name=name)


def batch64(seed: int = 4, count: int = 64, lo: int = 48, hi: int = 192):
    """Batched uneven solves: `count` independent Poisson problems with each
    dimension drawn from [lo, hi]; returns [(problem, rhs_seed)]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        p = random_problem(rng, lo, hi, name=f"batch{seed}_{i}")
        out.append((p, seed * 1000 + i))
    return out


SERVING_SIZES = (64, 96, 128, 160, 192, 256, 320, 384, 448, 512)


def serving_families(seed: int = 5, sizes: Sequence[int] = SERVING_SIZES):
    """Ten cubic grid families for the serving loop, each with its own beta in
    U[0, 2.5] and boundary-condition mix."""
    rng = np.random.default_rng(seed)
    fam = []
    for s in sizes:
        beta = float(rng.uniform(0.0, 2.5))
        bcx = XY_BCS[int(rng.integers(len(XY_BCS)))]
        bcy = XY_BCS[int(rng.integers(len(XY_BCS)))]
        bcz = Z_BCS[int(rng.integers(len(Z_BCS)))]
        fam.append(make_problem((s, s, s), (beta, beta, beta), (bcx, bcy, bcz), name=f"family{s}"))
    return fam


# ---------------------------------------------------------------------------
# Projection step inputs: velocity components on the faces of a pressure grid.
# ---------------------------------------------------------------------------

def velocity_shapes(p: Problem):
    """Shapes of u, v, w on the faces of the cell-centred pressure problem p:
    a direction carries N face unknowns if periodic (face m between cells m
    and m+1, the last wrapping) or N - 1 between walls (interior faces)."""
    nz, ny, nx = p.shape
    nf = [n if p.bc[d][0] == "P" else n - 1 for d, n in enumerate((nx, ny, nz))]
    return (nz, ny, nf[0]), (nz, nf[1], nx), (nf[2], ny, nx)


def white_noise_velocity(p: Problem, seed: int):
    """Seeded N(0, 1) values on every face unknown (a white-noise velocity
    field, as in the divergence test of §4.1)."""
    rng = np.random.default_rng(seed)
    return tuple(np.ascontiguousarray(rng.standard_normal(s)) for s in velocity_shapes(p))


def channel_pressure(n=(64, 48, 40), beta=2.0) -> Problem:
    """Pressure grid of a channel: x periodic uniform, walls in y and z
    (pressure Neumann), tanh-stretched."""
    return make_problem(n, (0.0, beta, beta), (PP, NN, NN), name=f"channel_p_{n[0]}x{n[1]}x{n[2]}")

"""The three-dimensional tensor-product--Thomas solve (oracle; test
infrastructure only).

Solution steps of the procedure of §2.2.2 (also Algorithm 1, solution part,
without the transposes, which only redistribute data):

2.1  f^(x)  = (Q_x^{-1} (x) I_y (x) I_z) f                    (Eq. forward-xy)
2.2  f^(xy) = (I_x (x) Q_y^{-1} (x) I_z) f^(x)
2.3  (lambda_ij I_z + T_z) phi^(xy)_ij = f^(xy)_ij, lambda_ij = lambda_x,i + lambda_y,j,
     one Thomas solve per (i, j) line
2.4  phi^(x) = (I_x (x) Q_y (x) I_z) phi^(xy)                  (Eq. inverse-xy)
2.5  phi     = (Q_x (x) I_y (x) I_z) phi^(x)

Helmholtz (I - alpha T) u = f uses the same eigenvectors with a constant
modal shift (end of §2.2.2): line (i, j) solves
(sigma + tau (lambda_ij + T_z)) u^ = f^ with sigma = 1, tau = -alpha;
Poisson is sigma = 0, tau = 1.

Implicit directions (§2.1, L_I of the Helmholtz step; §3: with y and z
implicit the x transforms are omitted, with only z the solve is the
tridiagonal one alone): a direction outside L_I is not transformed and adds
no eigenvalue to the line shift.

Gauge (§3): for a Poisson problem with a constant null mode, the line whose
shift is lambda_x = lambda_y = 0 has a vanishing final pivot; its last modal
unknown is set to zero and back substitution proceeds from there.

A periodic z direction makes every line cyclic; those lines are solved by
their plain definition (dense LU per line), with the same gauge on the
singular line (last unknown zero, last equation dropped).
"""
from __future__ import annotations

import numpy as np

from .eig import eig_direction
from .operator import operator_1d, has_null


def thomas_lines(az, bz, cz, lam, sigma, tau, rhs, pin=None):
    """Solve (sigma + tau (lam + T_z)) x = rhs for every line at once.

    rhs has shape (Nz,) + lam.shape; T_z has sub-diagonal az, diagonal bz,
    super-diagonal cz (az[0] and cz[-1] unused).  Plain Thomas algorithm:
    forward elimination then back substitution.  `pin` is the index tuple of
    the line whose final pivot vanishes; its last unknown is set to zero.
    Returns (x, last_pivot).
    """
    nz = len(bz)
    cp = np.empty_like(rhs)
    dp = np.empty_like(rhs)
    x = np.empty_like(rhs)
    with np.errstate(divide="ignore", invalid="ignore"):
        den = sigma + tau * (lam + bz[0])
        cp[0] = tau * cz[0] / den if nz > 1 else 0.0
        dp[0] = rhs[0] / den
        for k in range(1, nz):
            den = sigma + tau * (lam + bz[k]) - tau * az[k] * cp[k - 1]
            cp[k] = (tau * cz[k] / den) if k < nz - 1 else 0.0
            dp[k] = (rhs[k] - tau * az[k] * dp[k - 1]) / den
    last_pivot = np.array(den, copy=True)
    x[nz - 1] = dp[nz - 1]
    if pin is not None:
        x[(nz - 1,) + tuple(pin)] = 0.0
    for k in range(nz - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x, last_pivot


def cyclic_lines(az, bz, cz, lam, sigma, tau, rhs, pin=None):
    """Solve (sigma + tau (lam + T_z)) x = rhs for every line when z is
    periodic: T_z is cyclic (az[0] couples to x[nz-1], cz[nz-1] to x[0]).
    The plain definition: a dense LU solve of each line's matrix (no cyclic
    reduction).  On the pinned line of a singular problem the last unknown is
    set to zero and the last equation dropped, as the final-pivot gauge of §3
    does for the Thomas lines.  Returns x."""
    from .operator import dense_1d
    nz = len(bz)
    shape = rhs.shape
    lamf = np.broadcast_to(lam, shape[1:]).reshape(-1)
    R = rhs.reshape(nz, -1).T                      # (lines, nz)
    X = np.empty_like(R)
    T = dense_1d(az, bz, cz, True)
    eye = np.eye(nz)
    pin_flat = None if pin is None else int(np.ravel_multi_index(tuple(pin), shape[1:]))
    chunk = max(1, (1 << 22) // (nz * nz))         # lines per batched solve
    for s in range(0, R.shape[0], chunk):
        e = min(R.shape[0], s + chunk)
        M = sigma * eye + tau * (lamf[s:e, None, None] * eye + T)
        if pin_flat is not None and s <= pin_flat < e:
            M[pin_flat - s] = eye                  # placeholder row set; solved apart below
        X[s:e] = np.linalg.solve(M, R[s:e, :, None])[:, :, 0]
    if pin_flat is not None:
        M = sigma * eye + tau * (lamf[pin_flat] * eye + T)
        X[pin_flat, :nz - 1] = np.linalg.solve(M[:nz - 1, :nz - 1], R[pin_flat, :nz - 1])
        X[pin_flat, nz - 1] = 0.0
    return X.T.reshape(shape)


def _coeffs(p):
    if p.kind == "poisson":
        return 0.0, 1.0
    if p.kind == "helmholtz":
        return 1.0, -p.alpha
    raise ValueError(p.kind)


class Plan:
    """Initialization steps 1.1-1.3 for x and y, and T_z, for one problem."""

    def __init__(self, p):
        self.p = p
        imp = getattr(p, "implicit", "xyz")
        self.tx = imp == "xyz"             # x transformed
        self.ty = imp in ("xyz", "yz")     # y transformed
        self.zper = p.bc[2][0] == "P"
        self.ex = eig_direction(p.faces[0], p.bc[0], p.loc[0]) if self.tx else None
        self.ey = eig_direction(p.faces[1], p.bc[1], p.loc[1]) if self.ty else None
        self.az, self.bz, self.cz, _ = operator_1d(p.faces[2], p.bc[2], p.loc[2])
        self.sigma, self.tau = _coeffs(p)
        self.pin = None
        if (self.tx and self.ty and self.sigma == 0.0 and self.ex.null_index >= 0
                and self.ey.null_index >= 0 and has_null(p.bc[2], p.loc[2])):
            self.pin = (self.ey.null_index, self.ex.null_index)

    def forward(self, f):
        fx = f @ self.ex.Qinv.T if self.tx else f             # 2.1: sum_i Qx^{-1}[p, i] f[k, j, i]
        return np.matmul(self.ey.Qinv, fx) if self.ty else fx  # 2.2: sum_j Qy^{-1}[q, j] fx[k, j, p]

    def modal(self, fxy):
        nz, ny, nx = self.p.shape
        lx = self.ex.lam if self.tx else np.zeros(nx)
        ly = self.ey.lam if self.ty else np.zeros(ny)
        lam = ly[:, None] + lx[None, :]
        if self.zper:
            return cyclic_lines(self.az, self.bz, self.cz, lam, self.sigma, self.tau, fxy, self.pin)
        x, piv = thomas_lines(self.az, self.bz, self.cz, lam, self.sigma, self.tau, fxy, self.pin)
        self.last_pivot = piv
        return x

    def inverse(self, phixy):
        phix = np.matmul(self.ey.Q, phixy) if self.ty else phixy  # 2.4
        return phix @ self.ex.Q.T if self.tx else phix            # 2.5: sum_p Qx[i, p] phix[k, j, p]

    def solve(self, f):
        f = np.asarray(f, dtype=np.float64)
        if f.shape != self.p.shape:
            raise ValueError(f"rhs shape {f.shape} != {self.p.shape}")
        return self.inverse(self.modal(self.forward(f)))


def solve(p, f, plan: Plan | None = None):
    """phi for problem p and right-hand side f (shape p.shape)."""
    return (plan or Plan(p)).solve(f)


def gauge_normalise(p, x):
    """Subtract the volume-weighted mean for a singular problem (solutions are
    defined up to a constant); identity otherwise."""
    if not p.singular:
        return x
    dv = p.volumes()
    return x - (dv * x).sum() / dv.sum()


def relative_error(p, x, ref, norm="2"):
    """||g(x) - g(ref)|| / ||g(ref)|| with g = gauge_normalise."""
    gx, gr = gauge_normalise(p, np.asarray(x, dtype=np.float64)), gauge_normalise(p, ref)
    if norm == "2":
        return float(np.linalg.norm((gx - gr).ravel()) / np.linalg.norm(gr.ravel()))
    return float(np.abs(gx - gr).max() / np.abs(gr).max())

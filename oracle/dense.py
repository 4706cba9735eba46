"""Plain definition of the discrete solution (oracle; test infrastructure
only): x = A^{-1} f with A the assembled three-dimensional operator of §2.2.2
(or I - alpha A for Helmholtz), by dense LU.  For a singular Poisson problem
the system is bordered, [[A, 1], [dV^T, 0]] [x; mu] = [f; 0], which selects
the solution with zero volume-weighted mean (dV is the left null vector of A
because D A is symmetric, §2.2.1).  Only for small grids.
"""
from __future__ import annotations

import numpy as np

from .operator import assemble_3d


def solve_dense(p, f):
    f = np.asarray(f, dtype=np.float64)
    A = assemble_3d(p)
    n = A.shape[0]
    if n > 6000:
        raise ValueError("dense reference is for small grids only")
    if not p.singular:
        return np.linalg.solve(A, f.ravel()).reshape(f.shape)
    dv = p.volumes().ravel()
    B = np.zeros((n + 1, n + 1))
    B[:n, :n] = A
    B[:n, n] = 1.0
    B[n, :n] = dv
    rhs = np.concatenate([f.ravel(), [0.0]])
    return np.linalg.solve(B, rhs)[:n].reshape(f.shape)

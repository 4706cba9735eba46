"""Eigendecomposition of one diagonalised direction (oracle; test
infrastructure only).

§2.2.1: D T is symmetric (dx_i c_i = dx_{i+1} a_{i+1}), so T is similar to
the symmetric T~ = D^{1/2} T D^{-1/2} (Eq. reverse-similarity-transform), whose
eigendecomposition T~ = Q~ Lambda Q~^T has an orthogonal Q~; then
Q = D^{-1/2} Q~ and Q^{-1} = Q~^T D^{1/2} (Eq. q-from-tildeq).  Steps 1.1-1.3
of the initialization of the three-dimensional procedure (§2.2.2).

The eigensolver is the cyclic Jacobi method (``csrc/jacobi.c``), not the
divide-and-conquer / dense LAPACK routines of §3.  Its rotations run in 80-bit
extended precision: in double precision the smooth low modes of a stretched
operator, which carry the solution, are only determined to eps ||T|| / gap
(about 1e-12 at N = 256).

Null mode (periodic or Neumann-Neumann): T 1 = 0, so T~ has the exact null
vector D^{1/2} 1 / ||D^{1/2} 1||.  The eigenvalue of smallest magnitude is set
to exactly 0, its eigenvector to that exact null vector, and the remaining
eigenvectors are re-orthogonalised against it (a reading of the paper:
it treats the null mode through the final-pivot gauge of §3, which
needs the null line to be identified exactly).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from .operator import operator_1d, dense_1d, has_null

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        from . import build as _build
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        lib.oracle_jacobi.restype = ctypes.c_int
        lib.oracle_jacobi.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_double, ctypes.c_int]
        _LIB = lib
    return _LIB


def jacobi_eigh(S: np.ndarray, tol: float = 2.0 ** -63, max_sweeps: int = 60):
    """Eigenvalues w and orthonormal eigenvectors V (columns) of a dense
    symmetric matrix by cyclic Jacobi (rotations in extended precision, see
    csrc/jacobi.c); S V = V diag(w)."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    n = S.shape[0]
    A = S.copy()
    V = np.empty_like(A)
    w = np.empty(n)
    sweeps = _lib().oracle_jacobi(n, A.ctypes.data, V.ctypes.data, w.ctypes.data, tol, max_sweeps)
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge")
    return w, V


@dataclass
class DirectionEig:
    lam: np.ndarray       # eigenvalues Lambda (N)
    Qt: np.ndarray        # Q~ (N x N), orthogonal, columns = eigenvectors of T~
    Q: np.ndarray         # D^{-1/2} Q~
    Qinv: np.ndarray      # Q~^T D^{1/2}
    vol: np.ndarray       # diagonal of D
    null_index: int       # column of the null mode, or -1


def eig_direction(faces, bc, loc="C") -> DirectionEig:
    a, b, c, vol = operator_1d(faces, bc, loc)
    T = dense_1d(a, b, c, bc[0] == "P")
    s = np.sqrt(vol)
    Tt = (s[:, None] * T) / s[None, :]        # D^{1/2} T D^{-1/2}
    Tt = 0.5 * (Tt + Tt.T)                    # remove rounding asymmetry
    lam, Qt = jacobi_eigh(Tt)
    order = np.argsort(-lam, kind="stable")   # 0 (or the largest) first
    lam, Qt = lam[order].copy(), np.ascontiguousarray(Qt[:, order])
    null_index = -1
    if has_null(bc, loc):
        null_index = int(np.argmin(np.abs(lam)))
        lam[null_index] = 0.0
        v0 = s / np.linalg.norm(s)
        Qt[:, null_index] = v0
        for j in range(len(lam)):
            if j != null_index:
                q = Qt[:, j] - np.dot(v0, Qt[:, j]) * v0
                Qt[:, j] = q / np.linalg.norm(q)
    Q = Qt / s[:, None]
    Qinv = Qt.T * s[None, :]
    return DirectionEig(lam, Qt, Q, Qinv, vol, null_index)

"""CPU oracle for the tensor-product--Thomas Poisson/Helmholtz solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.
The HIP library never calls it and shares no code with it.

Plain, slow, obviously-correct FP64 implementations:

* ``operator``  - the one-dimensional second-order operator of §2.2.1
  (Eq. poisson-fd2, Eq. tridiagonal-coefficients) with its boundary rows, and
  the three-dimensional Kronecker-sum operator of §2.2.2 (assembly for small
  grids, stencil application for the residual);
* ``eig``       - symmetrisation T~ = D^{1/2} T D^{-1/2}
  (Eq. reverse-similarity-transform), cyclic Jacobi eigendecomposition (plain C,
  ``csrc/jacobi.c``) and Q = D^{-1/2} Q~, Q^{-1} = Q~^T D^{1/2}
  (Eq. q-from-tildeq);
* ``solver``    - the five solution steps of the three-dimensional procedure
  of §2.2.2: forward x and y transforms (Eq. forward-xy), one Thomas solve per
  (i, j) line with shift lambda_x,i + lambda_y,j, inverse y and x transforms
  (Eq. inverse-xy); the gauge of §3 (vanishing final pivot -> modal unknown 0);
* ``dense``     - the plain definition x = A^{-1} f by dense LU of the
  assembled operator (bordered by the volume-weighted mean for singular
  problems), for grids of at most a few thousand unknowns;
* ``projection`` - the staggered divergence and gradient of §2.1 and the
  projection step u = u* - G phi with L phi = D u*;
* ``navier_stokes`` - the advection term and one Runge--Kutta substep of
  §2.1 (Eq. rk3): predictor, Helmholtz solve per velocity component,
  pressure Poisson solve, correction and pressure update.

Every function is pinned by ``tests/test_oracle_*.py`` against values the
paper prints, closed forms, library routines and brute force.
"""
from .operator import operator_1d, dense_1d, apply_operator, residual, assemble_3d, has_null  # noqa: F401
from .eig import eig_direction, jacobi_eigh  # noqa: F401
from .solver import solve, thomas_lines, relative_error, gauge_normalise  # noqa: F401
from .dense import solve_dense  # noqa: F401
from . import projection  # noqa: F401
from . import navier_stokes  # noqa: F401

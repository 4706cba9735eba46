"""Pins of the oracle's operator assembly and Jacobi eigensolver.

* closed-form eigenvalues of the uniform-grid operators (the modified
  wavenumbers the paper relies on for uniform directions, §2.2.1 last
  paragraph and Algorithm 1 initialization): pins the boundary rows and
  the eigensolver together;
* D T symmetric (§2.2.1, dx_i c_i = dx_{i+1} a_{i+1}), T 1 = 0 for
  periodic/Neumann-Neumann, left null vector = control volumes;
* Jacobi eigenvalues against numpy's LAPACK eigvalsh (a library routine),
  orthogonality and reconstruction of Q~;
* stencil application against the assembled Kronecker sum of §2.2.2.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def closed_form(bc, loc, n, h):
    """Textbook eigenvalues -(4/h^2) sin^2(theta) of the uniform second
    difference with the boundary rows of each condition."""
    s = lambda th: -(4.0 / h ** 2) * np.sin(th) ** 2  # noqa: E731
    if bc == ("P", "P"):
        return s(np.pi * np.arange(n) / n)
    if loc == "F":                                    # n-1 interior faces, Dirichlet walls
        return s(np.pi * np.arange(1, n) / (2 * n))
    if bc == ("N", "N"):
        return s(np.pi * np.arange(n) / (2 * n))
    if bc == ("D", "D"):
        return s(np.pi * np.arange(1, n + 1) / (2 * n))
    return s(np.pi * (2 * np.arange(1, n + 1) - 1) / (4 * n))   # mixed N/D


CASES = [(("P", "P"), "C"), (("N", "N"), "C"), (("D", "D"), "C"), (("N", "D"), "C"),
         (("D", "N"), "C"), (("D", "D"), "F"), (("P", "P"), "F")]


@pytest.mark.parametrize("bc,loc", CASES)
@pytest.mark.parametrize("n", [5, 16, 33])
def test_uniform_closed_form_eigenvalues(bc, loc, n):
    L = 1.7
    faces = W.tanh_faces(n, 0.0, L)
    e = O.eig_direction(faces, bc, loc)
    ref = np.sort(closed_form(bc, loc, n, L / n))
    got = np.sort(e.lam)
    scale = 4.0 / (L / n) ** 2
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-13 * scale


@pytest.mark.parametrize("bc,loc", CASES)
@pytest.mark.parametrize("beta", [0.0, 1.5, 3.0])
def test_weighted_symmetry_and_null(bc, loc, beta):
    n = 23
    faces = W.tanh_faces(n, 0.0 if bc[0] == "P" else beta)
    a, b, c, vol = O.operator_1d(faces, bc, loc)
    T = O.dense_1d(a, b, c, bc[0] == "P")
    DT = vol[:, None] * T
    assert np.abs(DT - DT.T).max() <= 1e-13 * np.abs(DT).max()
    one = np.ones(len(b))
    if O.has_null(bc, loc):
        assert np.abs(T @ one).max() <= 1e-12 * np.abs(T).max()
        assert np.abs(vol @ T).max() <= 1e-12 * np.abs(T).max() * vol.max()
    else:
        # strictly non-singular: smallest |eigenvalue| well away from zero
        assert np.abs(np.linalg.eigvals(T)).min() > 1.0


def test_control_volumes_sum_to_length_and_match_workloads():
    faces = W.tanh_faces(40, 2.0, 3.0)
    for bc, loc in CASES:
        _, _, _, vol = O.operator_1d(faces if bc[0] != "P" else W.tanh_faces(40, 0.0, 3.0), bc, loc)
        f = faces if bc[0] != "P" else W.tanh_faces(40, 0.0, 3.0)
        assert np.allclose(vol, W.control_volumes(f, bc, loc), rtol=1e-15, atol=0)
        if loc == "C" or bc[0] == "P":
            assert abs(vol.sum() - 3.0) < 1e-13


@pytest.mark.parametrize("bc,loc", CASES)
def test_jacobi_against_lapack_and_orthogonality(bc, loc):
    n = 48
    faces = W.tanh_faces(n, 0.0 if bc[0] == "P" else 2.5)
    e = O.eig_direction(faces, bc, loc)
    a, b, c, vol = O.operator_1d(faces, bc, loc)
    T = O.dense_1d(a, b, c, bc[0] == "P")
    s = np.sqrt(vol)
    Tt = s[:, None] * T / s[None, :]
    Tt = 0.5 * (Tt + Tt.T)
    ref = np.linalg.eigvalsh(Tt)
    scale = np.abs(ref).max()
    assert np.abs(np.sort(e.lam) - ref).max() <= 1e-13 * scale
    N = len(e.lam)
    assert np.abs(e.Qt.T @ e.Qt - np.eye(N)).max() <= 1e-13
    assert np.abs(Tt @ e.Qt - e.Qt * e.lam[None, :]).max() <= 1e-12 * scale
    # Q = D^{-1/2} Q~ diagonalises T itself and Q^{-1} is its inverse
    assert np.abs(T @ e.Q - e.Q * e.lam[None, :]).max() <= 1e-11 * scale * np.abs(e.Q).max()
    assert np.abs(e.Qinv @ e.Q - np.eye(N)).max() <= 1e-13
    if O.has_null(bc, loc):
        assert e.lam[e.null_index] == 0.0
        v0 = s / np.linalg.norm(s)
        assert np.abs(np.abs(e.Qt[:, e.null_index]) - v0).max() <= 1e-15


def test_jacobi_random_symmetric():
    rng = np.random.default_rng(3)
    for n in (1, 2, 3, 7, 64):
        S = rng.standard_normal((n, n))
        S = S + S.T
        w, V = O.jacobi_eigh(S)
        assert np.abs(np.sort(w) - np.linalg.eigvalsh(S)).max() <= 1e-12 * max(1.0, np.abs(w).max())
        assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-13


@pytest.mark.parametrize("kind", ["poisson", "helmholtz"])
def test_stencil_matches_assembled_kron(kind):
    p = W.make_problem((7, 6, 5), (1.0, 2.0, 2.5), (W.PP, W.DD, ("N", "D")),
                       loc=("C", "F", "C"), kind=kind, alpha=3e-3)
    x = np.random.default_rng(0).standard_normal(p.shape)
    A = O.assemble_3d(p)
    assert np.abs(O.apply_operator(p, x).ravel() - A @ x.ravel()).max() <= 1e-12 * np.abs(A).max()

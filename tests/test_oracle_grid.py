"""Pins of the grid generator (tanh map, Eq. tanh_stretching of §4.1) against
the spacing numbers the paper prints (tests/golden/grid_spacing.txt)."""
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "grid_spacing.txt")


def _rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, n, L, beta, re_tau, q, v, tol = line.split()
            rows.append((k, int(n), float(L), float(beta), float(re_tau), q, float(v), float(tol)))
    return rows


@pytest.mark.parametrize("row", _rows(), ids=lambda r: f"{r[0]}-{r[1]}-{r[3]}-{r[5]}")
def test_printed_spacings(row):
    kind, n, L, beta, re_tau, q, value, tol = row
    w = np.diff(W.tanh_faces(n, beta, L))
    if q == "dmax_over_dmin":
        got = w.max() / w.min()
    else:
        plus = 2.0 * re_tau  # 1 / (nu/u_tau) with h = 1
        got = (w.max() if q == "dplus_max" else w.min()) * plus
    assert abs(got - value) <= tol, (got, value)


def test_large_n_ratio_is_cosh_squared():
    # footnote to Eq. tanh_stretching: Delta_max/Delta_min ~ cosh^2(beta/2) for many points
    for beta in (1.0, 2.0, 3.0):
        w = np.diff(W.tanh_faces(8192, beta))
        assert abs(w.max() / w.min() / np.cosh(beta / 2) ** 2 - 1) < 1e-3


def test_uniform_limit_and_endpoints():
    x = W.tanh_faces(64, 0.0, 2.0)
    assert np.allclose(np.diff(x), 2.0 / 64, rtol=0, atol=1e-15)
    x2 = W.tanh_faces(64, 1e-6, 2.0)
    assert np.abs(x2 - x).max() < 1e-9
    y = W.tanh_faces(50, 2.5, 3.0)
    assert y[0] == 0.0 and y[-1] == 3.0 and np.all(np.diff(y) > 0)
    # clustered at both ends, symmetric about the middle
    w = np.diff(y)
    assert np.allclose(w, w[::-1], rtol=1e-12)
    assert w[0] < w[25]

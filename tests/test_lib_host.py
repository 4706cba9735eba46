"""Host-side (no GPU) checks of the HIP library: the C-ABI library loads and
exports every symbol of include/tpt.h, and its plan building blocks (1-D
operators with boundary rows, own QL / Householder eigensolvers, analytic
bases, null-mode handling) agree with the oracle on host-only plans."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2603_09528_amd as T
    return T


def test_header_symbols_exported():
    T = _lib()
    with open(os.path.join(ROOT, "include", "tpt.h")) as fh:
        hdr = fh.read()
    declared = set(re.findall(r"\b(tpt_[a-z_0-9]+)\s*\(", hdr))
    assert declared, "no declarations found"
    L = ctypes.CDLL(T.LIB_PATH)
    missing = [s for s in sorted(declared) if not hasattr(L, s)]
    assert not missing, missing
    assert set(T.EXPORTED) == declared


CASES = [
    ((24, 20, 16), (0.0, 2.0, 2.0), (W.PP, W.NN, W.NN), ("C", "C", "C")),
    ((17, 23, 9), (1.5, 2.5, 1.0), (W.NN, W.DD, ("N", "D")), ("C", "C", "C")),
    ((19, 15, 12), (2.0, 0.0, 1.0), (("D", "N"), W.DD, W.DD), ("C", "F", "C")),
    ((16, 18, 10), (0.0, 1.0, 2.0), (W.PP, W.PP, W.NN), ("F", "C", "C")),
    ((21, 16, 8), (1.2, 0.7, 1.0), (W.PP, W.NN, W.DD), ("C", "C", "F")),
]


def _stretched_periodic(n, beta):
    # a non-uniform periodic direction (dense cyclic eigenproblem)
    x = W.tanh_faces(n, beta)
    return x


@pytest.mark.parametrize("case", CASES, ids=lambda c: "".join(b[0] + b[1] for b in c[2]) + "".join(c[3]))
def test_host_plan_matches_oracle(case):
    T = _lib()
    n, beta, bc, loc = case
    p = W.make_problem(n, beta, bc, loc=loc)
    plan = T.Plan.from_problem(p, host_only=True)
    assert plan.nxyz == (p.shape[2], p.shape[1], p.shape[0])
    for d in range(3):
        a, b, c, vol = plan.operator(d)
        oa, ob, oc, ov = O.operator_1d(p.faces[d], p.bc[d], p.loc[d])
        scale = np.abs(ob).max()
        for x, y in ((a, oa), (b, ob), (c, oc)):
            assert np.abs(x - y).max() <= 1e-13 * scale
        assert np.abs(vol - ov).max() <= 1e-15
    for d in range(2):
        lam, Qt = plan.eigen(d)
        e = O.eig_direction(p.faces[d], p.bc[d], p.loc[d])
        scale = np.abs(e.lam).max()
        assert np.abs(np.sort(lam) - np.sort(e.lam)).max() <= 1e-12 * scale
        N = len(lam)
        assert np.abs(Qt.T @ Qt - np.eye(N)).max() <= 1e-12
        a, b, c, vol = plan.operator(d)
        Td = O.dense_1d(a, b, c, p.bc[d][0] == "P")
        s = np.sqrt(vol)
        Tt = s[:, None] * Td / s[None, :]
        assert np.abs(Tt @ Qt - Qt * lam[None, :]).max() <= 1e-11 * scale
        if O.has_null(p.bc[d], p.loc[d]):
            i0 = int(np.argmin(np.abs(lam)))
            assert lam[i0] == 0.0
            assert np.abs(np.abs(Qt[:, i0]) - s / np.linalg.norm(s)).max() <= 1e-15


def test_stretched_periodic_dense_path():
    T = _lib()
    faces = [_stretched_periodic(40, 1.8), W.tanh_faces(12, 1.0), W.tanh_faces(8, 1.0)]
    plan = T.Plan((40, 12, 8), faces, (W.PP, W.NN, W.NN), host_only=True)
    lam, Qt = plan.eigen(0)
    e = O.eig_direction(faces[0], W.PP, "C")
    assert np.abs(np.sort(lam) - np.sort(e.lam)).max() <= 1e-12 * np.abs(e.lam).max()
    assert np.abs(Qt.T @ Qt - np.eye(40)).max() <= 1e-12


@pytest.mark.parametrize("bc,loc", [(W.PP, "C"), (W.NN, "C"), (W.DD, "C"), (W.DD, "F"), (W.PP, "F")])
def test_analytic_uniform_bases(bc, loc):
    T = _lib()
    n = 32
    faces = [W.tanh_faces(n, 0.0, 2.0), W.tanh_faces(6, 1.0), W.tanh_faces(6, 1.0)]
    plan = T.Plan((n, 6, 6), faces, (bc, W.NN, W.NN), loc=(loc, "C", "C"), host_only=True)
    lam, Qt = plan.eigen(0)
    e = O.eig_direction(faces[0], bc, loc)
    assert np.abs(np.sort(lam) - np.sort(e.lam)).max() <= 1e-12 * np.abs(e.lam).max()
    a, b, c, vol = plan.operator(0)
    Td = O.dense_1d(a, b, c, bc[0] == "P")
    assert np.abs(Td @ Qt - Qt * lam[None, :]).max() <= 1e-11 * np.abs(lam).max()


def test_invalid_arguments_rejected():
    T = _lib()
    f = W.tanh_faces(8, 1.0)
    T.Plan((8, 8, 8), (f, f, f), (W.NN, W.NN, W.PP), host_only=True)  # periodic z: cyclic lines
    with pytest.raises(T.TptError):
        T.Plan((8, 8, 8), (f, f, f), (W.NN, W.NN, ("P", "N")), host_only=True)
    with pytest.raises(T.TptError):
        T.Plan((8, 8, 8), (f, f[::-1].copy(), f), (W.NN, W.NN, W.NN), host_only=True)
    with pytest.raises(T.TptError):
        T.Plan((8, 8, 8), (f, f, f), (("P", "N"), W.NN, W.NN), host_only=True)
    with pytest.raises(T.TptError):
        T.Plan((8, 8, 8), (f, f, f), (W.NN, W.NN, W.NN), kind="helmholtz", alpha=0.0, host_only=True)
    with pytest.raises(T.TptError):
        T.Plan((8, 8, 8), (f, f, f), (W.NN, W.NN, W.NN), loc=("F", "C", "C"), host_only=True)


def test_thomas_variant_rejected_before_launch():
    """Bad or unfitting Thomas variants fail in the host checks (the dummy,
    never dereferenced pointers only get past the NULL checks)."""
    T = _lib()
    lib = T.lib()
    p = [4096 + 64 * k for k in range(8)]

    def call(nz, periodic, variant):
        return lib.tpt_thomas(4, 4, nz, 1, p[0], p[1], p[2], p[3], p[4], periodic, 0.0, 1.0, -1,
                              p[5], p[6], p[7], variant, 0)

    assert call(32, 0, 18) == -1       # no such variant
    assert call(32, 0, -2) == -1
    assert call(33, 0, 1) == -1        # 4 x 8 planes < 33
    assert call(1025, 0, 16) == -1     # 64 x 16 planes < 1025
    assert call(300, 0, 10) == -1      # 8 x 32 planes < 300
    assert call(32, 1, 2) == -1        # cyclic lines: sequential kernel only


def test_workspace_size_reported():
    T = _lib()
    p = W.make_problem((10, 9, 8), (1.0, 1.0, 1.0), (W.NN, W.NN, W.NN))
    plan = T.Plan.from_problem(p, host_only=True)
    assert plan.workspace_bytes() >= 16 * p.dof


def test_autotune_table_roundtrip(tmp_path):
    T = _lib()
    src = tmp_path / "table.txt"
    src.write_text("# prec kind M N K variant\n0 0 0 256 256 5\n2 1 96 96 96 3\nbogus line\n1 0 0 48 48 9\n"
                   "0 2 65536 256 0 10\n1 2 4096 64 0 30\n")
    T.autotune_load(str(src))
    out = tmp_path / "out.txt"
    T.autotune_save(str(out))
    lines = [l for l in out.read_text().splitlines() if l and not l.startswith("#")]
    assert "0 0 0 256 256 5" in lines
    assert "2 1 96 96 96 3" in lines
    assert not any(l.endswith(" 9") for l in lines)  # out-of-range variant ignored
    assert "0 2 65536 256 0 10" in lines              # Thomas entry (kind 2)
    assert not any(l.endswith(" 30") for l in lines)  # no such Thomas variant


def test_timing_collect_empty():
    T = _lib()
    T.timing_enable(False)
    assert T.timing_collect() == {}


def test_host_only_plan_reports_dense_transforms():
    # fast transforms need device twiddle tables: a host-only plan has none
    T = _lib()
    p = W.make_problem((64, 32, 8), (0.0, 0.0, 1.0), (W.PP, W.NN, W.NN))
    assert T.Plan.from_problem(p, host_only=True).transforms == ("gemm", "gemm")


@pytest.mark.parametrize("bc", [W.NN, W.DD])
def test_analytic_cosine_sine_bases_large_n(bc):
    # closed forms with the angle reduced exactly in integers: c_k cos(pi k (2i+1)/2N)
    # (Neumann) and c_k sin(pi k (2i+1)/2N), k = 1..N (Dirichlet), cell centres
    T = _lib()
    n = 1024
    faces = [W.tanh_faces(n, 0.0, 1.0), W.tanh_faces(4, 1.0), W.tanh_faces(4, 1.0)]
    plan = T.Plan((n, 4, 4), faces, (bc, W.NN, W.NN), host_only=True)
    _, Qt = plan.eigen(0)
    i = np.arange(n)[:, None]
    if bc == W.NN:
        k = np.arange(n)[None, :]
        c = np.where(k == 0, np.sqrt(1.0 / n), np.sqrt(2.0 / n))
        ref = c * np.cos(np.pi * ((k * (2 * i + 1)) % (4 * n)) / (2 * n))
    else:
        k = np.arange(1, n + 1)[None, :]
        c = np.where(k == n, np.sqrt(1.0 / n), np.sqrt(2.0 / n))
        ref = c * np.sin(np.pi * ((k * (2 * i + 1)) % (4 * n)) / (2 * n))
    assert np.abs(Qt - ref).max() <= 4e-16


def test_navier_stokes_context_rejects_bad_arguments():
    """tpt_ns_create's host checks (no GPU needed): NULL arguments, a
    host-only plan, and the parameters are rejected before any device work."""
    import ctypes
    T = pytest.importorskip("paper_2603_09528_amd")
    L = T.lib()
    p = W.make_problem((8, 6, 6), (0.0, 1.0, 1.0), (W.PP, W.NN, W.NN))
    plan = T.Plan.from_problem(p, host_only=True)
    h = ctypes.c_void_p()
    with pytest.raises(T.TptError) as ei:
        T._check(L.tpt_ns_create(None, 0.1, 1e-3, 0, ctypes.byref(h)))
    assert ei.value.code == -1
    with pytest.raises(T.TptError) as ei:
        T._check(L.tpt_ns_create(plan.handle, 0.1, 1e-3, 0, ctypes.byref(h)))
    assert ei.value.code == -1 and "host-only" in str(ei.value)
    with pytest.raises(T.TptError) as ei:
        T._check(L.tpt_ns_substep(None, 1, *([None] * 8), None, 0, None))
    assert ei.value.code == -1
    b = ctypes.c_size_t()
    with pytest.raises(T.TptError):
        T._check(L.tpt_ns_workspace_bytes(None, ctypes.byref(b)))

"""Kernel-level parity on the GPU: the batched Thomas kernel and the MFMA
GEMM kernels, called through the C-ABI on explicit seeded inputs, against
the oracle's Thomas lines and numpy products."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_util import cuda, host, say

pytestmark = pytest.mark.gpu


def _T():
    import paper_2603_09528_amd as T
    return T


def _thomas_variants(nz):
    """(variant, fits) for the automatic, sequential and partitioned kernels."""
    T = _T()
    out = [(-1, True), (0, True)]
    for v, (_, P, L) in enumerate(T.THOMAS_PARTS, start=1):
        out.append((v, P * L >= nz))
    return out


# long lines: a partial top chunk (131) and whole chunks with two systems
# (256); for the partitioned kernels: a line count that is not a multiple of
# the 64 lines of a block (210, 65 per system with blocks straddling systems),
# nz = P L exactly (64, 256), one plane short of it (255), padded segments
@pytest.mark.parametrize("nx,ny,nz,nsys", [(37, 5, 11, 1), (64, 64, 33, 2), (3, 2, 2, 1), (1, 1, 1, 1), (130, 7, 64, 1),
                                           (33, 9, 131, 1), (16, 8, 256, 2), (70, 3, 64, 1), (64, 2, 255, 1),
                                           (5, 13, 100, 3)])
@pytest.mark.parametrize("sigma,tau", [(0.0, 1.0), (1.0, -3e-3)])
def test_thomas_matches_oracle(nx, ny, nz, nsys, sigma, tau):
    import torch
    T = _T()
    say("thomas", nx, ny, nz, nsys, sigma, tau)
    rng = np.random.default_rng(nx * 1000 + ny * 10 + nz)
    w = rng.uniform(0.5, 2.0, nz)
    az = rng.uniform(0.5, 2.0, nz)
    cz = rng.uniform(0.5, 2.0, nz)
    az[0] = 0.0
    cz[-1] = 0.0
    bz = -(az + cz) - rng.uniform(0.0, 0.3, nz)
    lamx = -rng.uniform(0.0, 50.0, nx)
    lamy = -rng.uniform(0.0, 50.0, ny)
    f = rng.standard_normal((nsys, nz, ny, nx))
    lam = lamy[:, None] + lamx[None, :]
    ref = np.stack([O.thomas_lines(az, bz, cz, lam, sigma, tau, f[s])[0] for s in range(nsys)])
    x = torch.empty(f.shape, dtype=torch.float64, device="cuda")
    scratch = torch.empty((2,) + f.shape, dtype=torch.float64, device="cuda")
    fd = cuda(f)
    for variant, fits in _thomas_variants(nz):
        args = (nx, ny, nz, nsys, cuda(lamx), cuda(lamy), cuda(az), cuda(bz), cuda(cz), sigma, tau, -1, fd, x, scratch)
        if not fits:
            with pytest.raises(T.TptError):
                T.thomas(*args, variant=variant)
            continue
        x.fill_(float("nan"))
        T.thomas(*args, variant=variant)
        torch.cuda.synchronize()
        got = host(x)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), variant
    del w


# the pinned row (nz-1) inside a segment (17, 150) and as the interface row
# of the last segment (64 = 8 x 8, 128 = 8 x 16, 256 = 16 x 16)
@pytest.mark.parametrize("nz", [17, 64, 128, 150, 256])
def test_thomas_pinned_line_in_place(nz):
    import torch
    T = _T()
    nx, ny = 9, 4
    rng = np.random.default_rng(5)
    faces = np.cumsum(np.concatenate([[0.0], rng.uniform(0.5, 1.5, nz)]))
    az, bz, cz, _ = O.operator_1d(faces, ("N", "N"), "C")
    lamx = -rng.uniform(1.0, 20.0, nx)
    lamy = -rng.uniform(1.0, 20.0, ny)
    lamx[3] = 0.0
    lamy[2] = 0.0
    f = rng.standard_normal((nz, ny, nx))
    lam = lamy[:, None] + lamx[None, :]
    ref, _ = O.thomas_lines(az, bz, cz, lam, 0.0, 1.0, f, pin=(2, 3))
    scratch = torch.empty((2, nz, ny, nx), dtype=torch.float64, device="cuda")
    for variant, fits in _thomas_variants(nz):
        if not fits:
            continue
        xf = cuda(f)
        T.thomas(nx, ny, nz, 1, cuda(lamx), cuda(lamy), cuda(az), cuda(bz), cuda(cz), 0.0, 1.0, 3 + nx * 2,
                 xf, xf, scratch, variant=variant)
        torch.cuda.synchronize()
        got = host(xf)
        assert got[-1, 2, 3] == 0.0, variant
        assert np.isfinite(got).all(), variant
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max(), variant


GEMM_SHAPES = [(1, 1, 1, 1), (16, 16, 16, 1), (37, 53, 29, 3), (128, 128, 128, 1), (200, 131, 77, 2),
               (256, 64, 256, 1), (33, 300, 17, 1), (256, 384, 48, 3), (1024, 256, 256, 1)]


@pytest.mark.parametrize("b_nk", [False, True], ids=["kn", "nk"])
@pytest.mark.parametrize("M,N,K,batch", GEMM_SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_gemm_matches_numpy(prec, M, N, K, batch, b_nk):
    import torch
    T = _T()
    say("gemm", prec, M, N, K, batch, b_nk)
    rng = np.random.default_rng(M + 7 * N + 13 * K)
    A = rng.standard_normal((batch, M, K))
    B = rng.standard_normal((batch, N, K) if b_nk else (batch, K, N))
    if prec == "fp64":
        dt, tol = torch.float64, 1e-14
    else:
        dt = torch.float32
        A = A.astype(np.float32).astype(np.float64)
        B = B.astype(np.float32).astype(np.float64)
        tol = 2e-6 if prec == "fp32" else 2e-5
    ref = A @ (np.transpose(B, (0, 2, 1)) if b_nk else B)
    Ad = torch.from_numpy(A).to("cuda", dt)
    Bd = torch.from_numpy(B).to("cuda", dt)
    C = torch.empty((batch, M, N), dtype=dt, device="cuda")
    scale = np.abs(A).max() * np.abs(B).max() * K
    for variant in range(9):
        C.fill_(float("nan"))
        if prec == "bf16x3" and variant >= 6:
            # the persistent and eight-wave tiles are FP64 / FP32 only
            with pytest.raises(T.TptError):
                T.gemm(prec, Ad, Bd, C, M, N, K, batch, M * K, K * N, M * N, b_nk=b_nk, variant=variant)
            continue
        T.gemm(prec, Ad, Bd, C, M, N, K, batch, M * K, K * N, M * N, b_nk=b_nk, variant=variant)
        torch.cuda.synchronize()
        got = host(C).astype(np.float64)
        err = np.abs(got - ref).max() / scale
        assert err <= tol, (variant, err)

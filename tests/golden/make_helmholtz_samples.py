"""Write helmholtz1024_samples.txt: the oracle's solution of the
implicit-diffusion Helmholtz workload (I - alpha L) u = f, alpha = 1e-4,
1024 x 768 x 512 cells, x periodic uniform, y and z Dirichlet walls with tanh
beta = 2, for the three staggered velocity components (u on x-faces, v on
y-faces, w on z-faces; right-hand-side seeds 31, 32, 33) at seeded sample
positions, with the 2-norm and the max-norm of each whole oracle field.

The GPU tests compare the library's full-size solves with these values (an
oracle solve of one component takes about a minute and a half of CPU time
and ~20 GB of memory, too long to repeat inside a test).  Calls only
``oracle`` and ``workloads``; the sample positions are drawn from a fixed
seed and include the eight corners of every field.

Run from the repository root:  python tests/golden/make_helmholtz_samples.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "helmholtz1024_samples.txt")
SAMPLES = 1024
SEED = 2027


def sample_positions(shape, rng):
    nz, ny, nx = shape
    corners = [(k, j, i) for k in (0, nz - 1) for j in (0, ny - 1) for i in (0, nx - 1)]
    flat = [int(np.ravel_multi_index(c, shape)) for c in corners]
    flat += [int(v) for v in rng.integers(0, nz * ny * nx, SAMPLES - len(flat))]
    return flat


def main():
    rng = np.random.default_rng(SEED)
    lines = ["# Oracle solution of the 1024x768x512 implicit-diffusion Helmholtz workload",
             "# (three staggered velocity components, alpha = 1e-4, seeds 31-33), written by",
             "# make_helmholtz_samples.py from oracle/ only.",
             "# 'field <name> <Nz> <Ny> <Nx> <2-norm> <max-norm>' then '<flat index> <value>' lines"]
    for p, seed in W.helmholtz3():
        print("oracle", p.name, flush=True)
        x = O.solve(p, W.rhs(p, seed))
        flat = sample_positions(p.shape, rng)
        xf = x.reshape(-1)
        nz, ny, nx = p.shape
        lines.append(f"field {p.name} {nz} {ny} {nx} {np.linalg.norm(xf):.17e} {np.abs(xf).max():.17e}")
        lines += [f"{i} {xf[i]:.17e}" for i in flat]
        del x, xf
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()

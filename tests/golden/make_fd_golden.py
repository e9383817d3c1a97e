"""Write fd_32.json: FP64 central finite differences of the oracle's forward run for
the differentiable 32^3 problem, along 64 seeded directions (calls only oracle/ and
the seeded input generators; about a minute on 8 host cores).

Run: python tests/golden/make_fd_golden.py

Recipe (shared with tests/test_oracle_adjoint_ics.py and tests/test_gpu_adjoint.py):
one particle per cell of the 32^3 lattice, displacement psi from a Gaussian random
field with P(k) ~ k^-1.5, rms 0.3 cell, seed 61, FP32 and promoted exactly to FP64;
weights w uniform [0, 1), seed 62; 20 KDK steps a = 0.1 -> 0.3 with da = 0.01
(Einstein-de Sitter), TSC, exact seven-point solve; loss sum_c w_c delta_c^2.
Directions: 64 Gaussian white-noise fields over [np, 3], seed 56, each of unit L2
norm. Step: eps such that the perturbation's rms displacement per particle is
2.5e-4 of the rms of psi. Stored per direction: the fourth-order central difference
D(e) = (8 (L(+e) - L(-e)) - (L(+2e) - L(-2e))) / (12 e) at e = eps and at e = 2 eps,
all in FP64. The TSC window is only C^1 (its second derivative jumps at cell
boundaries), so the differences carry an error of first order in e from particles
that cross a boundary within the step; D(2 eps) - D(eps) estimates it.
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import icgen  # noqa: E402
from oracle import adjoint as oa  # noqa: E402

N = 32
A_RUN = [0.1 + 0.01 * i for i in range(21)]
PSI_SEED, W_SEED, DIR_SEED = 61, 62, 56
NDIR = 64


def inputs():
    psi = icgen.displacement_field(N, -1.5, 0.3, PSI_SEED).reshape(-1, 3).astype(np.float32)
    return psi, icgen.lattice_points(N), icgen.weight_grid(N, W_SEED)


def step_size(psi):
    rms = float(np.sqrt(np.mean(np.sum(psi.astype(np.float64) ** 2, axis=-1))))
    return 2.5e-4 * rms * np.sqrt(psi.shape[0])


def directions():
    return icgen.unit_directions(N ** 3, NDIR, DIR_SEED)


def fd_one(j):
    psi, q, w = inputs()
    p64, q64, w64 = psi.astype(np.float64), q.astype(np.float64), w.astype(np.float64)
    d = directions()[j]
    e = step_size(psi)
    loss = {m: oa.ic_loss(p64 + m * e * d, q64, A_RUN, N, w64) for m in (-4, -2, -1, 1, 2, 4)}
    fd4 = lambda s: (8 * (loss[s] - loss[-s]) - (loss[2 * s] - loss[-2 * s])) / (12 * s * e)  # noqa: E731
    return fd4(1), fd4(2)


def main():
    t = time.time()
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        res = list(ex.map(fd_one, range(NDIR)))
    psi, q, w = inputs()
    loss = oa.ic_loss(psi.astype(np.float64), q.astype(np.float64), A_RUN, N,
                      w.astype(np.float64))
    out = {
        "recipe": __doc__.split("Recipe")[1].strip(),
        "n": N, "steps": 20, "a": A_RUN,
        "seeds": {"psi": PSI_SEED, "w": W_SEED, "directions": DIR_SEED},
        "eps": step_size(psi),
        "loss": loss,
        "fd": [r[0] for r in res],
        "fd_2eps": [r[1] for r in res],
        "oracle_seconds": time.time() - t,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fd_32.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"wrote {path}: loss {loss:.10e}, {time.time() - t:.0f} s")


if __name__ == "__main__":
    main()

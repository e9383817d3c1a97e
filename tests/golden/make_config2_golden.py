"""Write config2_256.json: the FP64 oracle's 256^3 ten-step runs, one with the exact
seven-point solve (what multigrid converges to) and one with the FFT solver with TSC
deconvolution, stored at seeded samples (calls only oracle/ and the seeded input
generators; about ten minutes on two host cores and 20 GB of memory).

Run: python tests/golden/make_config2_golden.py

Recipe (shared with tests/test_gpu_config2.py): one particle per cell of the 256^3
lattice, Zel'dovich displacement from a Gaussian random field with P(k) ~ k^-1.5,
rms 0.3 cell, velocities a^(1/2) psi at a = 0.1, seed 2, FP32 positions and
velocities promoted exactly to FP64; 10 KDK steps a = 0.1 -> 0.2 with da = 0.01
(Einstein-de Sitter), TSC deposit and interpolation, 5-point gradient.
Stored per solver: the potential at 4096 seeded cells and the accelerations of
4096 seeded particles at the initial state (a = 0.1), and the positions,
velocities and accelerations of the same particles after the 10 steps.
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
from oracle import pm as opm  # noqa: E402

N = 256
A_RUN = [0.1 + 0.01 * i for i in range(11)]
IC_SEED, CELL_SEED, PART_SEED = 2, 21, 22
NSAMPLE = 4096


def inputs():
    ps = icgen.zeldovich_particles(N, -1.5, 0.3, A_RUN[0], seed=IC_SEED)
    return ps.pos, ps.vel


def samples():
    cells = np.sort(np.random.default_rng(CELL_SEED).choice(N ** 3, NSAMPLE, replace=False))
    parts = np.sort(np.random.default_rng(PART_SEED).choice(N ** 3, NSAMPLE, replace=False))
    return cells, parts


def run_one(solver):
    t = time.time()
    pos, vel = inputs()
    cells, parts = samples()
    x = pos.astype(np.float64)
    v = vel.astype(np.float64)
    acc0, fields = opm.accel(x * N, N, A_RUN[0], solver=solver, return_fields=True)
    phi0 = fields["phi"].reshape(-1)[cells]
    del fields
    acc = acc0
    for a0, a1 in zip(A_RUN[:-1], A_RUN[1:]):
        x, v, acc = opm.kdk_step(x, v, acc, a0, a1, N, solver=solver)
    return {
        "phi0": phi0.tolist(),
        "acc0": acc0[parts].tolist(),
        "acc0_rms": float(np.sqrt(np.mean(acc0 * acc0))),
        "x10": x[parts].tolist(),
        "v10": v[parts].tolist(),
        "acc10": acc[parts].tolist(),
        "seconds": time.time() - t,
    }


def main():
    t = time.time()
    with ProcessPoolExecutor(max_workers=2) as ex:
        res = dict(zip(("exact7", "fft"), ex.map(run_one, ("exact7", "fft"))))
    cells, parts = samples()
    out = {
        "recipe": __doc__.split("Recipe")[1].strip(),
        "n": N, "steps": 10, "a": A_RUN,
        "seeds": {"ic": IC_SEED, "cells": CELL_SEED, "particles": PART_SEED},
        "sample_cells": cells.tolist(),
        "sample_particles": parts.tolist(),
        "runs": res,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_256.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"wrote {path}: {time.time() - t:.0f} s")


if __name__ == "__main__":
    main()

"""Write batch_oracle.json: the FP64 oracle's ten-step runs of five independent
boxes, one of each grid size of the batched ensemble, stored at seeded samples
(calls only oracle/ and the seeded input generators; about two minutes on five
host cores).

Run: python tests/golden/make_batch_golden.py

Recipe (shared with tests/test_gpu_batch.py): boxes of 32^3, 48^3, 64^3, 96^3 and
128^3 cells with one particle per cell; spectral index of box b drawn uniformly
in [-2.5, -1] (numpy default_rng(4), five draws in box order); Zel'dovich
displacement with rms 0.25 cell and velocities a^(1/2) psi at a = 0.1, seed
1000 + b; FP32 positions and velocities promoted exactly to FP64; 10 KDK steps
a = 0.1 -> 0.2 with da = 0.01 (Einstein-de Sitter), TSC, exact seven-point
solve, 5-point gradient. Stored per box: the potential at 2048 seeded cells and
the accelerations of 2048 seeded particles at the initial state, and the
positions of the same particles after the 10 steps.
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

SIZES = (32, 48, 64, 96, 128)
A_RUN = [0.1 + 0.01 * i for i in range(11)]
INDEX_SEED, SAMPLE_SEED = 4, 77
NSAMPLE = 2048


def spectral_indices():
    return [float(x) for x in np.random.default_rng(INDEX_SEED).uniform(-2.5, -1.0, len(SIZES))]


def box_inputs(b):
    n = SIZES[b]
    ps = icgen.zeldovich_particles(n, spectral_indices()[b], 0.25, A_RUN[0], seed=1000 + b)
    return ps.pos, ps.vel


def box_samples(b):
    n = SIZES[b]
    rng = np.random.default_rng(SAMPLE_SEED + b)
    return (np.sort(rng.choice(n ** 3, NSAMPLE, replace=False)),
            np.sort(rng.choice(n ** 3, NSAMPLE, replace=False)))


def run_box(b):
    n = SIZES[b]
    pos, vel = box_inputs(b)
    cells, parts = box_samples(b)
    x, v = pos.astype(np.float64), vel.astype(np.float64)
    acc0, fields = opm.accel(x * n, n, A_RUN[0], return_fields=True)
    xr, _, _ = opm.run(x, v, A_RUN, n)
    return {"n": n, "spectral_index": spectral_indices()[b],
            "phi0": fields["phi"].reshape(-1)[cells].tolist(),
            "acc0": acc0[parts].tolist(),
            "x10": xr[parts].tolist()}


def main():
    t = time.time()
    with ProcessPoolExecutor(max_workers=len(SIZES)) as ex:
        boxes = list(ex.map(run_box, range(len(SIZES))))
    out = {"recipe": __doc__.split("Recipe")[1].strip(), "a": A_RUN,
           "seeds": {"index": INDEX_SEED, "sample": SAMPLE_SEED}, "boxes": boxes}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"wrote {path}: {time.time() - t:.0f} s")


if __name__ == "__main__":
    main()

"""Write adjoint_128.json: the FP64 oracle's loss and initial-condition gradient
for the 128^3 differentiable run (calls only oracle/ and the seeded input
generators; takes about a quarter of an hour on one host core).

Run: python tests/golden/make_adjoint_golden.py

Recipe (shared with tests/test_gpu_adjoint.py): one particle per cell of the
128^3 lattice, displacement psi from a Gaussian random field with
P(k) ~ k^-1.5, rms 0.3 cell, seed 51, FP32 and promoted exactly to FP64;
weights w uniform [0, 1), seed 52; 20 KDK steps a = 0.1 -> 0.3 with da = 0.01
(Einstein-de Sitter), TSC, exact seven-point solve; loss sum_c w_c delta_c^2.
Stored: the loss, dL/dpsi at 4096 seeded particle indices, and the full
gradient's inner products with 8 seeded direction fields (seed 53).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import icgen  # noqa: E402
from oracle import adjoint as oa  # noqa: E402

N = 128
A_RUN = [0.1 + 0.01 * i for i in range(21)]
PSI_SEED, W_SEED, DIR_SEED, SAMPLE_SEED = 51, 52, 53, 54


def inputs():
    psi = icgen.displacement_field(N, -1.5, 0.3, PSI_SEED).reshape(-1, 3).astype(np.float32)
    return psi, icgen.lattice_points(N), icgen.weight_grid(N, W_SEED)


def sample_indices():
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(N ** 3, 4096, replace=False))


def main():
    psi, q, w = inputs()
    t = time.time()
    loss, grad = oa.ic_gradient(psi.astype(np.float64), q.astype(np.float64), A_RUN, N,
                                w.astype(np.float64))
    dt = time.time() - t
    idx = sample_indices()
    dirs = icgen.direction_fields(N, 8, DIR_SEED)
    out = {
        "recipe": __doc__.split("Recipe")[1].strip(),
        "n": N, "steps": 20, "a": A_RUN,
        "seeds": {"psi": PSI_SEED, "w": W_SEED, "directions": DIR_SEED, "sample": SAMPLE_SEED},
        "loss": loss,
        "sample_index": idx.tolist(),
        "grad_sample": grad[idx].tolist(),
        "grad_rms": float(np.sqrt(np.mean(grad * grad))),
        "direction_dot": [float(np.sum(grad * d.astype(np.float64))) for d in dirs],
        "oracle_seconds": dt,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_128.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"wrote {path}: loss {loss:.10e}, {dt:.0f} s")


if __name__ == "__main__":
    main()

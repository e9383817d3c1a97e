"""Parity at the benchmark's full size and launch configuration.

512^3 particles on a 512^3 grid (P(k) ~ k^-1 with a Gaussian cutoff at half the
Nyquist wavenumber, rms displacement 0.25 cell at a = 0.02), cell-offset
positions re-sorted by tile, the benchmark's step parameters (sorted
deterministic deposit, tile-staged interpolation, multigrid with the
growth-rescaled warm start), three kick-drift-kick steps run as one chain
(pm_kdk_chain, as the benchmark times them: the closing and opening half-kicks and
the next drift fused into the interpolation pass). After the last step:
  * density: the benchmark's sorted tile deposit (the kernels the benchmark
    times), at 512 sampled cells, against the oracle deposit of the particles
    around them (FP32 rounding level; an oracle deposit of all 2^27 particles
    takes minutes of host time);
  * potential: whole grid against the oracle's exact seven-point solve of that
    sorted density (promoted to FP64): relative L2 <= 1e-5;
  * accelerations: 4096 sampled particles against the oracle's 5-point
    gradient of that solution interpolated with the TSC window: <= 1e-5.
"""
import math
import sys

import numpy as np
import pytest
import torch

import icgen
from oracle import pm as opm

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.mark.timeout(300)
def test_bench_configuration_512():
    import paper_2410_20501_amd as pm
    n = 512
    _say("full size 512^3: inputs")
    ps = icgen.zeldovich_particles(n, -1.0, 0.25, 0.02, seed=3, cutoff_k=math.pi * n / 2.0,
                                   precision="f32")
    cell_np, off = icgen.to_cell_offset(ps.pos, n)
    npart = off.shape[0]
    off_d = torch.from_numpy(off).cuda()
    cell_d = torch.from_numpy(cell_np).cuda()
    vel_d = torch.from_numpy(ps.vel).cuda()
    del ps, off, cell_np
    ctx = pm.Context(n, npart)
    phi = torch.zeros((n, n, n), device="cuda")
    acc = torch.empty((npart, 3), device="cuda")
    import bench
    params = bench.bench_step_params(pm)
    _say("full size 512^3: GPU steps")
    pm.pm_reorder(ctx, off_d, vel=vel_d, cell=cell_d)
    pm.pm_accel(ctx, off_d, 0.02, phi, acc, cell=cell_d, params=params)
    params.mg.guess = bench.BENCH_GUESS(pm)
    a_list = [0.02 + 0.0196 * i for i in range(4)]
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", pm.PMWarning)
        for i in range(3):
            a2 = a_list[i + 2] if i + 2 < len(a_list) else 0.0
            stage = pm.PM_CHAIN_FIRST if i == 0 else pm.PM_CHAIN_NEXT
            st = pm.pm_kdk_chain(ctx, off_d, vel_d, a_list[i], a_list[i + 1], a2, stage, phi, acc,
                                 cell=cell_d, params=params)
    rho = torch.empty((n, n, n), device="cuda")
    pm.pm_deposit(ctx, off_d, rho, cell=cell_d, order="sorted")
    torch.cuda.synchronize()
    rho_h = rho.cpu().numpy().astype(np.float64)
    phi_h = phi.cpu().numpy().astype(np.float64)
    _say(f"full size 512^3: oracle solve (cycles {st.mg.cycles}, relres {st.mg.history()[-1]:.2e})")
    phi_ref = opm.solve_exact7(opm.source(rho_h, a_list[-1]), 1.0 / n, workers=16)
    err_phi = np.linalg.norm(phi_h - phi_ref) / np.linalg.norm(phi_ref)
    print(f"phi rel L2 {err_phi:.3e}", flush=True)
    assert err_phi <= 1e-5
    del rho_h
    # sampled particles
    rng = np.random.Generator(np.random.PCG64(99))
    idx = rng.choice(npart, size=4096, replace=False)
    off_h = off_d.cpu().numpy()
    cell_h = cell_d.cpu().numpy()
    acc_h = acc.cpu().numpy().astype(np.float64)
    u = opm.cell_units(n, cell=cell_h[idx], off=off_h[idx])
    g_ref = opm.gradient(phi_ref, 1.0 / n)
    acc_ref = opm.interp(u, g_ref, "tsc")
    del g_ref
    err_acc = np.linalg.norm(acc_h[idx] - acc_ref) / np.linalg.norm(acc_ref)
    print(f"acc rel L2 (4096 sampled particles) {err_acc:.3e}", flush=True)
    assert err_acc <= 1e-5
    # sampled cells of the density: oracle deposit of the particles around them
    cells = rng.integers(0, n, size=(512, 3))
    near = np.zeros((n, n, n), dtype=bool)
    for c in cells:
        sl = [np.arange(c[d] - 1, c[d] + 2) % n for d in range(3)]
        near[np.ix_(*sl)] = True
    sel = near.reshape(-1)[cell_h]
    rho_sel = opm.deposit(opm.cell_units(n, cell=cell_h[sel], off=off_h[sel]), n, "tsc",
                          mass=float(n ** 3) / npart)
    got = rho.cpu().numpy()[cells[:, 0], cells[:, 1], cells[:, 2]]
    want = rho_sel[cells[:, 0], cells[:, 1], cells[:, 2]]
    err = np.abs(got - want).max()
    print(f"sorted density at 512 sampled cells: max |diff| {err:.3e} (max rho {want.max():.1f})",
          flush=True)
    assert err <= 4e-6 * max(1.0, want.max())

"""Benchmark: particle-mesh particle-steps/s on one MI355X.

Workload: 512^3 particles on a 512^3 grid, P(k) ~ k^-1 exp(-k^2/k_c^2) with
k_c = k_Nyquist / 2, rms displacement 0.25 cell at a = 0.02, 50 kick-drift-kick
steps uniform in a up to a = 1, positions stored as FP32 in-cell offsets plus
an int32 cell index, TSC, multigrid (2 + 2 red-black Gauss-Seidel sweeps, full
weighting) warm-started from the previous step's potential. Inputs are seeded
synthetic Gaussian random fields generated on the host and copied to HBM before
the timed region. The steps run as one chain (pm_kdk_chain): one "step" is one
call, that is deposit, multigrid solve, 5-point gradient and interpolation, with the
closing half-kick of the step, the opening half-kick of the next and the next drift
applied in the interpolation pass (--no-chain: one pm_kdk call per step, kick + drift
in a pass of its own).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak

# HBM traffic of the roofline kernel per launch, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of this benchmark at 512^3,
# scaled by the same counters read for a plain 512 MiB device copy (read x2.0,
# write x1.0). Valid only for the kernel source it was measured on: the bench
# reports null when the source file's hash differs.
MEASURED_TRAFFIC = {
    # kernel: (source file, sha256 of it, fetch KiB, write KiB, fetch scale, write scale)
    # smoother: level-0 passes, mean of the pre-smoothing pass (with the residual norm)
    # and the post-smoothing pass (with the prolongation) weighted by their counts (45
    # and 39 dispatches)
    "smooth": ("paper_2410_20501_amd/csrc/mg_stream.hip",
               "4ea35171df84f337cefdd3d1146566fb9eea23ffec47a4cdf832b17cc38d203f",
               628408.0, 524301.0, 2.0, 1.0),
    # deposit: the particle-owned tile kernel plus the gather pass over the tile boxes
    "deposit": ("paper_2410_20501_amd/csrc/particles.hip",
                "858c00d7abdcbe38589b6d15dd9ddc720ef29853cd37858ffc3bdf6709ea6f17",
                2005610.0, 1549791.0, 2.0, 1.0),
    # interpolation with the fused gradient, kicks and drift of a chained step
    "interp": ("paper_2410_20501_amd/csrc/particles.hip",
               "858c00d7abdcbe38589b6d15dd9ddc720ef29853cd37858ffc3bdf6709ea6f17",
               2749282.0, 5320506.0, 2.0, 1.0),
}


def _source_hash(rel):
    import hashlib
    with open(os.path.join(ROOT, rel), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def traffic_bytes(kernel):
    rec = MEASURED_TRAFFIC.get(kernel)
    if rec is None:
        return None
    src, digest, fkib, wkib, fs, ws = rec
    if _source_hash(src) != digest:
        return None
    return (fkib * fs + wkib * ws) * 1024.0


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# multigrid settings of the benchmark run (the full-size parity test uses the same)
BENCH_ORDER = "sorted"
BENCH_TOL = 1e-6
BENCH_MAX_CYCLES = 40


def BENCH_GUESS(pm):
    """Warm start of the steps after the first: the linear extrapolation of the
    growth-normalised potentials of the last two solves (one V-cycle fewer per step than
    the growth-rescaled previous potential, the same tolerance)."""
    return pm.PM_GUESS_EXTRAPOLATED


def bench_step_params(pm, order=BENCH_ORDER, tol=BENCH_TOL, omega=None):
    p = pm.default_step_params(order=order, tol=tol, max_cycles=BENCH_MAX_CYCLES)
    if omega is not None:
        p.mg.omega = omega
    return p


def make_inputs(n, seed=3, a0=0.02):
    import numpy as np

    import icgen
    t = time.time()
    cutoff = math.pi * n / 2.0                       # k_c = k_Nyquist / 2, k_Nyquist = pi n
    ps = icgen.zeldovich_particles(n, -1.0, 0.25, a0, seed=seed, cutoff_k=cutoff, precision="f32")
    cell, off = icgen.to_cell_offset(ps.pos, n)
    _log(f"inputs {n}^3 generated in {time.time() - t:.1f}s")
    return np.ascontiguousarray(off), np.ascontiguousarray(cell), np.ascontiguousarray(ps.vel)


def _host_info():
    """Host CPU model, logical core count and memory (Linux /proc)."""
    model, mem_gb = "unknown", None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    mem_gb = round(int(line.split()[1]) / 1024 ** 2, 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cores": os.cpu_count(), "mem_gb": mem_gb}


def cpu_baseline(n_sample=128, steps=6, seed=3):
    """The FP64 oracle, as is, on a bounded sample of the same recipe, with its FFTs on
    every host core (scipy workers; numpy's bincount and roll stay single-threaded)."""
    import numpy as np
    import scipy.fft as sfft

    import icgen
    from oracle import pm as opm
    a = [0.02 + 0.0196 * i for i in range(steps + 1)]
    ps = icgen.zeldovich_particles(n_sample, -1.0, 0.25, a[0], seed=seed,
                                   cutoff_k=math.pi * n_sample / 2.0)
    x = ps.pos.astype(np.float64)
    v = ps.vel.astype(np.float64)
    cores = os.cpu_count() or 1
    with sfft.set_workers(cores):
        acc = opm.accel(x * n_sample, n_sample, a[0])
        t = time.perf_counter()
        for a0, a1 in zip(a[:-1], a[1:]):
            x, v, acc = opm.kdk_step(x, v, acc, a0, a1, n_sample)
        dt = time.perf_counter() - t
    host = _host_info()
    return {
        "value": n_sample ** 3 * steps / dt,
        "unit": "particle-steps/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"FP64 numpy/scipy oracle, {n_sample}^3 particles on a {n_sample}^3 grid, "
                  f"{steps} KDK steps from a=0.02 (same recipe, exact 7-point solve), "
                  f"{dt:.1f}s, scipy FFTs on {cores} threads, deposit and interpolation on one",
        "host": host,
        "paper_context": "the paper quotes about one CPU hour for a 512^3 Newtonian run on a "
                         "laptop (introduction) and 15 to 25 s per 512^3 step on one CPU "
                         "core (Sect. 4.6)",
    }


def bench_adjoint(n=128, steps=20, reps=3):
    """Differentiable run (128^3, P ~ k^-1.5, 20 steps, checkpoints every 4): loss alone vs
    loss + gradient through the hand-written adjoint, on the same GPU."""
    import numpy as np
    import torch
    import warnings

    import icgen
    import paper_2410_20501_amd as pm
    from paper_2410_20501_amd import autodiff
    warnings.simplefilter("ignore", pm.PMWarning)
    a_list = [0.1 + 0.01 * i for i in range(steps + 1)]
    psi = icgen.displacement_field(n, -1.5, 0.3, 51).reshape(-1, 3).astype(np.float32)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    psi_d, q_d, w_d = dev(psi), dev(icgen.lattice_points(n)), dev(icgen.weight_grid(n, 52))
    run = autodiff.Run(n, n ** 3, a_list, checkpoint_every=4, poskind="celloff")
    autodiff.loss_and_gradient(psi_d, q_d, w_d, run)  # warm-up
    tf, tb = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        autodiff.loss_only(psi_d, q_d, w_d, run)
        torch.cuda.synchronize()
        tf.append(time.perf_counter() - t)
        t = time.perf_counter()
        autodiff.loss_and_gradient(psi_d, q_d, w_d, run)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t)
    run.close()
    f, b = min(tf), min(tb)
    return {
        "workload": f"{n}^3 particles, {steps} KDK steps a=0.1->0.3, TSC, multigrid tol 1e-6 "
                    f"(adjoint solves 1e-5), cell-offset positions, checkpoints every 4 steps, "
                    f"loss sum w delta^2",
        "forward_ms": 1e3 * f, "forward_and_gradient_ms": 1e3 * b,
        "gradient_over_forward": b / f,
        "forward_particle_steps_per_s": n ** 3 * steps / f,
        "gradient_particle_steps_per_s": n ** 3 * steps / b,
        "transposed_force_evaluations": steps + 1,
    }


def bench_batched(nboxes=96, steps=20, master_seed=2024):
    """Ensemble of 96 boxes (grids uniform in {32,48,64,96,128}^3, np = cells, n_s in
    [-2.5,-1]), 20 steps: one captured batched step replayed vs a loop of per-box pm_kdk."""
    import numpy as np
    import torch
    import warnings

    import icgen
    import paper_2410_20501_amd as pm
    warnings.simplefilter("ignore", pm.PMWarning)
    a_list = [0.1 + 0.01 * i for i in range(steps + 1)]
    draws = icgen.ensemble_draw(master_seed, nboxes)
    t = time.time()
    pos_l, vel_l = [], []
    for n, ns, seed in draws:
        ps = icgen.zeldovich_particles(n, ns, 0.25, a_list[0], seed=seed, precision="f32")
        pos_l.append(ps.pos)
        vel_l.append(ps.vel)
    sizes = [d[0] for d in draws]
    _log(f"batched inputs: {nboxes} boxes generated in {time.time() - t:.1f}s")
    pos0 = torch.from_numpy(np.concatenate(pos_l)).cuda()
    vel0 = torch.from_numpy(np.concatenate(vel_l)).cuda()
    del pos_l, vel_l
    B = pm.Batch(sizes, [n ** 3 for n in sizes])
    npart = B.np_total
    # plain loop: one context per box, pm_kdk per box and step (tolerance-driven multigrid)
    first = pm.default_step_params(tol=1e-6, max_cycles=40)
    warm = pm.default_step_params(tol=1e-6, max_cycles=40, guess="warm_rescaled")
    ctxs = {n: pm.Context(n, n ** 3) for n in sorted(set(sizes))}
    t_loop = 0.0
    for b, n in enumerate(sizes):
        sl = slice(B.p_off[b], B.p_off[b + 1])
        pb, vb = pos0[sl].clone(), vel0[sl].clone()
        phi = torch.zeros((n, n, n), device="cuda")
        acc = torch.empty_like(pb)
        pm.pm_accel(ctxs[n], pb, a_list[0], phi, acc, params=first)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(steps):
            pm.pm_kdk(ctxs[n], pb, vb, a_list[i], a_list[i + 1], phi, acc, params=warm)
        torch.cuda.synchronize()
        t_loop += time.perf_counter() - t
    for c in ctxs.values():
        c.close()
    # batched: tune, first solve, capture one step, replay
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        p, v = pos0.clone(), vel0.clone()
        acc = torch.zeros_like(p)
        phi = torch.zeros(B.ncell_total, device="cuda")
        pw = pm.default_step_params(fixed_cycles=4, guess="warm_rescaled")
        tune = pm.pm_tune(B, p, phi, pw)
        phi.zero_()
        pm.pm_batch_accel(B, p, acc, phi, a_list[0], pm.default_step_params(fixed_cycles=8))
        state = (p.clone(), v.clone(), acc.clone(), phi.clone())
        s.synchronize()
        t = time.perf_counter()
        pm.pm_batch_kdk(B, p, v, acc, phi, a_list, pw)
        s.synchronize()
        t_eager = time.perf_counter() - t
        for dst, src in zip((p, v, acc, phi), state):
            dst.copy_(src)
        pm.pm_graph_capture_step(B, p, v, acc, phi, pw)
        s.synchronize()
        t = time.perf_counter()
        pm.pm_batch_kdk(B, p, v, acc, phi, a_list, pw, use_graph=True)
        s.synchronize()
        t_graph = time.perf_counter() - t
    B.close()
    best = min(t_eager, t_graph)
    return {
        "workload": f"{nboxes} boxes, grids {{32,48,64,96,128}}^3 (seed {master_seed}), "
                    f"{npart} particles total, {steps} KDK steps a=0.1->0.3, TSC, multigrid "
                    f"(batched: 4 warm-started V-cycles per step; plain: tol 1e-6)",
        "particles": npart,
        "batched_graph_s": t_graph, "batched_eager_s": t_eager, "per_box_loop_s": t_loop,
        "batched_particle_steps_per_s": npart * steps / best,
        "per_box_loop_particle_steps_per_s": npart * steps / t_loop,
        "speedup_vs_per_box_loop": t_loop / best,
        "tuned_rows": tune,
    }


def bench_fft(n=256, reps=20):
    """FFT Poisson solve (Green's function with TSC deconvolution) and FFT_7pt on an n^3
    grid (the 256^3 ten-step workload's solver), timed with HIP events on the current
    stream. Algorithmic bytes: the five LDS-staged passes each read and write the half
    spectrum (n^2 (n/2+1) complex, about 4 B per cell each way), the first pass reads
    the real density (4 B/cell) instead and the last writes the real potential: about
    8 B per cell per pass, 40 B per cell per solve."""
    import numpy as np
    import torch

    import paper_2410_20501_amd as pm
    rng = np.random.Generator(np.random.PCG64(8))
    rho = torch.from_numpy((1.0 + 0.3 * rng.standard_normal((n, n, n))).astype(np.float32)).cuda()
    phi = torch.empty_like(rho)
    g = torch.empty((n, n, n, 3), device="cuda")
    ctx = pm.Context(n)
    out = {"workload": f"{n}^3 grid, FFT solve with TSC deconvolution (five passes), FFT_7pt, "
                       f"and FULL_FFT (force grid, twelve passes)"}
    for name, kern, dst, passes in (("fft", "green", phi, 5), ("fft_7pt", "7pt", phi, 5),
                                    ("full_fft", "full", g, 12)):
        for _ in range(2):
            pm.pm_solve_fft_kernel(ctx, rho, 0.3, dst, kernel=kern, deconv=3)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            pm.pm_solve_fft_kernel(ctx, rho, 0.3, dst, kernel=kern, deconv=3)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        alg = 8.0 * passes * n ** 3 + (8.0 * n ** 3 if name == "full_fft" else 0.0)
        out[name] = {"ms": ms, "algorithmic_bytes": alg, "gbs": alg / (ms * 1e-3) / 1e9,
                     "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    ctx.close()
    return out


def bench_fr(n=512, reps=5, n_step=256, steps=3):
    """f(R) (Hu-Sawicki n = 1, f_R0 = -1e-5, Omega_m 0.3, Omega_L 0.7, 100 Mpc/h box):
    (1) the scalaron's FAS F cycle (the paper's one cycle per force evaluation) on an n^3
    clustered density (log-normal, sigma 1, seeded), each cycle starting from the last,
    with the finest non-linear Gauss-Seidel sweep timed per launch (32 algorithmic bytes
    per cell: FP64 u read by both colour passes, s read and u written once); (2) the cost
    of a whole f(R) step against a Newtonian one at n_step^3 particles and cells."""
    import warnings

    import torch

    import icgen
    import paper_2410_20501_amd as pm
    warnings.simplefilter("ignore", pm.PMWarning)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(77)
    rho = torch.exp(torch.randn((n, n, n), device="cuda", generator=gen))
    rho /= rho.mean()
    box = 100.0
    p = pm.default_step_params(omega_m=0.3, omega_l=0.7, fr_f0=-1e-5, fr_n=1,
                               fr_c2=(2997.92458 / box) ** 2)
    ctx = pm.Context(n)
    u = torch.ones((n, n, n), dtype=torch.float64, device="cuda")
    for _ in range(2):
        pm.pm_solve_fr(ctx, rho, 0.5, p, u)
    torch.cuda.synchronize()
    pm.pm_kernel_timer(ctx, "fr_sweep", 64)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        pm.pm_solve_fr(ctx, rho, 0.5, p, u)
    t1.record()
    torch.cuda.synchronize()
    ms_cycle = t0.elapsed_time(t1) / reps
    kms, launches, kbytes = pm.pm_kernel_timer_read(ctx)
    rr = pm.pm_solve_fr(ctx, rho, 0.5, p, u, relres=True)
    ctx.close()
    sweep_ms = kms / max(launches, 1)
    sweep_gbs = kbytes / max(launches, 1) / (sweep_ms * 1e-3) / 1e9
    # one F cycle: 3 sweeps + residual (24 B/cell) + restriction (16) + prolongation (16)
    # on the finest grid; the coarser grids add about 0.3 of that
    alg = 1.3 * (3 * 32.0 + 56.0) * n ** 3
    out = {"workload": f"{n}^3 log-normal density (sigma 1), f(R) n=1 f_R0=-1e-5, a=0.5, one "
                       f"FAS F cycle (2 pre + 1 post non-linear red-black sweeps, levels "
                       f"{n} -> 4, 32 sweeps on 4^3), from the previous cycle's result",
           "ms_per_f_cycle": ms_cycle,
           "cycle_gbs_estimate": alg / (ms_cycle * 1e-3) / 1e9,
           "relres_one_more_cycle": list(rr),
           "sweep": {"avg_ms": sweep_ms, "launches": launches, "gbs": sweep_gbs,
                     "frac": sweep_gbs / HBM_PEAK_GBS,
                     "bytes_rule": "32 B/cell per sweep (both colours), FP64"}}
    # whole steps: Newtonian vs f(R), same particles, multigrid, sorted deposit
    ps = icgen.zeldovich_particles(n_step, -2.0, 0.5, 0.5, seed=78)
    res = {}
    for grav in ("newton", "fr"):
        ctx = pm.Context(n_step, n_step ** 3)
        q = pm.default_step_params(omega_m=0.3, omega_l=0.7, gravity=grav, order="sorted",
                                   fr_f0=-1e-5, fr_c2=(2997.92458 / box) ** 2)
        pos, vel = torch.from_numpy(ps.pos).cuda(), torch.from_numpy(ps.vel).cuda()
        phi = torch.zeros((n_step,) * 3, device="cuda")
        acc = torch.empty_like(pos)
        pm.pm_accel(ctx, pos, 0.5, phi, acc, params=q)
        q.mg.guess = pm.PM_GUESS_WARM_RESCALED
        a_list = [0.5 + 0.01 * i for i in range(steps + 2)]
        pm.pm_kdk(ctx, pos, vel, a_list[0], a_list[1], phi, acc, params=q)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for a0, a1 in zip(a_list[1:-1], a_list[2:]):
            pm.pm_kdk(ctx, pos, vel, a0, a1, phi, acc, params=q)
        torch.cuda.synchronize()
        res[grav] = 1e3 * (time.perf_counter() - t) / steps
        ctx.close()
    out["step_ms"] = {"workload": f"{n_step}^3 particles and cells, LCDM, sorted TSC deposit, "
                                  f"multigrid tol 1e-6 warm-started", **res,
                      "fr_over_newton": res["fr"] / res["newton"]}
    return out


def stage_bytes(npart, ncell, cycles, chained=False):
    """Algorithmic HBM bytes of each stage of one step at cell-offset positions (what the
    method must move, per unit of work: deposit 16 B per particle + 4 B per cell; a
    multigrid V-cycle 82 B per cell). With the sorted deposit
    the gradient is formed inside the interpolation kernel, which then reads the
    potential (4 B/cell) instead of the force grid; the gradient stage is empty. In a
    chained step the drift is part of the interpolation pass: offsets, cell index and
    velocity in and out and the tile key out (60 B per particle), no acceleration."""
    return {
        "ms_drift": 0.0 if chained else 68.0 * npart,
        "ms_deposit": 16.0 * npart + 4.0 * ncell,
        # V-cycles of 2 + 2 sweeps at 12 B/cell each, residual-restriction and
        # prolongation 8.5 B/cell each, all levels (x 8/7), + 8 B/cell for the finest
        # norm: 82 B/cell per cycle; + the two sweeps of the last norm pass, whose
        # smoothed output is kept (24 B/cell)
        "ms_solve": (cycles * 82.0 + 24.0) * ncell,
        "ms_interp": (60.0 if chained else 52.0) * npart + 4.0 * ncell,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=47)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--order", default=BENCH_ORDER, choices=["atomic", "sorted"])
    ap.add_argument("--tol", type=float, default=BENCH_TOL)
    ap.add_argument("--guess", choices=["extrapolated", "warm_rescaled"], default="extrapolated",
                    help="warm start of the multigrid solves after the first step")
    ap.add_argument("--omega", type=float, default=None,
                    help="over-relaxation factor of the red-black sweeps (default: the "
                         "library's)")
    ap.add_argument("--reorder-every", type=int, default=10,
                    help="re-sort particles by tile every this many steps (0: never)")
    ap.add_argument("--no-chain", action="store_true",
                    help="one pm_kdk call per step instead of a chain of pm_kdk_chain calls")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--roofline-kernel", default="smooth", choices=["deposit", "smooth", "interp"],
                    help="kernel timed with events for the roofline object (default: the "
                         "streaming smoother on the finest grid, the largest share of kernel time)")
    ap.add_argument("--stage-log", action="store_true",
                    help="record per-stage times of every timed step (adds events)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 512 MiB device copy (HBM counter calibration)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the adjoint, batched-ensemble, FFT and f(R) measurements")
    ap.add_argument("--only", choices=["adjoint", "batched", "fft", "fr"], default=None,
                    help="run only one of the extra measurements and print its JSON object")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2410_20501_amd as pm

    if args.only:
        res = {"adjoint": bench_adjoint, "batched": bench_batched, "fft": bench_fft,
               "fr": bench_fr}[args.only]()
        print(json.dumps({args.only: res}), flush=True)
        return

    if args.copy_calibration:
        src = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4}))
        return

    n = args.n
    total_steps = 50
    if args.warmup + args.steps > total_steps:
        raise SystemExit(f"warmup + steps must be <= {total_steps} (the run has 50 steps)")
    # the step after the timed ones (when warmup + steps < 50) is re-run with per-stage events
    a_list = [0.02 + (1.0 - 0.02) * i / total_steps for i in range(total_steps + 1)]

    off, cell, vel = make_inputs(n)
    npart = off.shape[0]
    dev = torch.device("cuda", 0)
    off_d = torch.from_numpy(off).to(dev)
    cell_d = torch.from_numpy(cell).to(dev)
    vel_d = torch.from_numpy(vel).to(dev)
    del off, cell, vel
    phi = torch.zeros((n, n, n), device=dev)
    acc = torch.empty((npart, 3), device=dev)
    ctx = pm.Context(n, npart)
    params = bench_step_params(pm, args.order, args.tol, args.omega)
    torch.cuda.synchronize()
    if args.reorder_every > 0:
        pm.pm_reorder(ctx, off_d, vel=vel_d, cell=cell_d)
    pm.pm_accel(ctx, off_d, a_list[0], phi, acc, cell=cell_d, params=params)
    params.mg.guess = (pm.PM_GUESS_WARM_RESCALED if args.guess == "warm_rescaled"
                       else BENCH_GUESS(pm))
    torch.cuda.synchronize()

    import warnings
    warnings.simplefilter("ignore", pm.PMWarning)

    def one_step(step, last=False):
        """Step a_list[step] -> a_list[step + 1]; with the chain, `last` ends it in the
        synchronised state (the next drift is not applied)."""
        if args.no_chain:
            return pm.pm_kdk(ctx, off_d, vel_d, a_list[step], a_list[step + 1], phi, acc,
                             cell=cell_d, params=params)
        a2 = a_list[step + 2] if (step + 2 <= total_steps and not last) else 0.0
        stage = pm.PM_CHAIN_FIRST if step == 0 else pm.PM_CHAIN_NEXT
        return pm.pm_kdk_chain(ctx, off_d, vel_d, a_list[step], a_list[step + 1], a2, stage, phi,
                               acc, cell=cell_d, params=params)

    step = 0
    for _ in range(args.warmup):
        one_step(step)
        step += 1
    torch.cuda.synchronize()
    _log(f"warmup done ({args.warmup} steps)")

    cycles = []
    hists = []
    stage_rows = []
    if args.stage_log:
        params.timing = 1
    pm.pm_kernel_timer(ctx, args.roofline_kernel, capacity=16384)
    t0 = time.perf_counter()
    for i in range(args.steps):
        if args.reorder_every > 0 and step % args.reorder_every == 0:
            # a chain keeps no accelerations between its steps (the next opening kick is
            # applied with the closing one): only pm_kdk steps need acc permuted too
            pm.pm_reorder(ctx, off_d, vel=vel_d, acc=acc if args.no_chain else None,
                          cell=cell_d)
        st = one_step(step)
        cycles.append(st.mg.cycles)
        if args.stage_log:
            stage_rows.append((step, round(st.ms_drift, 2), round(st.ms_deposit, 2),
                               round(st.ms_solve, 2), round(st.ms_gradient, 2),
                               round(st.ms_interp, 2)))
        if i in (0, args.steps // 2, args.steps - 1):
            hists.append(["%.2e" % r for r in st.mg.history()])
        step += 1
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    _log(f"timed {args.steps} steps in {elapsed:.3f}s; V-cycles per step {cycles}")
    _log(f"relres histories (first, middle, last timed step): {hists}")
    if args.stage_log:
        _log("step: drift deposit solve gradient interp (ms)")
        for row in stage_rows:
            _log(str(row))

    ms_per_step = 1000.0 * elapsed / max(args.steps, 1)
    value = npart * args.steps / elapsed
    k_ms, k_launches, k_bytes = pm.pm_kernel_timer_read(ctx)
    pm.pm_kernel_timer(ctx, "none", capacity=0)
    roofline = None
    if k_launches > 0 and k_ms > 0:
        per_launch_bytes = k_bytes / k_launches
        avg_ms = k_ms / k_launches
        achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
        traffic = traffic_bytes(args.roofline_kernel)
        roofline = {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": args.roofline_kernel, "launches": k_launches,
            "avg_ms": avg_ms, "algorithmic_bytes_per_launch": per_launch_bytes,
        }
        if args.roofline_kernel == "smooth":
            # achieved counts 12 B/cell per red-black sweep (two per pass); the least a
            # pass itself must move is one read of u and f and one write of u, 12 B/cell
            minimum = 12.0 * n ** 3
            roofline["bytes_rule"] = "12 B/cell per sweep, 2 sweeps per pass (+0.5 prolongation)"
            roofline["pass_minimum_bytes"] = minimum
            roofline["frac_of_pass_minimum"] = minimum / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
        _log(f"roofline {args.roofline_kernel}: {k_launches} launches, avg {avg_ms:.3f} ms, "
             f"{achieved:.0f} GB/s algorithmic")

    # per-stage times of one extra (untimed) step with stage events
    params.timing = 1
    # (a chain that has not reached its end keeps going: this step ends it unless more
    # steps follow, in which case it stays a chained step like the timed ones)
    stt = one_step(step, last=step + 2 > total_steps) if step < total_steps else None
    stages = None
    stage_gbs = None
    if stt is not None:
        stages = {k: round(getattr(stt, k), 4) for k in
                  ("ms_drift", "ms_deposit", "ms_solve", "ms_gradient", "ms_interp")}
        chained = not args.no_chain and step + 2 <= total_steps
        sb = stage_bytes(npart, n ** 3, stt.mg.cycles, chained)
        stage_gbs = {k.replace("ms_", ""): {
            "gbs": round(sb[k] / (stages[k] * 1e-3) / 1e9, 1),
            "frac": round(sb[k] / (stages[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            for k in sb if stages[k] > 0}
        stage_gbs["solve"]["vcycles"] = stt.mg.cycles

    out = {
        "metric": "PM particle-steps/s at 512^3",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded power-law Gaussian random field, Zel'dovich ICs)",
        "config": {"workload": f"{n}^3 particles on a {n}^3 grid, 50 KDK steps a=0.02->1, "
                               f"cell-offset positions, TSC {args.order} deposit, multigrid "
                               f"2+2 RBGS, "
                               + ("growth-rescaled warm start" if args.guess == "warm_rescaled"
                                  else "warm start extrapolated from the last two potentials")
                               + f", V-cycles until the FP32 "
                               f"rounding floor (relres {args.tol:g} is below it at this size), "
                               f"particles re-sorted by tile every {args.reorder_every} steps, "
                               + ("one pm_kdk call per step" if args.no_chain else
                                  "steps chained (kick-kick-drift fused into interpolation)"),
                   "particles": npart, "grid": n, "deposit": args.order,
                   "vcycles_per_step": cycles},
        "stages_ms_last_step": stages,
        "stage_gbs_last_step": stage_gbs,
        "roofline": roofline,
    }
    ctx.close()
    del off_d, cell_d, vel_d, phi, acc
    torch.cuda.empty_cache()
    if not args.no_extras:
        _log("adjoint (128^3, 20 steps) ...")
        out["adjoint"] = bench_adjoint()
        _log("batched ensemble (96 boxes, 20 steps) ...")
        out["batched"] = bench_batched()
        _log("FFT solvers (256^3) ...")
        out["fft"] = bench_fft()
        _log("f(R) scalaron (512^3 FAS F cycle, 256^3 steps) ...")
        out["fr"] = bench_fr()
    if not args.no_cpu_baseline:
        _log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

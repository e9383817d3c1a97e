"""Batched ensembles: one launch per stage for many boxes of uneven grid sizes,
checked against the plain single-box path box by box (the reference here is
the single-box library path, itself checked against the FP64 oracle in
test_gpu_parity.py), graph replay against eager launches, and the tuner.

Ensemble recipe: per-box grid sizes drawn uniformly from {32, 48, 64, 96, 128},
one particle per cell, spectral index uniform in [-2.5, -1], rms displacement
0.25 cell at a = 0.1, per-box seeds, steps of da = 0.01 (Einstein-de Sitter).
"""
import sys
import time
import warnings

import numpy as np
import pytest
import torch

import icgen

pytestmark = pytest.mark.gpu

A_LIST = [0.1 + 0.01 * i for i in range(21)]
JACOBI_CYCLES = 8   # first solve: relative residual at the FP32 floor (about 2e-5)
WARM_CYCLES = 4     # warm-started solves of later steps


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2410_20501_amd as pm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    warnings.simplefilter("ignore", pm.PMWarning)
    return pm


def ensemble(nboxes, master_seed=4):
    draws = icgen.ensemble_draw(master_seed, nboxes)
    pos, vel = [], []
    for n, ns, seed in draws:
        ps = icgen.zeldovich_particles(n, ns, 0.25, A_LIST[0], seed=seed)
        pos.append(ps.pos)
        vel.append(ps.vel)
    return [d[0] for d in draws], np.concatenate(pos), np.concatenate(vel)


def periodic_maxdist(a, b):
    d = np.abs(a.astype(np.float64) - b.astype(np.float64))
    return float(np.max(np.minimum(d, 1.0 - d)))


def rel(a, b):
    return float(torch.linalg.norm((a - b).double()) / torch.linalg.norm(b.double()))


def batch_params(lib, first):
    if first:
        return lib.default_step_params(fixed_cycles=JACOBI_CYCLES, guess="jacobi")
    return lib.default_step_params(fixed_cycles=WARM_CYCLES, guess="warm_rescaled")


def per_box_run(lib, sizes, pos, vel, p_off, nsteps):
    """The plain path: one context and one pm_kdk call per box and step."""
    outs = []
    first = lib.default_step_params(tol=1e-7, max_cycles=40)
    step = lib.default_step_params(tol=1e-7, max_cycles=40, guess="warm_rescaled")
    for b, n in enumerate(sizes):
        ctx = lib.Context(n, n ** 3)
        pb = pos[p_off[b]:p_off[b + 1]].clone()
        vb = vel[p_off[b]:p_off[b + 1]].clone()
        phi = torch.zeros((n, n, n), device="cuda")
        acc = torch.empty_like(pb)
        lib.pm_accel(ctx, pb, A_LIST[0], phi, acc, params=first)
        for i in range(nsteps):
            lib.pm_kdk(ctx, pb, vb, A_LIST[i], A_LIST[i + 1], phi, acc, params=step)
        torch.cuda.synchronize()
        outs.append((pb, vb, acc, phi.reshape(-1)))
        ctx.close()
    return outs


def test_batch_accel_matches_per_box(lib):
    sizes, pos, vel = ensemble(8)
    _say(f"batch accel vs per-box, sizes {sizes}")
    B = lib.Batch(sizes, [n ** 3 for n in sizes])
    pos_d = torch.from_numpy(pos).cuda()
    acc = torch.zeros_like(pos_d)
    phi = torch.zeros(B.ncell_total, device="cuda")
    relres = lib.pm_batch_accel(B, pos_d, acc, phi, A_LIST[0], batch_params(lib, True),
                                want_relres=True)
    assert max(relres) < 5e-5
    ref = per_box_run(lib, sizes, pos_d, torch.from_numpy(vel).cuda(), B.p_off, 0)
    for b, n in enumerate(sizes):
        ea = rel(acc[B.p_off[b]:B.p_off[b + 1]], ref[b][2])
        ep = rel(phi[B.c_off[b]:B.c_off[b + 1]], ref[b][3])
        _say(f"  box {b} n={n}: acc {ea:.1e} phi {ep:.1e}")
        assert ea < 1e-5 and ep < 1e-5
    B.close()


def test_batch_steps_match_per_box(lib):
    nsteps = 10
    sizes, pos, vel = ensemble(6, master_seed=9)
    _say(f"batch {nsteps} steps vs per-box, sizes {sizes}")
    B = lib.Batch(sizes, [n ** 3 for n in sizes])
    pos_d, vel_d = torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()
    ref = per_box_run(lib, sizes, pos_d, vel_d, B.p_off, nsteps)
    p, v = pos_d.clone(), vel_d.clone()
    acc = torch.zeros_like(p)
    phi = torch.zeros(B.ncell_total, device="cuda")
    lib.pm_batch_accel(B, p, acc, phi, A_LIST[0], batch_params(lib, True))
    lib.pm_batch_kdk(B, p, v, acc, phi, A_LIST[:nsteps + 1], batch_params(lib, False))
    torch.cuda.synchronize()
    for b, n in enumerate(sizes):
        sl = slice(B.p_off[b], B.p_off[b + 1])
        dx = periodic_maxdist(p[sl].cpu().numpy(), ref[b][0].cpu().numpy())
        ea = rel(acc[sl], ref[b][2])
        _say(f"  box {b} n={n}: max |dx| {dx:.1e} box, acc {ea:.1e}")
        assert dx < 1e-4 and ea < 1e-5
    B.close()


def test_graph_replay_matches_eager(lib):
    """Every replay of the captured step agrees with the same step launched eagerly."""
    sizes, pos, vel = ensemble(5, master_seed=11)
    _say(f"graph replay vs eager, sizes {sizes}")
    B = lib.Batch(sizes, [n ** 3 for n in sizes])
    pos_d, vel_d = torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()
    p1 = batch_params(lib, True)
    pw = batch_params(lib, False)
    # eager trajectory, state after every step
    pe, ve = pos_d.clone(), vel_d.clone()
    ae = torch.zeros_like(pe)
    fe = torch.zeros(B.ncell_total, device="cuda")
    lib.pm_batch_accel(B, pe, ae, fe, A_LIST[0], p1)
    eager = []
    for i in range(4):
        lib.pm_batch_kdk(B, pe, ve, ae, fe, A_LIST[i:i + 2], pw)
        torch.cuda.synchronize()
        eager.append((pe.clone(), ae.clone()))
    # graph trajectory from the same start
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pg, vg = pos_d.clone(), vel_d.clone()
        ag = torch.zeros_like(pg)
        fg = torch.zeros(B.ncell_total, device="cuda")
        lib.pm_batch_accel(B, pg, ag, fg, A_LIST[0], p1)
        lib.pm_graph_capture_step(B, pg, vg, ag, fg, pw)
        for i in range(4):
            lib.pm_batch_kdk(B, pg, vg, ag, fg, A_LIST[i:i + 2], pw, use_graph=True)
            s.synchronize()
            junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
            s.synchronize()
            dx = periodic_maxdist(pg.cpu().numpy(), eager[i][0].cpu().numpy())
            ea = rel(ag, eager[i][1])
            _say(f"  replay {i}: max |dx| {dx:.1e}, acc {ea:.1e} ({float(junk):.1f})")
            assert dx < 1e-6 and ea < 1e-5
    B.close()


def test_tuner_choice_and_results(lib):
    sizes, pos, vel = ensemble(5, master_seed=13)
    _say(f"tuner, sizes {sizes}")
    B = lib.Batch(sizes, [n ** 3 for n in sizes])
    pos_d = torch.from_numpy(pos).cuda()
    p1 = batch_params(lib, True)
    acc0 = torch.zeros_like(pos_d)
    phi0 = torch.zeros(B.ncell_total, device="cuda")
    lib.pm_batch_accel(B, pos_d, acc0, phi0, A_LIST[0], p1)
    choice = lib.pm_tune(B, pos_d, torch.zeros_like(phi0), p1)
    _say(f"  choice {choice}")
    assert choice["smooth_rows"] in (1, 2, 4) and choice["gradient_rows"] in (1, 2, 4)
    acc1 = torch.zeros_like(pos_d)
    phi1 = torch.zeros_like(phi0)
    lib.pm_batch_accel(B, pos_d, acc1, phi1, A_LIST[0], p1)
    # a different tile shape changes only the order of independent updates' rounding
    assert rel(acc1, acc0) < 1e-5 and rel(phi1, phi0) < 1e-5
    B.close()


def test_batch_argument_errors(lib):
    B = lib.Batch([32, 48], [32 ** 3, 48 ** 3])
    pos = torch.zeros((B.np_total, 3), device="cuda")
    phi = torch.zeros(B.ncell_total, device="cuda")
    with pytest.raises(lib.PMError):
        lib.pm_batch_accel(B, pos, pos.clone(), phi, 0.1, lib.default_step_params())  # no fixed
    with pytest.raises(lib.PMError):
        lib.pm_batch_accel(B, pos, pos.clone(), phi, 0.1,
                           lib.default_step_params(solver="fft", fixed_cycles=2))
    with pytest.raises(lib.PMError):
        lib.pm_batch_kdk(B, pos, pos.clone(), pos.clone(), phi, [0.1, 0.11],
                         batch_params(lib, False), use_graph=True)  # nothing captured
    with pytest.raises(lib.PMError):
        lib.Batch([30], [27000])  # 30 is not halved (not a multiple of 4): 30^3 > LDS limit
    B.close()


@pytest.mark.timeout(600)
def test_config4_ensemble_graph_vs_per_box_loop(lib):
    """96 boxes, 20 steps: the graph-replayed batch against a loop of plain per-box runs."""
    sizes, pos, vel = ensemble(96, master_seed=2024)
    _say(f"96-box ensemble: {sum(n ** 3 for n in sizes) / 1e6:.1f} M particles")
    B = lib.Batch(sizes, [n ** 3 for n in sizes])
    pos_d, vel_d = torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()
    torch.cuda.synchronize()
    t = time.perf_counter()
    ref = per_box_run(lib, sizes, pos_d, vel_d, B.p_off, 20)
    t_loop = time.perf_counter() - t
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        p, v = pos_d.clone(), vel_d.clone()
        acc = torch.zeros_like(p)
        phi = torch.zeros(B.ncell_total, device="cuda")
        pw = batch_params(lib, False)
        lib.pm_tune(B, p, phi, pw)
        phi.zero_()
        lib.pm_batch_accel(B, p, acc, phi, A_LIST[0], batch_params(lib, True))
        lib.pm_graph_capture_step(B, p, v, acc, phi, pw)
        s.synchronize()
        t = time.perf_counter()
        lib.pm_batch_kdk(B, p, v, acc, phi, A_LIST, pw, use_graph=True)
        s.synchronize()
        t_batch = time.perf_counter() - t
    _say(f"  per-box loop {t_loop:.2f} s (incl. first solves), batched graph {t_batch:.3f} s")
    # trajectories: positions after 20 steps (the two runs round differently, so their
    # accelerations drift apart at the FP32 level, ~1e-5 after 20 steps); forces: the
    # batch's final accelerations against the plain path evaluated at the same positions
    worst_dx, worst_a = 0.0, 0.0
    first = lib.default_step_params(tol=1e-7, max_cycles=40)
    for b, n in enumerate(sizes):
        sl = slice(B.p_off[b], B.p_off[b + 1])
        worst_dx = max(worst_dx, periodic_maxdist(p[sl].cpu().numpy(), ref[b][0].cpu().numpy()))
        ctx = lib.Context(n, n ** 3)
        pb = p[sl].contiguous()
        ab = torch.empty_like(pb)
        lib.pm_accel(ctx, pb, A_LIST[-1], phi[B.c_off[b]:B.c_off[b + 1]].clone().reshape(n, n, n),
                     ab, params=first)
        torch.cuda.synchronize()
        worst_a = max(worst_a, rel(acc[sl], ab))
        ctx.close()
    _say(f"  worst box: max |dx| {worst_dx:.1e} box, acc rel at equal positions {worst_a:.1e}")
    assert worst_dx < 1e-5 and worst_a < 1e-5
    B.close()


# ------------------------------------------------------------------ against the oracle

def _batch_golden():
    """The golden's recipe module and its stored oracle values (tests/golden/
    batch_oracle.json, written by make_batch_golden.py from oracle/ only)."""
    import json
    import os
    golden = os.path.join(os.path.dirname(__file__), "golden")
    if golden not in sys.path:
        sys.path.insert(0, golden)
    import make_batch_golden as mk
    with open(os.path.join(golden, "batch_oracle.json")) as fh:
        return mk, json.load(fh)


def _rel_np(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.timeout(300)
def test_batch_against_oracle_one_box_per_size(lib):
    """One box of each ensemble grid size (32, 48, 64, 96, 128) in one batch, against the
    FP64 oracle box by box: potential and accelerations at the initial state (sampled,
    relative L2 <= 1e-5), positions after 10 steps with the batched step's warm-started
    fixed-cycle solves (sampled, within 1e-4 box units), and the accelerations after the
    10 steps against the oracle's force chain at the batch's own final positions
    (relative L2 <= 1e-5)."""
    from oracle import pm as opm
    mk, gold = _batch_golden()
    sizes = list(mk.SIZES)
    _say(f"batch vs oracle, sizes {sizes}")
    ins = [mk.box_inputs(b) for b in range(len(sizes))]
    B = lib.Batch(sizes, [n ** 3 for n in sizes])
    p = torch.from_numpy(np.concatenate([x for x, _ in ins])).cuda()
    v = torch.from_numpy(np.concatenate([u for _, u in ins])).cuda()
    acc = torch.zeros_like(p)
    phi = torch.zeros(B.ncell_total, device="cuda")
    a = gold["a"]
    lib.pm_batch_accel(B, p, acc, phi, a[0], batch_params(lib, True))
    torch.cuda.synchronize()
    acc0, phi0 = acc.cpu().numpy(), phi.cpu().numpy()
    lib.pm_batch_kdk(B, p, v, acc, phi, a, batch_params(lib, False))
    torch.cuda.synchronize()
    x10, acc10 = p.cpu().numpy(), acc.cpu().numpy()
    for b, n in enumerate(sizes):
        ref = gold["boxes"][b]
        cells, parts = mk.box_samples(b)
        sl = slice(B.p_off[b], B.p_off[b + 1])
        e_phi = _rel_np(phi0[B.c_off[b]:B.c_off[b + 1]][cells], ref["phi0"])
        e_acc0 = _rel_np(acc0[sl][parts], ref["acc0"])
        dx = opm.periodic_distance(x10[sl][parts].astype(np.float64), np.array(ref["x10"])).max()
        xb = x10[sl].astype(np.float64)
        acc_ref = opm.accel(xb * n, n, a[-1])
        e_acc10 = _rel_np(acc10[sl], acc_ref)
        _say(f"  box n={n}: phi0 {e_phi:.1e} acc0 {e_acc0:.1e} |dx|max {dx:.1e} box, "
             f"acc at the final positions {e_acc10:.1e}")
        assert e_phi <= 1e-5 and e_acc0 <= 1e-5
        assert dx <= 1e-4
        assert e_acc10 <= 1e-5
    B.close()


def test_batch_back_to_back_calls_without_host_sync(lib):
    """Two pm_batch_kdk calls with different scale factors queued back to back (no host
    synchronisation between them) give the same result as the same calls with a
    synchronisation in between: the second call's step table never reaches the first."""
    sizes, pos, vel = ensemble(4, master_seed=13)
    _say(f"back-to-back batched calls, sizes {sizes}")
    B = lib.Batch(sizes, [n ** 3 for n in sizes])
    p0, v0 = torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()
    a1 = [0.1, 0.11, 0.12, 0.13]
    a2 = [0.13, 0.15, 0.17, 0.19, 0.21]
    outs = []
    for sync in (True, False):
        p, v = p0.clone(), v0.clone()
        acc = torch.zeros_like(p)
        phi = torch.zeros(B.ncell_total, device="cuda")
        lib.pm_batch_accel(B, p, acc, phi, a1[0], batch_params(lib, True))
        torch.cuda.synchronize()
        lib.pm_batch_kdk(B, p, v, acc, phi, a1, batch_params(lib, False))
        if sync:
            torch.cuda.synchronize()
        lib.pm_batch_kdk(B, p, v, acc, phi, a2, batch_params(lib, False))
        torch.cuda.synchronize()
        outs.append((p.cpu().numpy(), v.cpu().numpy()))
    B.close()
    dx = periodic_maxdist(outs[0][0], outs[1][0])
    ev = float(np.linalg.norm(outs[0][1] - outs[1][1]) / np.linalg.norm(outs[0][1]))
    _say(f"  max |dx| {dx:.1e} box, velocities {ev:.1e}")
    # the batched deposit sums in fixed point: the step is bitwise reproducible
    assert dx == 0.0 and ev == 0.0

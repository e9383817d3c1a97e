"""Chained kick-drift-kick steps (pm_kdk_chain) against the FP64 oracle and against
consecutive pm_kdk calls.

A chain applies the closing half-kick of one step, the opening half-kick of the next
and the next drift together (paper Sect. 3.4: both half-kicks use the accelerations
at the same positions); with the sorted deposit on 8^3 tiles this happens inside the
interpolation kernel. Same tolerances as the step tests: positions 1e-4 box units and
accelerations / velocities 1e-4 relative after 10 steps against the oracle; against
pm_kdk the only difference is FP32 rounding order.
"""
import sys

import numpy as np
import pytest
import torch

import icgen
from oracle import pm as opm

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2410_20501_amd as pm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pm


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _run(lib, n, pos, vel, a_list, order, celloff, chain, reorder_at=()):
    """Steps over a_list; returns positions (box units), velocities, accelerations in
    the input particle order (pm_reorder permutes the arrays; ids undo it)."""
    npart = pos.shape[0]
    ctx = lib.Context(n, npart)
    params = lib.default_step_params(order=order, tol=1e-7, max_cycles=40)
    phi = torch.zeros((n, n, n), device="cuda")
    acc = torch.empty((npart, 3), device="cuda")
    if celloff:
        cell_np, off = icgen.to_cell_offset(pos, n)
        p, cell = dev(off), dev(cell_np, torch.int32)
    else:
        p, cell = dev(pos), None
    v = dev(vel)
    ids = torch.arange(npart, device="cuda", dtype=torch.int64)
    lib.pm_accel(ctx, p, a_list[0], phi, acc, cell=cell, params=params)
    params.mg.guess = lib.PM_GUESS_WARM
    steps = list(zip(a_list[:-1], a_list[1:]))
    for i, (a0, a1) in enumerate(steps):
        if i in reorder_at:
            lib.pm_reorder(ctx, p, vel=v, acc=acc, ids=ids, cell=cell)
        if chain:
            a2 = steps[i + 1][1] if i + 1 < len(steps) else 0.0
            stage = lib.PM_CHAIN_FIRST if i == 0 else lib.PM_CHAIN_NEXT
            lib.pm_kdk_chain(ctx, p, v, a0, a1, a2, stage, phi, acc, cell=cell, params=params)
        else:
            lib.pm_kdk(ctx, p, v, a0, a1, phi, acc, cell=cell, params=params)
    x = host(p)
    if celloff:
        x = icgen.from_cell_offset(host(cell).astype(np.int64), x, n)
    order_ = np.argsort(host(ids).astype(np.int64))
    return x[order_], host(v)[order_], host(acc)[order_]


@pytest.mark.parametrize("order", ["sorted", "atomic"])
@pytest.mark.parametrize("celloff", [False, True])
def test_chain_ten_steps_against_oracle(lib, order, celloff):
    """10 chained steps a = 0.1 -> 0.2 at 64^3 (fused drift with the sorted deposit on
    tiles, separate kick-drift otherwise), particles re-sorted after step 4."""
    _say(f"chain ten steps order={order} celloff={celloff}")
    n = 64
    ps = icgen.zeldovich_particles(n, -1.5, 0.3, 0.1, seed=2)
    a_list = list(np.linspace(0.1, 0.2, 11))
    x, v, acc = _run(lib, n, ps.pos, ps.vel, a_list, order, celloff, chain=True, reorder_at=(4,))
    xr, vr, accr = opm.run(ps.pos.astype(np.float64), ps.vel.astype(np.float64), a_list, n,
                           solver="exact7")
    assert opm.periodic_distance(x, xr).max() <= 1e-4
    assert rel_l2(acc, accr) <= 1e-4
    assert rel_l2(v, vr) <= 1e-4


@pytest.mark.parametrize("celloff", [False, True])
def test_chain_matches_consecutive_steps(lib, celloff):
    """6 steps at 48^3 (n % 8 == 0: tile path), re-sort after steps 2 and 3: the chain and
    six pm_kdk calls agree to FP32 rounding order."""
    _say(f"chain vs pm_kdk celloff={celloff}")
    n = 48
    ps = icgen.zeldovich_particles(n, -2.0, 0.4, 0.2, seed=5)
    a_list = [0.2, 0.22, 0.25, 0.27, 0.3, 0.32, 0.35]
    xc, vc, ac = _run(lib, n, ps.pos, ps.vel, a_list, "sorted", celloff, chain=True,
                      reorder_at=(2, 3))
    xk, vk, ak = _run(lib, n, ps.pos, ps.vel, a_list, "sorted", celloff, chain=False,
                      reorder_at=(2, 3))
    assert opm.periodic_distance(xc, xk).max() <= 2e-6
    assert rel_l2(vc, vk) <= 1e-5
    assert rel_l2(ac, ak) <= 1e-5


def test_chain_single_step_is_kdk(lib):
    """A chain of one step (PM_CHAIN_FIRST, a2 = 0) is pm_kdk."""
    _say("chain of one step")
    n = 32
    ps = icgen.zeldovich_particles(n, -2.0, 0.3, 0.1, seed=7)
    a_list = [0.1, 0.12]
    xc, vc, ac = _run(lib, n, ps.pos, ps.vel, a_list, "sorted", True, chain=True)
    xk, vk, ak = _run(lib, n, ps.pos, ps.vel, a_list, "sorted", True, chain=False)
    assert np.array_equal(xc, xk)
    assert np.array_equal(vc, vk)
    assert np.array_equal(ac, ak)


def test_chain_rejects_bad_stage(lib):
    _say("chain argument errors")
    n = 16
    ctx = lib.Context(n, 8)
    p = torch.rand((8, 3), device="cuda")
    v = torch.zeros((8, 3), device="cuda")
    acc = torch.zeros((8, 3), device="cuda")
    phi = torch.zeros((n, n, n), device="cuda")
    with pytest.raises(lib.PMError):
        lib.pm_kdk_chain(ctx, p, v, 0.1, 0.2, 0.3, 7, phi, acc)
    with pytest.raises(lib.PMError):
        lib.pm_kdk_chain(ctx, p, v, 0.1, float("nan"), 0.3, lib.PM_CHAIN_FIRST, phi, acc)

"""f(R) gravity on the GPU against the FP64 oracle (oracle/fr.py).

The scalaron solve is FP64 on both sides and runs the same FAS cycles, so the GPU's u
matches the oracle's to rounding: |du| <= 1e-9 (u is about 1), and the reported relative
residuals agree to 1e-6 relative. Accelerations (FP32 Newtonian solve and force chain)
relative L2 <= 1e-5 at a shared state; positions within 1e-4 box units after 10 steps.
"""
import sys
import warnings

import numpy as np
import pytest
import torch

import icgen
from oracle import fr as ofr
from oracle import pm as opm

pytestmark = pytest.mark.gpu

OM, OL = 0.3, 0.7


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2410_20501_amd as pm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    warnings.simplefilter("ignore", pm.PMWarning)
    return pm


def _lognormal(n, sigma, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    rho = np.exp(sigma * g.standard_normal((n, n, n)))
    return (rho / rho.mean()).astype(np.float32)


def _fr_params(lib, f0, n_exp, box, **kw):
    return lib.default_step_params(omega_m=OM, omega_l=OL, fr_f0=f0, fr_n=n_exp,
                                   fr_c2=ofr.c_tilde(box) ** 2, **kw)


@pytest.mark.parametrize("n,n_exp,cycle,cycles,f0", [
    (32, 1, "F", 1, -1e-5), (32, 2, "F", 1, -1e-5), (48, 1, "F", 2, -1e-6),
    (64, 1, "V", 2, -1e-5), (64, 2, "W", 1, -1e-6), (128, 1, "F", 1, -1e-6),
    (128, 2, "F", 1, -1e-6), (256, 1, "F", 1, -1e-6), (256, 2, "V", 1, -1e-6),
    # f_R0 = -1e-8: q of order -66 and p > 0 in every cell (the cubic's one-real-root
    # form with a positive p)
    (32, 1, "F", 1, -1e-8), (32, 2, "F", 1, -1e-8)])
def test_scalaron_solve_parity(lib, n, n_exp, cycle, cycles, f0):
    rho = _lognormal(n, 1.0, 30 + n + n_exp)
    a = 0.5
    p = _fr_params(lib, f0, n_exp, 100.0, fr_cycle=cycle, fr_cycles=cycles)
    ctx = lib.Context(n)
    u = torch.ones((n, n, n), dtype=torch.float64, device="cuda")
    rr = lib.pm_solve_fr(ctx, torch.from_numpy(rho).cuda(), a, p, u, relres=True)
    co = ofr.Coeffs(a, f0, n_exp, ofr.c_tilde(100.0) ** 2, OM, OL)
    ref, hist = ofr.solve(rho.astype(np.float64), co, cycles=cycles, cycle=cycle)
    du = float(np.abs(u.cpu().numpy() - ref).max())
    _say(f"fr solve n={n} nexp={n_exp} {cycle}x{cycles}: max|du| {du:.2e}, relres "
         f"{rr[0]:.3e} -> {rr[1]:.3e} (oracle {hist[0]:.3e} -> {hist[-1]:.3e}), "
         f"u in [{ref.min():.3f}, {ref.max():.3f}]")
    ctx.close()
    assert ref.min() < 0.7 and hist[-1] < hist[0] / 5
    assert du <= 1e-9
    assert rr[0] == pytest.approx(hist[0], rel=1e-6)
    assert rr[1] == pytest.approx(hist[-1], rel=1e-6)


@pytest.mark.parametrize("n,n_exp,cycle,pre,post,relres", [
    (256, 1, "F", 2, 1, True), (320, 2, "F", 2, 1, True), (256, 1, "W", 1, 2, False),
    (512, 1, "F", 2, 1, True)])  # the benchmark's size, where no oracle run fits
def test_streaming_sweep_matches_colour_passes(lib, n, n_exp, cycle, pre, post, relres):
    """Grids of 256 cells per side and more (a multiple of 64) sweep in one streaming pass
    per red-black sweep when u is 16-byte aligned (the finest grid then forms its s from
    the density inside its passes, and writes s itself only for the residual norms); an
    8-byte offset u takes the two colour passes and the written s. Red-black Gauss-Seidel
    does not depend on the order of the cells within a colour and both paths evaluate the
    same arithmetic: the same bits. The W case (256^3 visited twice per cycle, one pre- and
    two post-sweeps) runs without the norms, so nothing writes the finest s before the
    streaming run."""
    rho = torch.from_numpy(_lognormal(n, 1.0, 60 + n_exp)).cuda()
    p = _fr_params(lib, -1e-5, n_exp, 100.0, fr_cycle=cycle, fr_cycles=2, fr_pre=pre,
                   fr_post=post)
    ctx = lib.Context(n)
    u_al = torch.ones((n, n, n), dtype=torch.float64, device="cuda")
    buf = torch.ones(n ** 3 + 1, dtype=torch.float64, device="cuda")
    u_off = buf[1:].view(n, n, n)
    assert u_al.data_ptr() % 16 == 0 and u_off.data_ptr() % 16 == 8
    rr_al = lib.pm_solve_fr(ctx, rho, 0.5, p, u_al, relres=relres)
    rr_off = lib.pm_solve_fr(ctx, rho, 0.5, p, u_off, relres=relres)
    diff = float((u_al - u_off).abs().max())
    _say(f"fr streaming vs colour passes n={n} nexp={n_exp} {cycle} {pre}+{post}: max|du| "
         f"{diff:.1e}, relres {rr_al} / {rr_off}")
    ctx.close()
    assert diff == 0.0 and rr_al == rr_off
    assert float((u_al - 1.0).abs().max()) > 1e-3  # the solve moved u
    if relres:
        assert rr_al[1] < rr_al[0] / 5


def test_scalaron_background_is_fixed(lib):
    n = 32
    p = _fr_params(lib, -1e-5, 1, 100.0)
    ctx = lib.Context(n)
    u = torch.ones((n, n, n), dtype=torch.float64, device="cuda")
    rr = lib.pm_solve_fr(ctx, torch.ones((n, n, n), device="cuda"), 0.7, p, u, relres=True)
    dev = float((u - 1.0).abs().max())
    ctx.close()
    assert dev < 1e-13 and rr[1] < 1e-13


def _accel_case(lib, n, n_exp, solver, f0, box, a=0.5, seed=40):
    ps = icgen.zeldovich_particles(n, -2.0, 0.5, a, seed=seed)
    ctx = lib.Context(n, n ** 3)
    p = _fr_params(lib, f0, n_exp, box, gravity="fr", solver=solver, order="sorted",
                   tol=1e-7, max_cycles=40)
    phi = torch.zeros((n, n, n), device="cuda")
    acc = torch.empty((n ** 3, 3), device="cuda")
    lib.pm_accel(ctx, torch.from_numpy(ps.pos).cuda(), a, phi, acc, params=p)
    x = ps.pos.astype(np.float64) * n
    ref, fl = ofr.accel(x, n, a, f0, n_exp, ofr.c_tilde(box) ** 2, OM, OL, return_fields=True)
    newton = opm.accel(x, n, a, omega_m=OM)
    ctx.close()
    return acc.cpu().numpy(), ref, newton, fl


@pytest.mark.parametrize("n_exp,solver", [(1, "mg"), (2, "mg"), (1, "fft_7pt")])
def test_accel_parity(lib, n_exp, solver):
    n = 32
    acc, ref, newton, fl = _accel_case(lib, n, n_exp, solver, -1e-5, 64.0)
    e = float(np.linalg.norm(acc - ref) / np.linalg.norm(ref))
    boost = float(np.linalg.norm(ref) / np.linalg.norm(newton))
    _say(f"fr accel nexp={n_exp} {solver}: acc rel l2 {e:.2e}, |F_fR| / |F_N| {boost:.3f}, "
         f"u in [{fl['u'].min():.3f}, {fl['u'].max():.3f}]")
    assert boost > 1.01
    assert e <= 1e-5


def test_accel_parity_64(lib):
    acc, ref, newton, _ = _accel_case(lib, 64, 1, "mg", -1e-6, 128.0, seed=41)
    e = float(np.linalg.norm(acc - ref) / np.linalg.norm(ref))
    _say(f"fr accel 64^3 f0 -1e-6: acc rel l2 {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("n_exp", [1, 2])
def test_ten_steps(lib, n_exp):
    """10 KDK steps a = 0.5 -> 1 in LCDM with f(R), each scalaron solve (one F cycle)
    starting from the previous one, 32^3."""
    n, f0, box = 32, -1e-5, 64.0
    ps = icgen.zeldovich_particles(n, -2.0, 0.4, 0.5, seed=42 + n_exp)
    a_list = list(np.linspace(0.5, 1.0, 11))
    ctx = lib.Context(n, n ** 3)
    p = _fr_params(lib, f0, n_exp, box, gravity="fr", order="sorted", tol=1e-7, max_cycles=40)
    pos, vel = torch.from_numpy(ps.pos).cuda(), torch.from_numpy(ps.vel).cuda()
    phi = torch.zeros((n, n, n), device="cuda")
    acc = torch.empty_like(pos)
    lib.pm_accel(ctx, pos, a_list[0], phi, acc, params=p)
    p.mg.guess = lib.PM_GUESS_WARM_RESCALED
    for a0, a1 in zip(a_list[:-1], a_list[1:]):
        lib.pm_kdk(ctx, pos, vel, a0, a1, phi, acc, params=p)
    xr, vr, _, _ = ofr.run(ps.pos.astype(np.float64), ps.vel.astype(np.float64), a_list, n, f0,
                           n_exp, ofr.c_tilde(box) ** 2, OM, OL)
    dx = opm.periodic_distance(pos.cpu().numpy(), xr).max()
    ev = float(np.linalg.norm(vel.cpu().numpy() - vr) / np.linalg.norm(vr))
    _say(f"fr ten steps nexp={n_exp}: max |dx| {dx:.2e} box, v rel l2 {ev:.2e}")
    ctx.close()
    assert dx <= 1e-4 and ev <= 1e-4


def test_fr_argument_errors(lib):
    n = 16
    ctx = lib.Context(n, 16)
    pos = torch.rand((16, 3), device="cuda")
    phi = torch.zeros((n, n, n), device="cuda")
    acc = torch.empty_like(pos)
    for kw in (dict(fr_n=3), dict(fr_f0=1e-5), dict(fr_f0=0.0), dict(fr_c2=0.0),
               dict(fr_cycles=0), dict(fr_pre=0), dict(fr_post=0), dict(fr_coarse_sweeps=0),
               dict(fr_cycle=5), dict(solver="full_fft")):
        p = lib.default_step_params(gravity="fr", omega_m=OM, omega_l=OL, **kw)
        with pytest.raises(lib.PMError) as e:
            lib.pm_accel(ctx, pos, 0.5, phi, acc, params=p)
        assert e.value.code == lib.PM_ERR_ARG, kw
    u = torch.ones((n, n, n), dtype=torch.float64, device="cuda")
    rho = torch.ones((n, n, n), device="cuda")
    with pytest.raises(lib.PMError):
        lib.pm_solve_fr(ctx, rho, -0.5, lib.default_step_params(), u)
    with pytest.raises(TypeError):
        lib.pm_solve_fr(ctx, rho, 0.5, lib.default_step_params(), u.float())
    ctx.close()

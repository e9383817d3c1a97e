"""GPU initial conditions (pm_ic_lpt, Lagrangian perturbation theory to third order) and
the power-spectrum estimator (pm_power_spectrum) against the FP64 oracle (oracle/ics.py)
on the same seeded white noise and P(k) table.

Bounds: velocities (which carry the displacements without the FP32 rounding of a box
position) relative L2 <= 1e-5 for the whole field, and <= 1e-4 for the increment of each
order over the order below (the second- and third-order terms are 10 and 100 times
smaller, so the same FP32 rounding is a larger share of them); positions in the
cell-offset form within 2e-5 cell of the oracle; P(k) per shell <= 1e-5 relative, mode
counts exact.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import ics as oics

pytestmark = pytest.mark.gpu

A0 = 0.5
K_TAB, P_TAB = oics.power_law_table(0.1, -2.0, kmin=1.0, kmax=1e4)  # rms displacement about 0.5 cell at n = 32


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2410_20501_amd as pm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pm


def _noise(n, seed):
    return np.random.Generator(np.random.PCG64(seed)).standard_normal((n, n, n)).astype(np.float32)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _gpu_state(lib, n, noise, order, dealias, celloff):
    ctx = lib.Context(n, n ** 3)
    pos = torch.empty((n ** 3, 3), device="cuda")
    vel = torch.empty((n ** 3, 3), device="cuda")
    cell = torch.empty(n ** 3, dtype=torch.int32, device="cuda") if celloff else None
    lib.pm_ic_lpt(ctx, torch.from_numpy(noise).cuda(), K_TAB, P_TAB, A0, pos, vel, cell=cell,
                  order=order, dealias=dealias)
    torch.cuda.synchronize()
    out = (pos.cpu().numpy().astype(np.float64), vel.cpu().numpy().astype(np.float64),
           None if cell is None else cell.cpu().numpy())
    ctx.close()
    return out


@pytest.mark.parametrize("n,dealias", [(32, False), (32, True), (64, True)])
def test_lpt_parity_by_order(lib, n, dealias):
    noise = _noise(n, 40 + n)
    prev_g = prev_o = None
    for order in (1, 2, 3):
        _say(f"lpt n={n} order={order} dealias={dealias}")
        _, v, _ = _gpu_state(lib, n, noise, order, dealias, celloff=False)
        _, vr = oics.lpt_state(noise.astype(np.float64), K_TAB, P_TAB, A0, order, dealias)
        e = _rel(v, vr)
        msg = f"  velocities rel l2 {e:.2e}"
        assert e <= 1e-5, msg
        if prev_g is not None:
            ei = _rel(v - prev_g, vr - prev_o)
            share = np.linalg.norm(vr - prev_o) / np.linalg.norm(vr)
            msg += f"; order-{order} increment ({share:.1e} of the field) rel l2 {ei:.2e}"
            assert ei <= 1e-4, msg
        _say(msg)
        prev_g, prev_o = v, vr


@pytest.mark.parametrize("order", [1, 3])
def test_lpt_positions_cell_offset_and_box(lib, order):
    n = 32
    noise = _noise(n, 77)
    xr, _ = oics.lpt_state(noise.astype(np.float64), K_TAB, P_TAB, A0, order, True)
    off, _, cell = _gpu_state(lib, n, noise, order, True, celloff=True)
    c = cell.astype(np.int64)
    ijk = np.stack([c // (n * n), (c // n) % n, c % n], axis=-1)
    x = (ijk + off) / n
    d = x - xr
    d -= np.round(d)
    err_cells = np.abs(d).max() * n
    box, _, _ = _gpu_state(lib, n, noise, order, True, celloff=False)
    db = box - xr
    db -= np.round(db)
    _say(f"lpt positions order={order}: cell-offset max err {err_cells:.2e} cell, "
         f"box max err {np.abs(db).max():.2e} box")
    assert err_cells <= 2e-5
    assert np.abs(db).max() <= 2e-5 / n + 2.0 ** -23
    assert off.min() >= 0.0 and off.max() < 1.0


@pytest.mark.parametrize("deconv", [0, 3])
@pytest.mark.parametrize("n", [32, 128])
def test_power_spectrum_parity(lib, n, deconv):
    _say(f"power spectrum n={n} deconv={deconv}")
    noise = _noise(n, 5)
    dk = oics.linear_density_spectrum(noise.astype(np.float64), K_TAB, P_TAB)
    rho = (1.0 + 0.5 * np.fft.irfftn(dk, s=(n, n, n), axes=(0, 1, 2))).astype(np.float32)
    ctx = lib.Context(n)
    pk, km, nm = lib.pm_power_spectrum(ctx, torch.from_numpy(rho).cuda(), deconv=deconv)
    ctx.close()
    pr, kr, cr = oics.power_spectrum(rho.astype(np.float64), deconv=deconv)
    np.testing.assert_array_equal(np.array(nm), cr)
    np.testing.assert_allclose(km, kr, rtol=1e-12)
    e = np.max(np.abs(np.array(pk) - pr) / pr)
    _say(f"  max rel per shell {e:.2e}")
    assert e <= 1e-5


def test_ic_argument_errors(lib):
    ctx = lib.Context(32, 32 ** 3)
    noise = torch.zeros((32, 32, 32), device="cuda")
    pos = torch.empty((32 ** 3, 3), device="cuda")
    vel = torch.empty_like(pos)
    with pytest.raises(lib.PMError) as e:
        lib.pm_ic_lpt(ctx, noise, [1.0, 2.0], [1.0, 1.0], 0.1, pos, vel, order=4)
    assert e.value.code == lib.PM_ERR_ARG
    with pytest.raises(lib.PMError) as e:
        lib.pm_ic_lpt(ctx, noise, [2.0, 1.0], [1.0, 1.0], 0.1, pos, vel)
    assert e.value.code == lib.PM_ERR_ARG
    ctx.close()
    ctx = lib.Context(48, 48 ** 3)
    with pytest.raises(lib.PMError) as e:
        lib.pm_ic_lpt(ctx, torch.zeros((48, 48, 48), device="cuda"), [1.0, 2.0], [1.0, 1.0], 0.1,
                      torch.empty((48 ** 3, 3), device="cuda"), torch.empty((48 ** 3, 3), device="cuda"))
    assert e.value.code == lib.PM_ERR_SHAPE
    ctx.close()

"""Host-side guards that need a device context: the opt-in finite check of particle
positions and velocities (PM_CREATE_CHECK_FINITE) rejects NaN and Inf before any kernel
reads them, and passes finite input through unchanged."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2410_20501_amd as pm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pm


def _state(n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    pos = torch.from_numpy(g.random((n ** 3, 3), dtype=np.float32)).cuda()
    vel = torch.from_numpy((1e-3 * g.standard_normal((n ** 3, 3))).astype(np.float32)).cuda()
    return pos, vel


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
def test_nonfinite_positions_rejected(lib, bad):
    n = 16
    ctx = lib.Context(n, n ** 3, flags=lib.PM_CREATE_CHECK_FINITE)
    pos, vel = _state(n, 1)
    pos[1234, 1] = bad
    phi = torch.zeros((n, n, n), device="cuda")
    acc = torch.zeros_like(pos)
    p = lib.default_step_params()
    with pytest.raises(lib.PMError) as e:
        lib.pm_accel(ctx, pos, 0.5, phi, acc, params=p)
    assert e.value.code == lib.PM_ERR_NONFINITE
    with pytest.raises(lib.PMError) as e:
        lib.pm_kdk(ctx, pos, vel, 0.5, 0.51, phi, acc, params=p)
    assert e.value.code == lib.PM_ERR_NONFINITE
    ctx.close()


def test_nonfinite_velocity_rejected_and_finite_accepted(lib):
    n = 16
    ctx = lib.Context(n, n ** 3, flags=lib.PM_CREATE_CHECK_FINITE)
    pos, vel = _state(n, 2)
    phi = torch.zeros((n, n, n), device="cuda")
    acc = torch.zeros_like(pos)
    p = lib.default_step_params()
    lib.pm_accel(ctx, pos, 0.5, phi, acc, params=p)
    pos0 = pos.clone()
    lib.pm_kdk(ctx, pos, vel, 0.5, 0.51, phi, acc, params=p)
    assert not torch.equal(pos, pos0) and bool(torch.isfinite(acc).all())
    vel[7, 0] = float("nan")
    before = pos.clone()
    with pytest.raises(lib.PMError) as e:
        lib.pm_kdk(ctx, pos, vel, 0.51, 0.52, phi, acc, params=p)
    assert e.value.code == lib.PM_ERR_NONFINITE
    assert torch.equal(pos, before)
    ctx.close()


"""The allocation-free FFT solve (pm_solve_fft_noalloc, for callers that cannot
allocate device memory) against the context entry point pm_solve_fft on the same
inputs, through the C ABI: two calls in a row, the second on a smaller grid (the
static scratch keeps the first call's contents), and the size limit."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from oracle import pm as opm

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2410_20501_amd as pm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = ctypes.CDLL(pm.hippm.LIB_PATH)
    c.pm_solve_fft_noalloc.restype = ctypes.c_int
    c.pm_solve_fft_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_void_p]
    return pm, c


def _noalloc(c, rho, coef, deconv, phi):
    return c.pm_solve_fft_noalloc(ctypes.c_void_p(rho.data_ptr()), rho.shape[0], coef, deconv,
                                  ctypes.c_void_p(phi.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _density(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return (1.0 + 0.3 * rng.standard_normal((n, n, n))).astype(np.float32)


def test_noalloc_fft_matches_context_entry_point(lib):
    pm, c = lib
    for n, deconv, seed in ((128, 3, 1), (32, 2, 2), (64, 0, 3), (8, 3, 4)):
        _say(f"noalloc fft n={n} deconv={deconv}")
        rho_h = _density(n, seed)
        rho = torch.from_numpy(rho_h).cuda()
        phi_a = torch.full((n, n, n), float("nan"), device="cuda")
        phi_b = torch.zeros((n, n, n), device="cuda")
        assert _noalloc(c, rho, 0.3, deconv, phi_a) == pm.PM_OK
        ctx = pm.Context(n)
        pm.pm_solve_fft(ctx, rho, 0.3, phi_b, deconv=deconv)
        torch.cuda.synchronize()
        a, b = phi_a.cpu().numpy(), phi_b.cpu().numpy()
        ctx.close()
        assert np.array_equal(a, b), float(np.abs(a - b).max())
        ref = opm.solve_fft(0.3 * (rho_h.astype(np.float64) - rho_h.astype(np.float64).mean()),
                            1.0 / n, deconv)
        assert np.linalg.norm(a - ref) <= 1e-5 * np.linalg.norm(ref)


def test_noalloc_fft_rejects_sizes_beyond_its_scratch(lib):
    pm, c = lib
    for n in (256, 48, 4):
        rho = torch.ones((n, n, n), device="cuda")
        phi = torch.zeros_like(rho)
        assert _noalloc(c, rho, 1.0, 3, phi) == pm.PM_ERR_SHAPE
    rho = torch.ones((16, 16, 16), device="cuda")
    assert _noalloc(c, rho, 1.0, 5, rho) == pm.PM_ERR_ARG

"""Pins of the oracle adjoint (finite differences, transposition identities) and the inputs."""
import numpy as np
import pytest

import icgen
from oracle import pm, adjoint

RNG = lambda s: np.random.Generator(np.random.PCG64(s))  # noqa: E731


def _fd(fun, x, d, eps):
    return (fun(x + eps * d) - fun(x - eps * d)) / (2 * eps)


@pytest.mark.parametrize("mas", ["tsc", "cic"])
def test_deposit_vjp_matches_finite_differences(mas):
    n = 8
    rng = RNG(41)
    x = rng.uniform(0.05, 0.95, size=(40, 3))
    rb = rng.standard_normal((n, n, n))
    xb = adjoint.deposit_vjp(x, n, rb, mas)
    fun = lambda y: np.sum(rb * pm.deposit(y * n, n, mas))  # noqa: E731
    for _ in range(3):
        d = rng.standard_normal(x.shape)
        fd = _fd(fun, x, d, 1e-7)
        assert np.sum(xb * d) == pytest.approx(fd, rel=1e-5 if mas == "tsc" else 1e-3)


def test_interp_vjp_transpose_and_position_derivative():
    n = 8
    rng = RNG(43)
    x = rng.uniform(0, 1, size=(30, 3))
    g = rng.standard_normal((n, n, n, 3))
    lam = rng.standard_normal((30, 3))
    gb, xb = adjoint.interp_vjp(x, g, lam)
    g2 = rng.standard_normal((n, n, n, 3))
    assert np.sum(gb * g2) == pytest.approx(np.sum(lam * pm.interp(x * n, g2)), rel=1e-12)
    fun = lambda y: np.sum(lam * pm.interp(y * n, g))  # noqa: E731
    d = rng.standard_normal(x.shape)
    assert np.sum(xb * d) == pytest.approx(_fd(fun, x, d, 1e-7), rel=1e-5)


def test_gradient_and_solve_vjp_transposition():
    n, h = 8, 1.0 / 8
    rng = RNG(47)
    phi = rng.standard_normal((n, n, n))
    gb = rng.standard_normal((n, n, n, 3))
    assert np.sum(pm.gradient(phi, h) * gb) == pytest.approx(np.sum(phi * adjoint.gradient_vjp(gb, h)), rel=1e-12)
    rho = rng.standard_normal((n, n, n))
    pb = rng.standard_normal((n, n, n))
    coef = 0.45
    lhs = np.sum(pm.solve_exact7(coef * (rho - rho.mean()), h) * pb)
    assert lhs == pytest.approx(np.sum(rho * adjoint.solve_vjp(pb, h, coef)), rel=1e-12)


def test_accel_vjp_matches_finite_differences():
    n = 8
    rng = RNG(53)
    x = rng.uniform(0, 1, size=(64, 3))
    lam = rng.standard_normal((64, 3))
    xb = adjoint.accel_vjp(x, n, 0.3, lam)
    fun = lambda y: np.sum(lam * pm.accel(y * n, n, 0.3))  # noqa: E731
    for _ in range(2):
        d = rng.standard_normal(x.shape)
        assert np.sum(xb * d) == pytest.approx(_fd(fun, x, d, 1e-7), rel=1e-5)


def test_initial_condition_gradient_matches_finite_differences():
    n = 8
    ps = icgen.zeldovich_particles(n, -1.5, 0.3, 0.1, seed=5)
    c = (np.arange(n) + 0.5) / n
    q = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    psi = ps.vel.astype(np.float64) / np.sqrt(0.1)
    a_list = [0.1, 0.15, 0.2, 0.25]
    w = RNG(55).uniform(0, 1, size=(n, n, n))
    loss, grad = adjoint.ic_gradient(psi, q, a_list, n, w)
    rng = RNG(56)
    for _ in range(3):
        d = rng.standard_normal(psi.shape)
        d /= np.linalg.norm(d)
        eps = 1e-3 * np.sqrt(np.mean(np.sum(psi ** 2, -1)))
        fd = _fd(lambda p: adjoint.ic_loss(p, q, a_list, n, w), psi, d, eps)
        assert np.sum(grad * d) == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(loss))


# ---------------------------------------------------------------- inputs

def test_ic_rms_and_spectrum_slope():
    n, ns = 32, -1.5
    psi = icgen.displacement_field(n, ns, 0.3, seed=2)
    rms = np.sqrt(np.mean(np.sum(psi ** 2, -1))) * n
    assert rms == pytest.approx(0.3, rel=1e-12)
    # divergence of Psi in Fourier space gives -delta; its shell power follows k^ns
    dk = sum(1j * (2 * np.pi * np.fft.fftfreq(n, 1.0 / n)).reshape([-1 if a == d else 1 for a in range(3)])
             * np.fft.fftn(psi[..., d]) for d in range(3))
    m = np.fft.fftfreq(n, 1.0 / n)
    kk = np.sqrt(m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2)
    shells = [(2, 4), (6, 10)]
    p = [np.mean(np.abs(dk[(kk >= lo) & (kk < hi)]) ** 2) for lo, hi in shells]
    kc = [np.mean(kk[(kk >= lo) & (kk < hi)]) for lo, hi in shells]
    slope = np.log(p[1] / p[0]) / np.log(kc[1] / kc[0])
    assert slope == pytest.approx(ns, abs=0.25)


def test_cell_offset_roundtrip():
    n = 16
    ps = icgen.zeldovich_particles(n, -2.0, 0.2, 0.1, seed=1)
    cell, off = icgen.to_cell_offset(ps.pos, n)
    assert off.min() >= 0 and off.max() < 1 and cell.min() >= 0 and cell.max() < n ** 3
    back = icgen.from_cell_offset(cell, off, n)
    assert pm.periodic_distance(back, ps.pos).max() < 1e-7 / n


# ---------------------------------------------------------------- differentiable run, 32^3

def _fd_golden():
    """The golden's recipe module and its stored values."""
    import json
    import os
    import sys
    golden = os.path.join(os.path.dirname(__file__), "golden")
    if golden not in sys.path:
        sys.path.insert(0, golden)
    import make_fd_golden as mk
    with open(os.path.join(golden, "fd_32.json")) as fh:
        return mk, json.load(fh)


def test_oracle_adjoint_matches_fp64_finite_differences_per_direction():
    """The oracle's reverse leapfrog against FP64 central differences of its own forward
    run (exact seven-point solve), 32^3, 20 steps, 64 normalised white-noise directions:
    every direction to 1e-3 relative. The differences come from tests/golden/fd_32.json
    (written by make_fd_golden.py, oracle only); their own error, estimated from the same
    difference at twice the step, must be far below the bound."""
    mk, gold = _fd_golden()
    fd = np.array(gold["fd"])
    fd2 = np.array(gold["fd_2eps"])
    assert np.max(np.abs(fd2 - fd) / np.abs(fd)) < 1e-4
    psi, q, w = mk.inputs()
    loss, grad = adjoint.ic_gradient(psi.astype(np.float64), q.astype(np.float64), mk.A_RUN,
                                     mk.N, w.astype(np.float64))
    assert loss == pytest.approx(gold["loss"], rel=1e-12)
    ad = np.array([np.sum(grad * d) for d in mk.directions()])
    rel = np.abs(ad - fd) / np.abs(fd)
    assert rel.max() < 1e-3, (rel.max(), int(np.argmax(rel)))
    # the stored differences are reproducible from the committed recipe
    fd0, _ = mk.fd_one(0)
    assert fd0 == pytest.approx(fd[0], rel=1e-9)

"""Pins of the background, parametrised-gravity and QUMOND oracle (oracle/gravity.py)."""
import numpy as np
import pytest
from scipy.special import hyp2f1

from oracle import gravity as og
from oracle import pm

RNG = lambda s: np.random.Generator(np.random.PCG64(s))  # noqa: E731


def test_tau_closed_forms():
    """Supercomoving time: Einstein-de Sitter 2 (a0^-1/2 - a1^-1/2); flat LCDM
    T(a1) - T(a0) with T(a) = -2 a^-1/2 2F1(1/2, -1/6; 5/6; -(Omega_L / Omega_m) a^3) /
    sqrt(Omega_m) (the integral of a^-3/2 (Omega_m + Omega_L a^3)^-1/2 by the
    substitution s = a^3)."""
    assert og.tau(0.1, 0.11) == pytest.approx(pm.tau_eds(0.1, 0.11), rel=1e-13)
    om, ol = 0.3, 0.7
    T = lambda a: -2.0 / np.sqrt(om) * a ** -0.5 * hyp2f1(0.5, -1.0 / 6.0, 5.0 / 6.0, -ol / om * a ** 3)  # noqa: E731
    for a0, a1 in ((0.02, 0.05), (0.1, 0.5), (0.5, 1.0)):
        assert og.tau(a0, a1, om, ol) == pytest.approx(T(a1) - T(a0), rel=1e-11)


def test_mu_parametrisation():
    """mu(a) = 1 + mu0 Omega_L(a) / Omega_L0: mu0 is the coupling today (flat LCDM), and
    the deviation fades in the matter era."""
    om, ol = 0.3, 0.7
    assert og.mu_of_a(1.0, 0.4, om, ol) == pytest.approx(1.4, rel=1e-14)
    a = 0.5
    ola = ol / (om * a ** -3 + ol)                      # Omega_L(a)
    assert og.mu_of_a(a, 0.4, om, ol) == pytest.approx(1.0 + 0.4 * ola / ol, rel=1e-14)
    assert og.mu_of_a(0.01, 0.4, om, ol) - 1.0 < 1e-5
    with pytest.raises(ValueError):
        og.mu_of_a(0.5, 0.1, 1.0, 0.0)


def test_nu_functions_limits_and_duality():
    """nu -> 1 for y >> 1 and y^-1/2 for y << 1; the simple function is the inverse of
    mu(x) = x / (1 + x) (g = nu(y) g_N solves mu(g/g0) g = g_N); the n-family with n = 1
    is the simple function; the delta family is the gamma family without its second term
    at gamma = 1."""
    for fam, par in (("simple", 1.0), ("n", 2.0), ("beta", 1.0), ("gamma", 2.0), ("delta", 2.0)):
        assert og.nu_function(1e8, fam, par) == pytest.approx(1.0, abs=1e-7)
        assert og.nu_function(1e-10, fam, par) * 1e-5 == pytest.approx(1.0, rel=1e-3)
    y = np.geomspace(1e-3, 1e3, 50)
    x = og.nu_function(y, "simple") * y
    np.testing.assert_allclose(x / (1.0 + x) * x, y, rtol=1e-12)
    np.testing.assert_allclose(og.nu_function(y, "n", 1.0), og.nu_function(y, "simple"), rtol=1e-14)
    np.testing.assert_allclose(og.nu_function(y, "delta", 1.0), og.nu_function(y, "gamma", 1.0),
                               rtol=1e-14)


def _brute_source(phin, h, g0):
    """The discrete MOND source by explicit index loops (simple nu)."""
    n = phin.shape[0]
    P = lambda i, j, k: phin[i % n, j % n, k % n]  # noqa: E731
    out = np.zeros_like(phin)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                tot = 0.0
                for ax in range(3):
                    for side in (0, 1):                 # face A (side 0) or B (side 1)
                        c = [i, j, k]
                        lo = list(c)
                        if side == 0:
                            lo[ax] -= 1                 # face between lo and lo + e_ax
                        hi = list(lo)
                        hi[ax] += 1
                        g = [0.0, 0.0, 0.0]
                        g[ax] = (P(*hi) - P(*lo)) / h
                        for t in range(3):
                            if t == ax:
                                continue
                            e = [0, 0, 0]
                            e[t] = 1
                            d_hi = P(hi[0] + e[0], hi[1] + e[1], hi[2] + e[2]) - P(hi[0] - e[0], hi[1] - e[1], hi[2] - e[2])
                            d_lo = P(lo[0] + e[0], lo[1] + e[1], lo[2] + e[2]) - P(lo[0] - e[0], lo[1] - e[1], lo[2] - e[2])
                            g[t] = (d_hi + d_lo) / (4 * h)
                        mag = np.sqrt(sum(q * q for q in g))
                        nu = 0.5 + 0.5 * np.sqrt(1.0 + 4.0 * g0 / mag)
                        flux = nu * g[ax]
                        tot += flux if side == 1 else -flux
                out[i, j, k] = tot / h
    return out


def test_qumond_source_brute_force_and_newtonian_limit():
    """The oracle's vectorised source against explicit index loops on a 6^3 grid, and
    the Newtonian limit: with nu = 1 the source is the seven-point Laplacian of phi_N, so
    the MOND potential is the Newtonian one."""
    n, h = 6, 1.0 / 6
    phin = RNG(4).standard_normal((n, n, n))
    got = og.qumond_source(phin, h, 0.7)
    np.testing.assert_allclose(got, _brute_source(phin, h, 0.7), rtol=1e-12, atol=1e-12)
    n, h = 16, 1.0 / 16
    f = RNG(5).standard_normal((n, n, n))
    f -= f.mean()
    phin = pm.solve_exact7(f, h)
    s = og.qumond_source(phin, h, 1e-30)
    np.testing.assert_allclose(s, pm.laplacian7(phin, h), atol=1e-9 * np.abs(f).max())
    np.testing.assert_allclose(pm.solve_exact7(s, h), phin, atol=1e-9 * np.abs(phin).max())


def test_qumond_boosts_a_weak_field():
    """In the deep-MOND regime (g0 far above the Newtonian field) a test mass is pulled
    towards a point mass harder than in Newtonian gravity, and the boost grows with
    distance (the MOND force falls as 1/r instead of 1/r^2)."""
    n = 32
    src = np.array([[16.5, 16.5, 16.5]])
    probes = np.array([[16.5 + 3.0, 16.5, 16.5], [16.5 + 8.0, 16.5, 16.5]])
    u = np.concatenate([src, probes])
    an = pm.accel(u, n, 1.0, "exact7", "tsc")
    am = og.qumond_accel(u, n, 1.0, g0=1e3)
    assert am[1, 0] < an[1, 0] < 0 and am[2, 0] < an[2, 0] < 0
    assert am[2, 0] / an[2, 0] > am[1, 0] / an[1, 0] > 1.0

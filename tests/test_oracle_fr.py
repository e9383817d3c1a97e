"""Pins of the f(R) oracle (oracle/fr.py): the closed-form roots against numpy's
polynomial roots, the background as the exact fixed point, each smoothed cell solving its
own discrete equation, the FAS fixed point against a Newton solve of the field equation
written in the scalaron itself, the linear-regime solution in closed form (the 1/3 force
enhancement below the Compton wavelength), and the Newtonian limit."""
import numpy as np
import pytest

from oracle import fr
from oracle import mg as omg
from oracle import pm

RNG = lambda s: np.random.Generator(np.random.PCG64(s))  # noqa: E731
OM, OL = 0.3, 0.7


def _largest_real_root(coeffs):
    r = np.roots(coeffs)
    return max(z.real for z in r if abs(z.imag) <= 1e-9 * max(1.0, abs(z)))


def test_cubic_roots_match_polynomial_roots():
    g = RNG(1)
    p = np.concatenate([g.uniform(-3, 3, 400), [0.0, 2.0, -2.0, -0.75]])
    q = -np.concatenate([10 ** g.uniform(-6, 0.5, 400), [0.3, 1e-3, 1e-3, 0.25]])
    u = fr.root_cubic(p, q)
    d0, d1 = -3 * p, 27 * q
    branches = {"zero": p == 0, "one": (p != 0) & ((p > 0) | (d1 ** 2 - 4 * d0 ** 3 > 0)),
                "three": (p < 0) & (d1 ** 2 - 4 * d0 ** 3 <= 0)}
    assert all(b.any() for b in branches.values())
    for i in range(len(p)):
        ref = _largest_real_root([1.0, 0.0, p[i], q[i]])
        assert u[i] == pytest.approx(ref, rel=1e-9, abs=1e-12), (p[i], q[i])
        assert u[i] > 0
    scale = np.abs(u) ** 3 + np.abs(p * u) + np.abs(q)
    assert (np.abs(u ** 3 + p * u + q) / scale).max() < 1e-9


def test_quartic_roots_match_polynomial_roots():
    g = RNG(2)
    p = np.concatenate([g.uniform(-3, 3, 400), [0.0, 1.0, -1.0]])
    q = -np.concatenate([10 ** g.uniform(-6, 0.5, 400), [0.5, 1e-3, 1e-3]])
    u = fr.root_quartic(p, q)
    assert (p > 0).any() and (p < 0).any() and (p == 0).any()
    for i in range(len(p)):
        ref = _largest_real_root([1.0, 0.0, 0.0, p[i], q[i]])
        assert u[i] == pytest.approx(ref, rel=1e-8, abs=1e-12), (p[i], q[i])
    scale = u ** 4 + np.abs(p * u) + np.abs(q)
    assert (np.abs(u ** 4 + p * u + q) / scale).max() < 1e-9


def _polished_root(coeffs):
    """Largest real root from numpy, refined by Newton steps in extended precision."""
    x = np.longdouble(_largest_real_root(coeffs))
    c = [np.longdouble(v) for v in coeffs]
    deg = len(c) - 1
    for _ in range(6):
        f = sum(ci * x ** (deg - i) for i, ci in enumerate(c))
        df = sum((deg - i) * ci * x ** (deg - i - 1) for i, ci in enumerate(c[:-1]))
        x = x - f / df
    return float(x)


def test_roots_near_zero_and_large_p():
    """Where the neighbour term nearly balances the source (p near 0) and in deep
    screening (large p, small root) both closed forms keep full precision."""
    ps = [s * 10.0 ** e for e in (-12, -9, -6, -3, 0, 2, 4) for s in (1.0, -1.0)]
    for q in (-1e-6, -1e-3, -1.0, -70.0):
        p = np.array(ps)
        u3, u4 = fr.root_cubic(p, q), fr.root_quartic(p, q)
        for i, pi in enumerate(ps):
            r3 = _polished_root([1.0, 0.0, pi, q])
            r4 = _polished_root([1.0, 0.0, 0.0, pi, q])
            assert u3[i] == pytest.approx(r3, rel=1e-12), (pi, q)
            assert u4[i] == pytest.approx(r4, rel=1e-12), (pi, q)


def test_background_values():
    """f_R_bar(1) = f_R0; R_bar in units of H0^2/c^2 is 3 (Omega_m a^-3 + 4 Omega_L);
    c~ for a 100 Mpc/h box is c / (100 km/s/Mpc * 100 Mpc)."""
    assert fr.fr_bar(1.0, -1e-5, 1, OM, OL) == pytest.approx(-1e-5, rel=1e-15)
    assert fr.r_bar(0.5, OM, OL) == pytest.approx(3 * (OM * 8 + 2.8), rel=1e-15)
    ratio = (3 * (OM + 4 * OL)) / (3 * (OM / 0.125 + 4 * OL))
    assert fr.fr_bar(0.5, -1e-5, 2, OM, OL) == pytest.approx(ratio ** 3 * -1e-5, rel=1e-14)
    assert fr.c_tilde(100.0) == pytest.approx(29.9792458, rel=1e-15)


@pytest.mark.parametrize("n_exp", [1, 2])
def test_uniform_density_is_the_fixed_point(n_exp):
    co = fr.Coeffs(0.4, -1e-5, n_exp, fr.c_tilde(128.0) ** 2, OM, OL)
    rho = np.ones((16, 16, 16))
    u, hist = fr.solve(rho, co, cycles=2)
    assert np.abs(u - 1.0).max() < 1e-13
    assert hist[-1] < 1e-13


@pytest.mark.parametrize("n_exp", [1, 2])
def test_each_smoothed_cell_solves_its_equation(n_exp):
    """After a red half-sweep every red cell satisfies N_h(u) = s given its neighbours."""
    n, h = 8, 1.0 / 8
    co = fr.Coeffs(0.7, -1e-5, n_exp, fr.c_tilde(64.0) ** 2, OM, OL)
    g = RNG(3 + n_exp)
    rho = np.exp(0.8 * g.standard_normal((n, n, n)))
    rho /= rho.mean()
    s = co.source(rho)
    u = 1.0 + 0.2 * g.random((n, n, n))
    fr.nl_sweep(u, s, h, co, order=(0,))
    red = ~omg._colour_mask(n)
    res = (s - fr.operator(u, h, co))[red]
    assert np.abs(res).max() <= 1e-9 * np.abs(s).max()


def _newton_scalaron(rho, co, n_exp, iters=60):
    """Newton's method on the field equation written in f~ (Eq. fr_sim_2 with the
    seven-point Laplacian): F(f) = lap7 f + cA (rho - mean) - K [(f_bar / f)^(1/(n+1)) - 1],
    a dense Jacobian over all cells."""
    n = rho.shape[0]
    h = 1.0 / n
    N = n ** 3
    idx = np.arange(N).reshape(n, n, n)
    L = np.zeros((N, N))
    for ax in range(3):
        for sh in (1, -1):
            L[idx.ravel(), np.roll(idx, sh, axis=ax).ravel()] += 1.0 / (h * h)
    L[np.arange(N), np.arange(N)] -= 6.0 / (h * h)
    b = co.cA * (rho - rho.mean()).ravel()
    e = 1.0 / (n_exp + 1)
    f = np.full(N, co.fbar)
    for _ in range(iters):
        x = co.fbar / f
        F = L @ f + b - co.K * (x ** e - 1.0)
        J = L + np.diag(co.K * e * x ** e / f)
        step = np.linalg.solve(J, -F)
        # keep the scalaron on the background's side of zero
        t = 1.0
        while np.any((f + t * step) / co.fbar <= 0):
            t *= 0.5
        f = f + t * step
        if np.abs(step).max() < 1e-14 * abs(co.fbar):
            break
    return f.reshape(n, n, n), np.abs(F).max()


@pytest.mark.parametrize("n_exp", [1, 2])
def test_fas_fixed_point_matches_newton(n_exp):
    """Many FAS cycles on 8^3 converge to the scalaron that Newton's method finds for the
    un-substituted field equation (no u, no polynomial, no closed-form roots)."""
    n = 8
    co = fr.Coeffs(0.6, -2e-6, n_exp, fr.c_tilde(32.0) ** 2, OM, OL)
    g = RNG(10 + n_exp)
    rho = np.exp(1.2 * g.standard_normal((n, n, n)))
    rho /= rho.mean()
    u, hist = fr.solve(rho, co, cycles=25)
    assert hist[-1] < 1e-12
    f_fas = fr.scalaron(u, co)
    f_newton, res = _newton_scalaron(rho, co, n_exp)
    # the field is screened somewhere (f~ well below its background) and not elsewhere
    ratio = f_newton / co.fbar
    assert ratio.min() < 0.5 and ratio.max() > 1.0
    assert np.abs(f_fas - f_newton).max() <= 1e-9 * abs(co.fbar)


@pytest.mark.parametrize("n_exp", [1, 2])
def test_linear_regime_closed_form(n_exp):
    """A small single-mode density contrast in an unscreened background: the scalaron
    perturbation is delta f~_k = (n+1) f~_bar cA delta_k / ((n+1) f~_bar k7^2 - K), and the
    total potential of the mode is the Newtonian one times 1 + (1/3) k7^2 / (k7^2 + m^2),
    m^2 = -K / ((n+1) f~_bar), with k7^2 the seven-point Laplacian's eigenvalue."""
    n, A, mode = 16, 1e-5, 2
    h = 1.0 / n
    co = fr.Coeffs(1.0, -1e-4, n_exp, fr.c_tilde(200.0) ** 2, OM, OL)
    x = np.arange(n)
    delta = A * np.cos(2 * np.pi * mode * x / n)[:, None, None] * np.ones((n, n, n))
    rho = 1.0 + delta
    u, hist = fr.solve(rho, co, cycles=12)
    assert hist[-1] < 1e-10
    df = fr.scalaron(u, co) - co.fbar
    k2 = 4.0 / h ** 2 * np.sin(np.pi * mode / n) ** 2
    lin = (n_exp + 1) * co.fbar * co.cA * delta / ((n_exp + 1) * co.fbar * k2 - co.K)
    assert np.abs(df - lin).max() <= 1e-3 * np.abs(lin).max()
    phin = pm.solve_exact7(pm.source(rho, 1.0, OM), h)
    phi = phin - 0.5 * co.c2 * fr.scalaron(u, co)
    phi -= phi.mean()
    m2 = -co.K / ((n_exp + 1) * co.fbar)
    boost = 1.0 + k2 / (3.0 * (k2 + m2))
    assert 1.05 < boost < 4.0 / 3.0
    assert np.abs(phi - boost * phin).max() <= 1e-3 * np.abs(phin).max()


def test_fas_cycles_converge():
    """On a clustered 32^3 density one F cycle cuts the residual by at least 5x, and V
    and W cycles also converge."""
    n = 32
    co = fr.Coeffs(0.5, -1e-5, 1, fr.c_tilde(100.0) ** 2, OM, OL)
    g = RNG(20)
    rho = np.exp(1.0 * g.standard_normal((n, n, n)))
    rho /= rho.mean()
    for cyc in ("F", "V", "W"):
        _, hist = fr.solve(rho, co, cycles=3, cycle=cyc)
        assert hist[1] < hist[0] / 5 and hist[3] < hist[2], (cyc, hist)


def test_tiny_f_r0_recovers_newton():
    n = 16
    g = RNG(21)
    x = g.random((n ** 3, 3)) * n
    acc = fr.accel(x, n, 0.5, -1e-13, 1, fr.c_tilde(100.0) ** 2)
    ref = pm.accel(x, n, 0.5, omega_m=OM)
    assert np.linalg.norm(acc - ref) <= 1e-6 * np.linalg.norm(ref)

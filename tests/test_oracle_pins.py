"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the paper's
worked example, closed forms, a textbook dense solve, brute force on tiny
inputs, invariants and convergence orders.
"""
import os

import numpy as np
import pytest

from oracle import pm, mg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = lambda s: np.random.Generator(np.random.PCG64(s))  # noqa: E731


# ---------------------------------------------------------------- deposit

def test_point_mass_worked_example():
    """Paper App. D: point mass at a cell centre / cell corner."""
    n = 8
    rows = []
    with open(os.path.join(GOLDEN, "point_mass_deposit.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    assert len(rows) == 4
    for scheme, place, count, vals in rows:
        u = np.array([[3.5, 4.5, 5.5]]) if place == "centre" else np.array([[3.0, 4.0, 5.0]])
        rho = pm.deposit(u, n, scheme, mass=1.0)
        nz = rho[rho != 0.0]
        assert nz.size == int(count), (scheme, place)
        ax = np.array([float(v) for v in vals.split(",")])
        expect = np.sort(np.einsum("i,j,k->ijk", ax, ax, ax).ravel())
        np.testing.assert_allclose(np.sort(nz), expect, rtol=0, atol=1e-15)
        assert rho.sum() == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("mas", ["tsc", "cic", "ngp"])
def test_deposit_brute_force_definition(mas):
    """Every (particle, cell) pair evaluated with the paper's piecewise window."""
    n = 6
    rng = RNG(11)
    u = rng.uniform(0, n, size=(17, 3))
    u[0] = [0.0, 5.999999, 3.0]          # on faces / near the wrap
    u[1] = [2.5, 2.5, 2.5]               # cell centre
    win = {"tsc": pm.w_tsc, "cic": pm.w_cic, "ngp": pm.w_ngp}[mas]
    ref = np.zeros((n, n, n))
    c = np.arange(n) + 0.5
    for p in range(u.shape[0]):
        s = [u[p, d] - c for d in range(3)]
        s = [(x + n / 2) % n - n / 2 for x in s]     # minimum image
        w = [win(x) for x in s]
        ref += np.einsum("i,j,k->ijk", *w)
    got = pm.deposit(u, n, mas, mass=1.0)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("mas", ["tsc", "cic", "ngp"])
def test_deposit_mass_conservation_and_lattice(mas):
    n = 16
    rng = RNG(3)
    u = rng.uniform(0, n, size=(5000, 3))
    rho = pm.deposit(u, n, mas)
    assert rho.sum() == pytest.approx(n ** 3, rel=1e-12)
    i = (np.arange(n) + 0.5)
    lattice = np.stack(np.meshgrid(i, i, i, indexing="ij"), -1).reshape(-1, 3)
    np.testing.assert_allclose(pm.deposit(lattice, n, mas), 1.0, atol=1e-14)


# ---------------------------------------------------------------- interpolation

@pytest.mark.parametrize("mas", ["tsc", "cic"])
def test_interp_partition_of_unity_and_linear_exactness(mas):
    n = 12
    rng = RNG(5)
    u = rng.uniform(3, 9, size=(200, 3))          # away from the periodic seam
    const = np.full((n, n, n, 3), 2.5)
    np.testing.assert_allclose(pm.interp(u, const, mas), 2.5, atol=1e-13)
    c = np.arange(n) + 0.5
    lin = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1)   # g_c = cell centre
    np.testing.assert_allclose(pm.interp(u, lin, mas), u, atol=1e-12)


@pytest.mark.parametrize("mas", ["tsc", "cic", "ngp"])
def test_interp_is_transpose_of_deposit(mas):
    n = 10
    rng = RNG(7)
    u = rng.uniform(0, n, size=(300, 3))
    q = rng.standard_normal(300)
    g = rng.standard_normal((n, n, n))
    lhs = np.sum(pm.deposit_charges(u, n, q, mas) * g)
    rhs = np.sum(q * pm.interp(u, g, mas))
    assert lhs == pytest.approx(rhs, rel=1e-12)


# ---------------------------------------------------------------- Poisson

def _dense_laplacian(n, h):
    """7-point periodic Laplacian as an explicit matrix, from index arithmetic."""
    N = n ** 3
    A = np.zeros((N, N))
    for i in range(n):
        for j in range(n):
            for k in range(n):
                r = (i * n + j) * n + k
                A[r, r] = -6.0 / h ** 2
                for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    c = (((i + di) % n) * n + (j + dj) % n) * n + (k + dk) % n
                    A[r, c] += 1.0 / h ** 2
    return A


def test_exact7_matches_dense_solve_8cubed():
    n, h = 8, 1.0 / 8
    f = RNG(13).standard_normal((n, n, n))
    A = _dense_laplacian(n, h)
    ones = np.ones((n ** 3, 1))
    phi_dense = np.linalg.solve(A + ones @ ones.T, (f - f.mean()).ravel())
    np.testing.assert_allclose(pm.solve_exact7(f, h).ravel(), phi_dense, rtol=0, atol=1e-12 * np.abs(phi_dense).max())
    # the oracle's stencil is the dense operator
    np.testing.assert_allclose(pm.laplacian7(f, h).ravel(), A @ f.ravel(), atol=1e-10)


def test_exact7_single_mode_closed_form():
    n, h = 32, 1.0 / 32
    i = np.arange(n)
    m = (3, 5, 1)
    theta = 2 * np.pi * (m[0] * i[:, None, None] + m[1] * i[None, :, None] + m[2] * i[None, None, :]) / n
    f = np.cos(theta)
    lam = sum(2.0 * (np.cos(2 * np.pi * md / n) - 1.0) for md in m) / h ** 2
    np.testing.assert_allclose(pm.solve_exact7(f, h), f / lam, atol=1e-14)


def test_fft_solver_single_mode_closed_form():
    """Paper Sect. 3.8: phi(k) = -f(k) / (k^2 W_TSC(k)^2), W_TSC = prod sinc^3(omega/2)."""
    n, h = 32, 1.0 / 32
    i = np.arange(n)
    m = (2, -7, 4)
    theta = 2 * np.pi * (m[0] * i[:, None, None] + m[1] * i[None, :, None] + m[2] * i[None, None, :]) / n
    f = np.sin(theta)
    k = [2 * np.pi * md for md in m]
    k2 = sum(kd * kd for kd in k)
    w = 1.0
    for kd in k:
        x = kd * h / 2
        w *= (np.sin(x) / x) ** 3
    np.testing.assert_allclose(pm.solve_fft(f, h, 3), -f / (k2 * w * w), atol=1e-15)
    # Nyquist mode: omega = pi, sinc(pi/2) = 2/pi
    f = np.cos(np.pi * i)[:, None, None] * np.ones((n, n, n))
    expect = -f / ((np.pi * n) ** 2 * (2 / np.pi) ** 6)
    np.testing.assert_allclose(pm.solve_fft(f, h, 3), expect, atol=1e-15)


def test_ngp_window_cells():
    """NGP (paper Sect. 3.5): every particle lands whole in the cell that contains it,
    floor(u) per axis, including a particle on a cell face and one at the periodic seam."""
    n = 5
    u = np.array([[0.2, 3.99, 4.5], [2.0, 0.0, 1.0], [4.999999, 2.5, 0.5]])
    rho = pm.deposit(u, n, "ngp", mass=1.0)
    assert np.count_nonzero(rho) == 3 and rho.sum() == 3.0
    for p in u.astype(int):
        assert rho[p[0], p[1], p[2]] == 1.0
    g = RNG(3).standard_normal((n, n, n))
    np.testing.assert_array_equal(pm.interp(u, g, "ngp"), g[tuple(u.astype(int).T)])


def _mode(n, m, fn=np.cos):
    i = np.arange(n)
    theta = 2 * np.pi * (m[0] * i[:, None, None] + m[1] * i[None, :, None] + m[2] * i[None, None, :]) / n
    return fn(theta)


def test_fft_7pt_single_mode_and_seven_point_system():
    """FFT_7pt (paper Sect. 3.8): on a single mode, phi = f / lambda(m) with the
    seven-point eigenvalue lambda = sum_d 2 (cos(2 pi m_d / n) - 1) / h^2 (the closed
    form written independently of the sinc form the solver uses), and on any field the
    result solves the seven-point system, i.e. equals the exact seven-point solve (the
    equivalence of multigrid and FFT_7pt the paper reports)."""
    n, h = 32, 1.0 / 32
    m = (3, -5, 7)
    f = _mode(n, m)
    lam = sum(2.0 * (np.cos(2 * np.pi * md / n) - 1.0) for md in m) / h ** 2
    np.testing.assert_allclose(pm.solve_fft_7pt(f, h), f / lam, atol=1e-14)
    r = RNG(19).standard_normal((n, n, n))
    r -= r.mean()
    phi = pm.solve_fft_7pt(r, h)
    np.testing.assert_allclose(pm.laplacian7(phi, h), r, atol=1e-10 * np.abs(r).max())
    np.testing.assert_allclose(phi, pm.solve_exact7(r, h), atol=1e-13 * np.abs(phi).max())


@pytest.mark.parametrize("p", [3, 2])
def test_full_fft_force_single_mode_closed_form(p):
    """FULL_FFT (paper Sect. 3.8, Eq. exact_fullfft_kernel): for f = cos(k . x) the
    potential is -f / (k^2 W^2) and the force -grad phi = -k sin(k . x) / (k^2 W^2),
    W = prod_d sinc(k_d h / 2)^p. On the Nyquist plane of an axis the derivative along
    that axis is 0 (the self-conjugate mode has no real odd image)."""
    n, h = 16, 1.0 / 16
    m = (2, -3, 5)
    f = _mode(n, m)
    k = [2 * np.pi * md for md in m]
    k2 = sum(kd * kd for kd in k)
    w = 1.0
    for kd in k:
        w *= (np.sin(kd * h / 2) / (kd * h / 2)) ** p
    g = pm.force_full_fft(f, h, p)
    s = _mode(n, m, np.sin)
    for d in range(3):
        np.testing.assert_allclose(g[..., d], -k[d] * s / (k2 * w * w), atol=1e-15)
    # a mode on the Nyquist plane of axis 0: no force along axis 0, the others as above
    m = (-8, 1, 2)
    f = _mode(n, m)
    g = pm.force_full_fft(f, h, 0)
    k = [2 * np.pi * md for md in m]
    assert np.abs(g[..., 0]).max() < 1e-15
    s = _mode(n, m, np.sin)
    for d in (1, 2):
        np.testing.assert_allclose(g[..., d], -k[d] * s / sum(kd * kd for kd in k), atol=1e-15)


def test_multigrid_converges_to_exact7_and_rate():
    n, h = 32, 1.0 / 32
    f = RNG(17).standard_normal((n, n, n))
    f -= f.mean()
    u, hist = mg.solve(f, h, tol=1e-12, max_cycles=30)
    ref = pm.solve_exact7(f, h)
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-10
    rates = [hist[i] / hist[i + 1] for i in range(1, 5)]
    # paper App. C: about a factor 10 per V-cycle without over-relaxation
    assert all(4.0 < r < 60.0 for r in rates), rates


@pytest.mark.parametrize("cycle", ["V", "W", "F"])
def test_multigrid_cycle_shapes_and_convergence(cycle, monkeypatch):
    """Cycle shapes by their textbook definitions, counted on a 64 -> 32 -> 16 hierarchy:
    one cycle visits level l (0 the finest) once (V), 2^l times (W) or l + 1 times (F);
    every shape converges to the exact seven-point solution, W and F at least as fast
    per cycle as V (on three levels the coarse problem is already well solved by one V
    cycle, so the gain is small)."""
    n, h = 64, 1.0 / 64
    f = RNG(29).standard_normal((n, n, n))
    f -= f.mean()
    visits = {}
    real_coarse = mg.coarse_solve
    real_sweep = mg.rbgs_sweep

    def sweep(u, *a, **k):
        key = ("sweep", u.shape[0])
        visits[key] = visits.get(key, 0) + 1
        return real_sweep(u, *a, **k)

    def coarse(u, *a, **k):
        visits[("coarse", u.shape[0])] = visits.get(("coarse", u.shape[0]), 0) + 1
        monkeypatch.setattr(mg, "rbgs_sweep", real_sweep)   # its own sweeps are not visits
        try:
            return real_coarse(u, *a, **k)
        finally:
            monkeypatch.setattr(mg, "rbgs_sweep", sweep)

    monkeypatch.setattr(mg, "rbgs_sweep", sweep)
    monkeypatch.setattr(mg, "coarse_solve", coarse)
    mg.vcycle(-(h * h) * f / 6.0, f, h, pre=2, post=2, cycle=cycle)
    expect = {"V": (1, 1, 1), "W": (1, 2, 4), "F": (1, 2, 3)}[cycle]
    assert visits[("sweep", 64)] == 4 * expect[0]      # pre + post sweeps per visit
    assert visits[("sweep", 32)] == 4 * expect[1]
    assert visits[("coarse", 16)] == expect[2]
    monkeypatch.undo()
    u, hist = mg.solve(f, h, tol=1e-11, max_cycles=40, cycle=cycle)
    ref = pm.solve_exact7(f, h)
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-9
    _, hv = mg.solve(f, h, tol=0.0, max_cycles=3, cycle="V")
    _, hc = mg.solve(f, h, tol=0.0, max_cycles=3, cycle=cycle)
    if cycle != "V":
        assert hc[3] < hv[3], (hc, hv)


def test_multigrid_restriction_is_scaled_prolongation_transpose():
    rng = RNG(19)
    r = rng.standard_normal((8, 8, 8))
    v = rng.standard_normal((4, 4, 4))
    assert np.sum(mg.restrict(r, "fw") * v) == pytest.approx(np.sum(r * mg.prolong(v)) / 8.0, rel=1e-13)
    # paper's prolongation weights: a single coarse value spreads as (1,3,3,1)/4 per axis
    e = np.zeros((4, 4, 4))
    e[1, 1, 1] = 1.0
    p = mg.prolong(e)
    assert p[2, 2, 2] == pytest.approx(27 / 64)
    assert p[1, 2, 2] == pytest.approx(9 / 64)
    assert p[1, 1, 2] == pytest.approx(3 / 64)
    assert p[1, 1, 1] == pytest.approx(1 / 64)
    assert p.sum() == pytest.approx(8.0)


@pytest.mark.parametrize("restriction", ["fw", "avg"])
def test_truncation_error_single_mode_closed_form(restriction):
    """tau = L_H(R u) - R(L_h u) for u = cos(k . x) sampled at cell centres: the
    seven-point operator multiplies the mode by lambda_h = sum_d (2 cos(k_d h) - 2) / h^2
    (lambda_H with H = 2h on the coarse grid), and the restriction by rho = prod_d of
    (2 cos(3 k_d h / 2) + 6 cos(k_d h / 2)) / 8 (full weighting over the fine centres at
    -3h/2 .. 3h/2 from the coarse centre) or cos(k_d h / 2) (mean of the two children),
    so tau = (lambda_H - lambda_h) rho cos(k . X) on the coarse centres X."""
    n = 32
    h, H = 1.0 / n, 2.0 / n
    for m in ([1, 0, 0], [2, 3, 1], [5, -4, 7]):
        k = 2 * np.pi * np.array(m, dtype=np.float64)
        x = (np.arange(n) + 0.5) * h
        X = (np.arange(n // 2) + 0.5) * H
        u = np.cos(k[0] * x[:, None, None] + k[1] * x[None, :, None] + k[2] * x[None, None, :])
        lam_h = np.sum(2 * np.cos(k * h) - 2) / h ** 2
        lam_H = np.sum(2 * np.cos(k * H) - 2) / H ** 2
        if restriction == "fw":
            rho = np.prod((2 * np.cos(1.5 * k * h) + 6 * np.cos(0.5 * k * h)) / 8)
        else:
            rho = np.prod(np.cos(0.5 * k * h))
        expect = (lam_H - lam_h) * rho * np.cos(
            k[0] * X[:, None, None] + k[1] * X[None, :, None] + k[2] * X[None, None, :])
        got = mg.truncation_error(u, h, restriction)
        np.testing.assert_allclose(got, expect, atol=1e-9 * abs(lam_h))


def test_truncation_error_stop_rule():
    """solve(alpha=...) stops at the first cycle whose residual norm is below alpha times
    the norm of the truncation-error estimate of the same iterate."""
    n, h = 32, 1.0 / 32
    rng = RNG(23)
    f = rng.standard_normal((n, n, n))
    f = mg.prolong(mg.restrict(f))  # a smoother source, so that tau is well above the floor
    f -= f.mean()
    alpha = 0.5
    u, hist = mg.solve(f, h, alpha=alpha, max_cycles=30)
    c = len(hist) - 1
    assert 1 <= c < 30

    def check(cycles):
        v = -(h * h) * f / 6.0
        for _ in range(cycles):
            mg.vcycle(v, f, h)
        return np.linalg.norm(f - pm.laplacian7(v, h)), np.linalg.norm(mg.truncation_error(v, h))

    d, t = check(c)
    assert d < alpha * t
    d, t = check(c - 1)
    assert d >= alpha * t


# ---------------------------------------------------------------- gradient

def test_gradient_single_mode_multiplier_and_identities():
    n, h = 32, 1.0 / 32
    i = np.arange(n)
    m = 5
    omega = 2 * np.pi * m / n
    phi = np.sin(omega * i)[None, :, None] * np.ones((n, n, n))
    g = pm.gradient(phi, h)
    mult = ((4.0 / 3.0) * np.sin(omega) - (1.0 / 6.0) * np.sin(2 * omega)) / h
    np.testing.assert_allclose(g[..., 1], -mult * np.cos(omega * i)[None, :, None] * np.ones((n, n, n)), atol=1e-12)
    np.testing.assert_allclose(g[..., 0], 0.0, atol=1e-13)
    assert np.abs(pm.gradient(np.full((n, n, n), 3.0), h)).max() < 1e-12
    rng = RNG(23)
    a, b = rng.standard_normal((2, n, n, n))
    for ax in range(3):
        assert np.sum(pm.derivative(a, h, ax) * b) == pytest.approx(-np.sum(a * pm.derivative(b, h, ax)), rel=1e-12)


def test_gradient_fourth_order_convergence():
    errs = []
    for n in (16, 32):
        h = 1.0 / n
        x = (np.arange(n) + 0.5) * h
        phi = np.exp(np.sin(2 * np.pi * x))[:, None, None] * np.ones((n, n, n))
        exact = -(2 * np.pi * np.cos(2 * np.pi * x) * np.exp(np.sin(2 * np.pi * x)))
        errs.append(np.abs(pm.gradient(phi, h)[:, 0, 0, 0] - exact).max())
    assert 12.0 < errs[0] / errs[1] < 20.0, errs


# ---------------------------------------------------------------- force chain

@pytest.mark.parametrize("solver", ["exact7", "fft", "fft_7pt", "full_fft"])
@pytest.mark.parametrize("mas", ["tsc", "cic"])
def test_self_force_zero_and_pair_antisymmetry(solver, mas):
    n = 16
    rng = RNG(29)
    one = rng.uniform(0, n, size=(1, 3))
    a1 = pm.accel(one, n, 1.0, solver, mas, mass=1.0)
    assert np.abs(a1).max() < 1e-12
    two = rng.uniform(0, n, size=(2, 3))
    a2 = pm.accel(two, n, 1.0, solver, mas, mass=1.0)
    assert np.abs(a2).max() > 1e-6
    np.testing.assert_allclose(a2[0], -a2[1], atol=1e-12 * np.abs(a2).max())
    many = rng.uniform(0, n, size=(400, 3))
    am = pm.accel(many, n, 1.0, solver, mas)
    assert np.abs(am.sum(axis=0)).max() < 1e-10 * np.abs(am).sum()


def test_point_mass_far_field_is_attractive():
    """A test mass is pulled towards a point mass (paper App. D)."""
    n = 32
    src = np.array([[16.5, 16.5, 16.5]])
    probe = np.array([[16.5 + 6.0, 16.5, 16.5]])
    u = np.concatenate([src, probe])
    acc = pm.accel(u, n, 1.0, "exact7", "tsc", mass=np.array(1.0))
    assert acc[1, 0] < 0 and abs(acc[1, 1]) < 1e-12 and abs(acc[1, 2]) < 1e-12


# ---------------------------------------------------------------- integrator

def test_tau_closed_form_numbers():
    assert pm.tau_eds(0.1, 0.11) == pytest.approx(0.294328, rel=2e-6)
    a = 0.02 + 0.0196 * np.arange(51)
    total = sum(pm.tau_eds(a0, a1) for a0, a1 in zip(a[:-1], a[1:]))
    assert total == pytest.approx(2 * (0.02 ** -0.5 - 1.0), rel=1e-12)
    # d^2 D / d tau^2 = 1.5 a Omega_m D for D = a: check by finite differences of a(tau)
    a0, eps = 0.3, 1e-4
    # a(tau) = (a0^{-1/2} - tau/2)^{-2}
    at = lambda t: (a0 ** -0.5 - t / 2) ** -2  # noqa: E731
    d2 = (at(eps) - 2 * at(0) + at(-eps)) / eps ** 2
    assert d2 == pytest.approx(1.5 * a0 * a0, rel=1e-6)


def test_kdk_time_reversal():
    n = 16
    rng = RNG(31)
    x = rng.uniform(0, 1, size=(2000, 3))
    v = 0.01 * rng.standard_normal((2000, 3))
    a_list = [0.1, 0.12, 0.14, 0.16]
    xf, vf, _ = pm.run(x, v, a_list, n)
    xb, vb, _ = pm.run(xf, vf, a_list[::-1], n)
    assert pm.periodic_distance(xb, x).max() < 1e-12
    np.testing.assert_allclose(vb, v, atol=1e-12)


def _plane_wave(n, a0, a1, steps):
    """Zel'dovich plane wave x = q + a Psi0(q), Psi0 = -(1/k) sin(k q) x (shell crossing at a=1)."""
    k = 2 * np.pi
    c = (np.arange(n) + 0.5) / n
    q = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    psi0 = np.zeros_like(q)
    psi0[:, 0] = -np.sin(k * q[:, 0]) / k
    x = pm.wrap01(q + a0 * psi0)
    v = np.sqrt(a0) * a0 * psi0
    a_list = list(np.linspace(a0, a1, steps + 1))
    xf, _, _ = pm.run(x, v, a_list, n, solver="exact7", mas="tsc")
    exact = pm.wrap01(q + a1 * psi0)
    d = xf - exact
    d -= np.round(d)
    return np.abs(d[:, 0]).max() / (a1 / k), np.abs(d[:, 1:]).max()


def test_zeldovich_plane_wave_before_shell_crossing():
    e16, t16 = _plane_wave(16, 0.1, 0.5, 40)
    e32, t32 = _plane_wave(32, 0.1, 0.5, 40)
    assert t16 < 1e-12 and t32 < 1e-12          # transverse motion is exactly zero
    assert e32 < 1e-2                            # relative to the displacement amplitude
    assert 2.5 < e16 / e32 < 6.0, (e16, e32)     # second order in h


# ---------------------------------------------------------------- position forms

def test_cell_units_decodes_cell_offset_form():
    """The cell-offset form (Sect. 3.2 layout, row-major with k fastest): the linear
    index (i n + j) n + k built by hand from explicit, distinct (i, j, k) decodes to
    cell units (i, j, k) + offset, axis by axis (a swapped axis or a wrong stride fails)."""
    n = 7                                       # odd, so no axis mapping is symmetric
    ijk = np.array([[1, 4, 2], [6, 0, 3], [0, 0, 6], [5, 6, 0], [3, 2, 1]])
    off = np.array([[0.25, 0.5, 0.75], [0.0, 0.999, 0.125], [0.5, 0.5, 0.5],
                    [0.875, 0.0, 0.0625], [0.3, 0.6, 0.9]])
    lin = ijk[:, 0] * n * n + ijk[:, 1] * n + ijk[:, 2]
    np.testing.assert_array_equal(lin, [79, 297, 6, 287, 162])   # by hand
    got = pm.cell_units(n, cell=lin.astype(np.int32), off=off)
    np.testing.assert_array_equal(got, ijk + off)
    # box-unit branch: u = x n
    np.testing.assert_array_equal(pm.cell_units(n, pos=(ijk + off) / n), (ijk + off) / n * n)


@pytest.mark.parametrize("mas", ["tsc", "cic"])
def test_cell_offset_deposit_equals_brute_force(mas):
    """A deposit through the cell-offset decode equals the brute-force window sum over
    every (particle, cell) pair of the same points given in box units."""
    n = 6
    rng = RNG(23)
    ijk = rng.integers(0, n, size=(40, 3))
    off = rng.uniform(0, 1, size=(40, 3))
    ijk[0], off[0] = [5, 0, 2], [0.999, 0.0, 0.5]         # near the seam, on a face
    lin = (ijk[:, 0] * n + ijk[:, 1]) * n + ijk[:, 2]
    got = pm.deposit(pm.cell_units(n, cell=lin, off=off), n, mas, mass=1.0)
    x = (ijk + off) / n                                     # box units
    win = pm.w_tsc if mas == "tsc" else pm.w_cic
    c = np.arange(n) + 0.5
    ref = np.zeros((n, n, n))
    for p in range(x.shape[0]):
        s = [(x[p, d] * n - c + n / 2) % n - n / 2 for d in range(3)]
        ref += np.einsum("i,j,k->ijk", *[win(v) for v in s])
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


def test_wrap01_edges():
    """Periodic wrap into [0, 1): values that reduce to exactly 1.0 map to 0 (a position
    of 1.0 is the same point as 0.0), negatives wrap from the top, and interior values
    are unchanged."""
    x = np.array([1.0, 0.0, -0.0, -1e-17, -0.25, 1.5, 2.0, 0.999999, -1.0, 3.25])
    got = pm.wrap01(x)
    expect = np.array([0.0, 0.0, 0.0, 0.0, 0.75, 0.5, 0.0, 0.999999, 0.0, 0.25])
    np.testing.assert_array_equal(got, expect)
    assert np.all((got >= 0.0) & (got < 1.0))

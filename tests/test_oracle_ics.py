"""Pins of the FP64 initial-condition and power-spectrum oracle (oracle/ics.py) against
closed forms, the paper's own growth equations and brute force."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import ics

RNG = lambda s: np.random.Generator(np.random.PCG64(s))  # noqa: E731


def _grid(n):
    c = (np.arange(n) + 0.5) / n
    return np.meshgrid(c, c, c, indexing="ij")


def _spec(field):
    n = field.shape[0]
    sp = np.fft.rfftn(field)
    _, keep = ics._modes(n)
    return np.where(keep, sp, 0.0)


@pytest.mark.parametrize("dealias", [False, True])
def test_plane_wave_is_first_order_exact(dealias):
    """One plane wave: Psi(1) = -A k sin(k.q) / k^2 and every higher order vanishes
    (the Hessian of the potential has rank one, so the second and third invariants are
    zero: the Zel'dovich solution of a plane wave is exact before shell crossing)."""
    n, A = 16, 0.02
    x, y, z = _grid(n)
    m = np.array([2, -1, 3])
    k = 2 * np.pi * m
    theta = k[0] * x + k[1] * y + k[2] * z
    psi = ics.lpt_from_density(_spec(A * np.cos(theta)), n, order=3, dealias=dealias)
    k2 = float(k @ k)
    for d in range(3):
        np.testing.assert_allclose(psi["1"][..., d], -A * k[d] * np.sin(theta) / k2, atol=1e-15)
    for key in ("2", "3a", "3b", "3c"):
        assert np.abs(psi[key]).max() < 1e-16, key


def _orthogonal_waves(n, B):
    """phi(1) = sum_d B_d cos(k q_d) with k = 2 pi: delta = lap phi(1)."""
    x, y, z = _grid(n)
    k = 2 * np.pi
    c = [np.cos(k * v) for v in (x, y, z)]
    s = [np.sin(k * v) for v in (x, y, z)]
    delta = -k * k * sum(B[d] * c[d] for d in range(3))
    return k, c, s, delta


@pytest.mark.parametrize("dealias", [False, True])
def test_second_order_of_two_orthogonal_waves(dealias):
    """phi(1) = B1 cos(k x) + B2 cos(k y): the second-order source is phi_xx phi_yy =
    k^4 B1 B2 cos cos, a mode of |K|^2 = 2 k^2, so phi(2) = -(k^2/2) B1 B2 cos(kx) cos(ky)
    and Psi(2) = grad phi(2)."""
    n = 16
    B = (0.003, -0.002, 0.0)
    k, c, s, delta = _orthogonal_waves(n, B)
    psi = ics.lpt_from_density(_spec(delta), n, order=2, dealias=dealias)
    amp = 0.5 * k ** 3 * B[0] * B[1]
    np.testing.assert_allclose(psi["2"][..., 0], amp * s[0] * c[1], atol=1e-16)
    np.testing.assert_allclose(psi["2"][..., 1], amp * c[0] * s[1], atol=1e-16)
    assert np.abs(psi["2"][..., 2]).max() < 1e-18


def test_dealiasing_drops_the_sum_frequency():
    """Two waves m1 = (5, 1, 0), m2 = (5, -2, 0) on a 16^3 grid: their second-order source
    [k1^2 k2^2 - (k1.k2)^2] cos(t1) cos(t2) holds the difference mode (0, 3, 0) and the sum
    mode (10, -1, 0), beyond the grid's band. Products formed on the finer grid keep the
    difference only (phi(2) = -C cos(t1 - t2) / (2 |k1 - k2|^2)); on the n grid the sum
    mode would fold back to (-6, -1, 0)."""
    n = 16
    x, y, z = _grid(n)
    m1, m2 = np.array([5, 1, 0]), np.array([5, -2, 0])
    k1, k2 = 2 * np.pi * m1, 2 * np.pi * m2
    t1 = k1[0] * x + k1[1] * y + k1[2] * z
    t2 = k2[0] * x + k2[1] * y + k2[2] * z
    # phi(1) = cos t1 + cos t2 scaled: delta = -(k1^2 cos t1 + k2^2 cos t2) eps
    eps = 1e-3
    delta = -eps * (float(k1 @ k1) * np.cos(t1) + float(k2 @ k2) * np.cos(t2))
    C = eps * eps * (float(k1 @ k1) * float(k2 @ k2) - float(k1 @ k2) ** 2)
    kd = k1 - k2
    phi2 = -C * np.cos(t1 - t2) / (2 * float(kd @ kd))
    grad = [-C * (-kd[d]) * np.sin(t1 - t2) / (2 * float(kd @ kd)) for d in range(3)]
    psi = ics.lpt_from_density(_spec(delta), n, order=2, dealias=True)
    for d in range(3):
        np.testing.assert_allclose(psi["2"][..., d], grad[d], atol=1e-14 * np.abs(phi2).max() * 100)
    aliased = ics.lpt_from_density(_spec(delta), n, order=2, dealias=False)
    assert np.abs(aliased["2"] - psi["2"]).max() > 1e-3 * np.abs(psi["2"]).max()


def test_third_order_sources_of_three_orthogonal_waves():
    """phi(1) = sum_d B_d cos(k q_d): the third-order fields against their sources written
    out from analytic derivatives (phi(2) = -(k^2/2) sum_{d<e} B_d B_e c_d c_e), each
    inverted with numpy's FFT: Psi(3a) from det phi(1)_ij, Psi(3b) from the mixed
    invariant, Psi(3c) from the curl of A(3c), which is divergence-free."""
    n = 16
    B = (0.003, -0.002, 0.0025)
    k, c, s, delta = _orthogonal_waves(n, B)
    psi = ics.lpt_from_density(_spec(delta), n, order=3, dealias=True)
    k4 = k ** 4
    p1 = [-B[d] * k * k * c[d] for d in range(3)]                  # phi(1)_dd
    p2d = [0.5 * k4 * c[0] * (B[0] * B[1] * c[1] + B[0] * B[2] * c[2]),
           0.5 * k4 * c[1] * (B[0] * B[1] * c[0] + B[1] * B[2] * c[2]),
           0.5 * k4 * c[2] * (B[0] * B[2] * c[0] + B[1] * B[2] * c[1])]
    p2xy = -0.5 * k4 * B[0] * B[1] * s[0] * s[1]
    p2xz = -0.5 * k4 * B[0] * B[2] * s[0] * s[2]
    p2yz = -0.5 * k4 * B[1] * B[2] * s[1] * s[2]
    det = p1[0] * p1[1] * p1[2]
    s3b = 0.5 * (p1[0] * (p2d[1] + p2d[2]) + p1[1] * (p2d[0] + p2d[2]) + p1[2] * (p2d[0] + p2d[1]))
    rx = -p2yz * (p1[1] - p1[2])
    ry = -p2xz * (p1[2] - p1[0])
    rz = -p2xy * (p1[0] - p1[1])
    m = np.fft.fftfreq(n, 1.0 / n)
    K = [2 * np.pi * m.reshape([-1 if a == d else 1 for a in range(3)]) for d in range(3)]
    K2 = K[0] ** 2 + K[1] ** 2 + K[2] ** 2
    K2[0, 0, 0] = 1.0

    def grad_inv_lap(src):
        f = -np.fft.fftn(src) / K2
        f[0, 0, 0] = 0.0
        return [np.real(np.fft.ifftn(1j * K[d] * f)) for d in range(3)]

    def inv_lap(src):
        f = -np.fft.fftn(src) / K2
        f[0, 0, 0] = 0.0
        return f

    ref3a = grad_inv_lap(det)
    ref3b = grad_inv_lap(s3b)
    A = [inv_lap(r) for r in (rx, ry, rz)]
    ref3c = [np.real(np.fft.ifftn(1j * (K[1] * A[2] - K[2] * A[1]))),
             np.real(np.fft.ifftn(1j * (K[2] * A[0] - K[0] * A[2]))),
             np.real(np.fft.ifftn(1j * (K[0] * A[1] - K[1] * A[0])))]
    for d in range(3):
        np.testing.assert_allclose(psi["3a"][..., d], ref3a[d], atol=1e-12 * np.abs(ref3a[d]).max() + 1e-22)
        np.testing.assert_allclose(psi["3b"][..., d], ref3b[d], atol=1e-12 * np.abs(ref3b[d]).max() + 1e-22)
        np.testing.assert_allclose(psi["3c"][..., d], ref3c[d], atol=1e-12 * np.abs(ref3c[0]).max() + 1e-22)
    assert np.abs(psi["3a"]).max() > 0 and np.abs(psi["3b"]).max() > 0
    # Psi(3c) is a curl: divergence-free
    div = sum(np.real(np.fft.ifftn(1j * K[d] * np.fft.fftn(psi["3c"][..., d]))) for d in range(3))
    assert np.abs(div).max() < 1e-10 * np.abs(psi["3c"]).max() * k


def test_growth_factors_solve_the_papers_growth_equations():
    """The Einstein-de Sitter closed forms D2 = -3/7 D^2, D3a = -1/3 D^3, D3b = 10/21 D^3,
    D3c = -1/7 D^3 (App. A) against the paper's ODEs in ln a (beta = 3/2, gamma = 1/2 in
    EdS) integrated numerically from a growing-mode start."""
    beta, gamma = 1.5, 0.5

    def rhs(t, y):
        D, Dp, E, Ep, Fa, Fap, Fb, Fbp, Fc, Fcp = y
        return [Dp, -gamma * Dp + beta * D,
                Ep, -gamma * Ep + beta * (E - D * D),
                Fap, -gamma * Fap + beta * (Fa - 2 * D ** 3),
                Fbp, -gamma * Fbp + beta * (Fb - 2 * D * (E - D * D)),
                Fcp, (1 - gamma) * Fcp + E * Dp - D * Ep - beta * D ** 3]

    a0 = 1e-3
    c = ics.LPT_GROWTH
    y0 = [a0, a0, c["2"] * a0 ** 2, 2 * c["2"] * a0 ** 2, c["3a"] * a0 ** 3, 3 * c["3a"] * a0 ** 3,
          c["3b"] * a0 ** 3, 3 * c["3b"] * a0 ** 3, c["3c"] * a0 ** 3, 3 * c["3c"] * a0 ** 3]
    sol = solve_ivp(rhs, (np.log(a0), 0.0), y0, rtol=1e-11, atol=1e-20)
    D, _, E, _, Fa, _, Fb, _, Fc, _ = sol.y[:, -1]
    assert D == pytest.approx(1.0, rel=1e-8)
    assert E == pytest.approx(-3.0 / 7.0, rel=1e-8)
    assert Fa == pytest.approx(-1.0 / 3.0, rel=1e-8)
    assert Fb == pytest.approx(10.0 / 21.0, rel=1e-8)
    assert Fc == pytest.approx(-1.0 / 7.0, rel=1e-8)


def test_lpt_state_first_order_matches_zeldovich_and_velocity_factors():
    """1LPT positions and velocities: x = q + a Psi(1), v = a^(1/2) a Psi(1) (EdS growing
    mode), and at second order the velocity weights the order-2 term twice."""
    n, a = 16, 0.1
    noise = RNG(3).standard_normal((n, n, n))
    k_tab, p_tab = ics.power_law_table(1e-4, -1.5)
    psi = ics.lpt_displacements(noise, k_tab, p_tab, order=2, dealias=False)
    x1, v1 = ics.lpt_state(noise, k_tab, p_tab, a, order=1, dealias=False)
    x2, v2 = ics.lpt_state(noise, k_tab, p_tab, a, order=2, dealias=False)
    q = np.stack(_grid(n), -1).reshape(-1, 3)
    d = x1 - q
    d -= np.round(d)
    np.testing.assert_allclose(d, a * psi["1"].reshape(-1, 3), atol=1e-15)
    np.testing.assert_allclose(v1, np.sqrt(a) * a * psi["1"].reshape(-1, 3), atol=1e-16)
    np.testing.assert_allclose(v2 - v1, np.sqrt(a) * 2 * (-3 / 7) * a * a * psi["2"].reshape(-1, 3),
                               atol=1e-16)


def test_linear_density_follows_the_table():
    """sqrt(N) sqrt(P) DFT[w]: for white noise the shell-averaged power of the density
    equals the table within the sampling scatter, and the power-law table interpolates
    exactly in log-log."""
    k_tab, p_tab = ics.power_law_table(2.0e-3, -2.0)
    kk = np.array([7.0, 33.3, 210.0])
    np.testing.assert_allclose(ics.interp_pk(kk, k_tab, p_tab), 2.0e-3 * kk ** -2.0, rtol=1e-12)
    n = 32
    dk = ics.linear_density_spectrum(RNG(9).standard_normal((n, n, n)), k_tab, p_tab)
    delta = np.fft.irfftn(dk, s=(n, n, n))
    pk, kb, cnt = ics.power_spectrum(1.0 + delta, deconv=0)
    sel = (cnt > 200) & (np.arange(1, len(pk) + 1) < n // 2 - 1)
    ratio = pk[sel] / ics.interp_pk(kb[sel], k_tab, p_tab)
    assert np.all(np.abs(ratio - 1.0) < 5.0 / np.sqrt(cnt[sel] / 2.0))


def test_power_spectrum_of_one_mode_and_mode_counts():
    """A single mode delta = A cos(2 pi m.x): P in its shell is (A^2 / 2) over the shell's
    mode count, which is checked by brute force over the full cube of wavevectors; every
    other shell is empty of power."""
    n, A = 16, 0.3
    x, y, z = _grid(n)
    m = np.array([3, -4, 1])
    rho = 1.0 + A * np.cos(2 * np.pi * (m[0] * x + m[1] * y + m[2] * z))
    pk, kb, cnt = ics.power_spectrum(rho, deconv=0, nbins=12)
    r = np.arange(n) - n // 2
    mm = np.sqrt(r[:, None, None] ** 2 + r[None, :, None] ** 2 + r[None, None, :] ** 2)
    brute = np.array([np.sum(np.rint(mm) == b) for b in range(1, 13)])
    np.testing.assert_array_equal(cnt, brute)
    b = int(np.rint(np.sqrt(m @ m)))
    assert pk[b - 1] == pytest.approx(A * A / 2 / brute[b - 1], rel=1e-12)
    others = np.delete(pk, b - 1)
    assert np.abs(others).max() < 1e-30
    assert kb[b - 1] == pytest.approx(np.mean(2 * np.pi * mm[np.rint(mm) == b]), rel=1e-12)


@pytest.mark.parametrize("dealias", [False, True])
def test_lpt_sources_equal_matrix_invariants(dealias):
    """On a generic random field (every off-diagonal second derivative non-zero), the
    oracle's expanded component formulas of the paper against their compact matrix forms
    evaluated with numpy linear algebra on the Hessians H1 = phi(1)_ij, H2 = phi(2)_ij at
    every point: lap phi(2) = [(tr H1)^2 - tr(H1 H1)] / 2, det H1, lap phi(3b) =
    [tr H2 tr H1 - tr(H2 H1)] / 2, and lap A(3c) = sum_i grad phi(2)_,i x grad phi(1)_,i
    (columns of H2 crossed with columns of H1)."""
    n = 16
    k_tab, p_tab = ics.power_law_table(1e-3, -1.0)
    dk = ics.linear_density_spectrum(RNG(21).standard_normal((n, n, n)), k_tab, p_tab)
    _, _, _, f = ics.lpt_sources(dk, n, order=3, dealias=dealias)

    def hessian(d):
        h = np.empty(d[(0, 0)].shape + (3, 3))
        for i in range(3):
            for j in range(3):
                h[..., i, j] = d[(min(i, j), max(i, j))]
        return h

    H1, H2 = hessian(f["d1"]), hessian(f["d2"])
    tr1, tr2 = np.trace(H1, axis1=-2, axis2=-1), np.trace(H2, axis1=-2, axis2=-1)
    scale1 = np.abs(H1).max()
    np.testing.assert_allclose(f["s2"], 0.5 * (tr1 ** 2 - np.trace(H1 @ H1, axis1=-2, axis2=-1)),
                               atol=1e-12 * scale1 ** 2)
    np.testing.assert_allclose(f["det"], np.linalg.det(H1), atol=1e-12 * scale1 ** 3)
    scale2 = np.abs(H2).max() * scale1
    np.testing.assert_allclose(f["s3b"], 0.5 * (tr2 * tr1 - np.trace(H2 @ H1, axis1=-2, axis2=-1)),
                               atol=1e-12 * scale2)
    cross = sum(np.cross(H2[..., :, i], H1[..., :, i]) for i in range(3))
    for c, key in enumerate(("rx", "ry", "rz")):
        np.testing.assert_allclose(f[key], cross[..., c], atol=1e-12 * scale2)
    assert np.abs(cross).max() > 1e-3 * scale2

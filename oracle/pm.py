"""FP64 reference of the particle-mesh loop (deposit, solve, gradient, interp, KDK).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (readings of the paper that it leaves implicit):
  * Unit periodic box, n cells per side, h = 1/n. Cell c = (i, j, k) has its
    centre at (c + 1/2) h; particles start at cell centres (paper App. B.2).
  * Grids are [n, n, n] row-major, vector grids [n, n, n, 3], particles
    [np, 3] (paper Sect. 3.2).
  * Positions are handled in cell units u = x / h.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

# --------------------------------------------------------------------------
# mass-assignment weights (paper Sect. 3.5, the NGP/CIC/TSC window functions)
# --------------------------------------------------------------------------

MAS_ORDER = {"ngp": 1, "cic": 2, "tsc": 3}


def w_ngp(s):
    """NGP window of the normalised separation s (paper Sect. 3.5): 1 inside the cell.
    The boundary |s| = 1/2 belongs to the cell whose lower face it is (the particle's
    cell is floor(u)), i.e. s in [-1/2, 1/2)."""
    s = np.asarray(s, dtype=np.float64)
    return np.where((s >= -0.5) & (s < 0.5), 1.0, 0.0)


def w_tsc(s):
    """TSC window of the normalised separation s (paper Sect. 3.5)."""
    s = np.abs(np.asarray(s, dtype=np.float64))
    return np.where(s < 0.5, 0.75 - s * s, np.where(s < 1.5, 0.5 * (1.5 - s) ** 2, 0.0))


def w_cic(s):
    """CIC window of the normalised separation s (paper Sect. 3.5)."""
    s = np.abs(np.asarray(s, dtype=np.float64))
    return np.where(s < 1.0, 1.0 - s, 0.0)


def axis_support(u, mas):
    """Cells touched along one axis and their weights.

    u: positions in cell units (float64 array). Returns (first_index, weights)
    where weights has shape [support, ...]. The support is the set of cells
    whose window value can be non-zero; the weights are the window evaluated
    at the separation between u and each cell centre (c + 1/2).
    TSC: 3 cells starting at floor(u) - 1; CIC: 2 cells starting at floor(u - 1/2);
    NGP: the cell floor(u).
    """
    u = np.asarray(u, dtype=np.float64)
    if mas == "ngp":
        first = np.floor(u)
        return first.astype(np.int64), w_ngp(u[None] - (first[None] + 0.5))
    if mas == "tsc":
        first = np.floor(u) - 1.0
        cells = first[None] + np.arange(3.0).reshape((3,) + (1,) * u.ndim)
        return first.astype(np.int64), w_tsc(u[None] - (cells + 0.5))
    if mas == "cic":
        first = np.floor(u - 0.5)
        cells = first[None] + np.arange(2.0).reshape((2,) + (1,) * u.ndim)
        return first.astype(np.int64), w_cic(u[None] - (cells + 0.5))
    raise ValueError(mas)


def _stencil_entries(u, n, mas):
    """Yield (flat cell index [np], weight [np]) over the support of every particle."""
    firsts, ws = [], []
    for d in range(3):
        f, w = axis_support(u[:, d], mas)
        firsts.append(f)
        ws.append(w)
    s = ws[0].shape[0]
    for a in range(s):
        ia = (firsts[0] + a) % n
        for b in range(s):
            ib = (firsts[1] + b) % n
            for c in range(s):
                ic = (firsts[2] + c) % n
                yield (ia * n + ib) * n + ic, ws[0][a] * ws[1][b] * ws[2][c]


def cell_units(n, pos=None, cell=None, off=None):
    """Positions in cell units [np, 3] (float64), from box units or cell + offset."""
    if pos is not None:
        return np.asarray(pos, dtype=np.float64) * n
    c = np.asarray(cell, dtype=np.int64)
    ci = np.stack([c // (n * n), (c // n) % n, c % n], axis=-1).astype(np.float64)
    return ci + np.asarray(off, dtype=np.float64)


def deposit(u, n, mas="tsc", mass=None):
    """Density rho~_c = w sum_p W(u_p - (c + 1/2)) (paper Sect. 3.5).

    The particle weight w defaults to n^3 / np, so that the mean density is 1
    (the paper normalises the sum to the particle count, which equals n^3 when
    there is one particle per cell).
    """
    u = np.asarray(u, dtype=np.float64)
    npart = u.shape[0]
    if mass is None:
        mass = (n ** 3) / max(npart, 1)
    rho = np.zeros(n ** 3, dtype=np.float64)
    if npart == 0:
        return rho.reshape(n, n, n)
    for flat, w in _stencil_entries(u, n, mas):
        rho += np.bincount(flat, weights=w, minlength=n ** 3)
    return (mass * rho).reshape(n, n, n)


def deposit_charges(u, n, q, mas="tsc"):
    """Deposit arbitrary per-particle charges q [np] (no normalisation)."""
    u = np.asarray(u, dtype=np.float64)
    rho = np.zeros(n ** 3, dtype=np.float64)
    for flat, w in _stencil_entries(u, n, mas):
        rho += np.bincount(flat, weights=w * q, minlength=n ** 3)
    return rho.reshape(n, n, n)


def interp(u, grid, mas="tsc"):
    """a_p = sum_c W(u_p - (c + 1/2)) g_c with the deposit's window (paper Sect. 3.5).

    grid: [n, n, n] or [n, n, n, k]; returns [np] or [np, k].
    """
    u = np.asarray(u, dtype=np.float64)
    n = grid.shape[0]
    flat_grid = grid.reshape(n ** 3, -1)
    out = np.zeros((u.shape[0], flat_grid.shape[1]), dtype=np.float64)
    for flat, w in _stencil_entries(u, n, mas):
        out += w[:, None] * flat_grid[flat]
    return out if grid.ndim == 4 else out[:, 0]


# --------------------------------------------------------------------------
# Poisson problem
# --------------------------------------------------------------------------

def source(rho, a, omega_m=1.0):
    """f = (3/2) a Omega_m (rho~ - mean rho~) (paper Sect. 3.1, supercomoving Poisson).

    The computed mean is subtracted so that the periodic problem is solvable.
    """
    rho = np.asarray(rho, dtype=np.float64)
    return 1.5 * a * omega_m * (rho - rho.mean())


def laplacian7(u, h):
    """Seven-point Laplacian (L(u) - 6 u) / h^2 on the periodic grid (paper Sect. 3.5)."""
    s = np.zeros_like(u)
    for ax in range(3):
        s += np.roll(u, 1, axis=ax) + np.roll(u, -1, axis=ax)
    return (s - 6.0 * u) / (h * h)


def _mode_numbers(n):
    m = np.fft.fftfreq(n, d=1.0 / n)
    mh = np.arange(n // 2 + 1, dtype=np.float64)
    return m[:, None, None], m[None, :, None], mh[None, None, :]


def solve_exact7(f, h, workers=1):
    """Zero-mean solution of the periodic seven-point system laplacian7(phi) = f.

    The discrete operator is diagonal in the Fourier basis with eigenvalue
    lambda(m) = -(4 / h^2) sum_d sin^2(pi m_d / n); the mean of f is removed
    and the mean of phi is fixed to zero. Multigrid converges to this result.
    """
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    mx, my, mz = _mode_numbers(n)
    lam = -(4.0 / (h * h)) * (np.sin(np.pi * mx / n) ** 2 + np.sin(np.pi * my / n) ** 2
                              + np.sin(np.pi * mz / n) ** 2)
    fk = sfft.rfftn(f, workers=workers)
    lam[0, 0, 0] = 1.0
    phik = fk / lam
    phik[0, 0, 0] = 0.0
    return sfft.irfftn(phik, s=f.shape, workers=workers)


def solve_fft(f, h, p=3):
    """FFT solver with mass-assignment deconvolution (paper Sect. 3.8, 'FFT').

    phi(k) = -f(k) / (k^2 W(k)^2), W(k) = [prod_d sinc(omega_d / 2)]^p,
    omega_d = k_d h in [-pi, pi], k = 2 pi m in the unit box, sinc x = sin x / x.
    p = 3 for TSC, 2 for CIC, 0 for no deconvolution. phi(0) = 0.
    """
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    mx, my, mz = _mode_numbers(n)
    kx, ky, kz = 2 * np.pi * mx, 2 * np.pi * my, 2 * np.pi * mz
    k2 = kx * kx + ky * ky + kz * kz

    def sinc_half(k):
        w = 0.5 * k * h
        return np.where(w == 0.0, 1.0, np.sin(w) / np.where(w == 0.0, 1.0, w))

    wmas = (sinc_half(kx) * sinc_half(ky) * sinc_half(kz)) ** p
    k2[0, 0, 0] = 1.0
    green = -1.0 / (k2 * wmas * wmas)
    green[0, 0, 0] = 0.0
    return sfft.irfftn(sfft.rfftn(f) * green, s=f.shape)


def solve_fft_7pt(f, h):
    """FFT_7pt solver (paper Sect. 3.8): the Fourier-space form of the seven-point
    Laplacian, phi(k) = -f(k) / sum_d (omega_d/h sinc(omega_d/2))^2 with omega_d = k_d h,
    no mass-assignment compensation; phi(0) = 0. (The paper prints the factor as
    h omega_d; the stencil it names has eigenvalue (omega_d / h)^2 sinc^2(omega_d/2)
    = (4/h^2) sin^2(omega_d/2) per axis, which is what is used.)"""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    mx, my, mz = _mode_numbers(n)
    lam = np.zeros((n, n, n // 2 + 1))
    for m in (mx, my, mz):
        om = 2 * np.pi * m * h                                     # omega = k h
        sinc = np.where(om == 0.0, 1.0, np.sin(om / 2) / np.where(om == 0.0, 1.0, om / 2))
        lam = lam + (om / h * sinc) ** 2
    lam[0, 0, 0] = 1.0
    phik = -sfft.rfftn(f) / lam
    phik[0, 0, 0] = 0.0
    return sfft.irfftn(phik, s=f.shape)


def force_full_fft(f, h, p=3):
    """FULL_FFT (paper Sect. 3.8, Eq. exact_fullfft_kernel): the force g = -grad phi
    taken directly in Fourier space, g_d(k) = i k_d f(k) / (k^2 W(k)^2) (the derivative
    of phi(k) = -f(k) / (k^2 W^2) is i k_d phi(k), numpy's transform convention), with
    W the deconvolution window of solve_fft. On the Nyquist plane of axis d
    (m_d = -n/2) the derivative multiplier k_d is taken as 0: the mode is its own
    conjugate, so an odd multiplier has no real-valued image there. Returns [n,n,n,3]."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    mx, my, mz = _mode_numbers(n)
    kx, ky, kz = 2 * np.pi * mx, 2 * np.pi * my, 2 * np.pi * mz
    k2 = kx * kx + ky * ky + kz * kz

    def sinc_half(k):
        w = 0.5 * k * h
        return np.where(w == 0.0, 1.0, np.sin(w) / np.where(w == 0.0, 1.0, w))

    wmas = (sinc_half(kx) * sinc_half(ky) * sinc_half(kz)) ** p
    k2[0, 0, 0] = 1.0
    base = sfft.rfftn(f) / (k2 * wmas * wmas)
    base[0, 0, 0] = 0.0
    out = np.empty(f.shape + (3,))
    for d, (kd, md) in enumerate(((kx, mx), (ky, my), (kz, mz))):
        mult = np.where(md == -n // 2, 0.0, kd) if d < 2 else np.where(md == n // 2, 0.0, kd)
        out[..., d] = sfft.irfftn(1j * mult * base, s=f.shape)
    return out


GRAD_COEFFS = {
    # central-derivative stencils of the paper's gradient table: offsets 1, 2, 3
    3: (0.5, 0.0, 0.0),
    5: (2.0 / 3.0, -1.0 / 12.0, 0.0),
    7: (0.75, -3.0 / 20.0, 1.0 / 60.0),
}


def derivative(u, h, axis, points=5):
    """D_axis u = (1/h) sum_n c_n u_{i+n} with the paper's central coefficients."""
    c = GRAD_COEFFS[points]
    out = np.zeros_like(u, dtype=np.float64)
    for off, cn in enumerate(c, start=1):
        if cn != 0.0:
            out += cn * (np.roll(u, -off, axis=axis) - np.roll(u, off, axis=axis))
    return out / h


def gradient(phi, h, points=5):
    """Acceleration grid g = -grad(phi), shape [n, n, n, 3] (paper gradient table)."""
    phi = np.asarray(phi, dtype=np.float64)
    return np.stack([-derivative(phi, h, ax, points) for ax in range(3)], axis=-1)


# --------------------------------------------------------------------------
# force chain and integrator
# --------------------------------------------------------------------------

def accel(u, n, a, solver="exact7", mas="tsc", omega_m=1.0, mass=None, points=5,
          return_fields=False):
    """Particle accelerations at scale factor a: deposit -> source -> solve -> gradient -> interp.

    solver: "exact7" (the seven-point system, which multigrid solves),
            "fft" (mass-assignment-deconvolved FFT kernel), "fft_7pt" (the seven-point
            Laplacian in Fourier space) or "full_fft" (the force in Fourier space, no
            finite-difference gradient; the returned potential is then None).
    """
    h = 1.0 / n
    rho = deposit(u, n, mas, mass)
    f = source(rho, a, omega_m)
    if solver == "full_fft":
        phi = None
        g = force_full_fft(f, h, MAS_ORDER[mas])
    else:
        if solver == "exact7":
            phi = solve_exact7(f, h)
        elif solver == "fft":
            phi = solve_fft(f, h, MAS_ORDER[mas])
        elif solver == "fft_7pt":
            phi = solve_fft_7pt(f, h)
        else:
            raise ValueError(solver)
        g = gradient(phi, h, points)
    acc = interp(u, g, mas)
    if return_fields:
        return acc, dict(rho=rho, f=f, phi=phi, g=g)
    return acc


def tau_eds(a0, a1):
    """Supercomoving time between a0 and a1 in Einstein-de Sitter.

    dt~ = H0 dt / a^2 (paper Sect. 3.1) and H = H0 a^{-3/2} give
    da/dt~ = a^{3/2}, so tau = 2 (a0^{-1/2} - a1^{-1/2}).
    """
    return 2.0 * (a0 ** -0.5 - a1 ** -0.5)


def wrap01(x):
    x = np.mod(np.asarray(x, dtype=np.float64), 1.0)
    x[x >= 1.0] = 0.0
    return x


def kdk_step(x, v, acc0, a0, a1, n, **force_kw):
    """One kick-drift-kick step (paper Sect. 3.4) in supercomoving time.

    x, v: box units [np, 3] (float64); acc0 = a(x, a0). Returns (x1, v1, acc1).
    """
    tau = tau_eds(a0, a1)
    vh = v + 0.5 * tau * acc0
    x1 = wrap01(x + tau * vh)
    acc1 = accel(x1 * n, n, a1, **force_kw)
    v1 = vh + 0.5 * tau * acc1
    return x1, v1, acc1


def run(x, v, a_list, n, **force_kw):
    """Integrate through the scale factors a_list[0] -> a_list[-1]; returns (x, v, acc)."""
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    acc = accel(x * n, n, a_list[0], **force_kw)
    for a0, a1 in zip(a_list[:-1], a_list[1:]):
        x, v, acc = kdk_step(x, v, acc, a0, a1, n, **force_kw)
    return x, v, acc


def periodic_distance(x, y):
    """Minimum-image distance per particle between two position arrays (box units)."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    d -= np.round(d)
    return np.sqrt(np.sum(d * d, axis=-1))

"""FP64 reference of the background expansion, parametrised gravity and QUMOND.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Background (paper Sect. 3.1 units): supercomoving time dt~ = H0 dt / a^2, so with
H(a)^2 / H0^2 = Omega_m a^-3 + Omega_k a^-2 + Omega_L (Omega_k = 1 - Omega_m - Omega_L)
the scale factor advances as da/dt~ = a^3 H / H0 = sqrt(Omega_m a^3 + Omega_k a^4 +
Omega_L a^6), and the time step between a0 and a1 is the integral of its inverse. The
supercomoving Poisson equation is lap phi~ = (3/2) Omega_m a mu(a) (rho~ - 1).

Parametrised gravity (Sect. 2.4, Eq. mu_parametrized_gravity):
mu(a) = 1 + mu0 Omega_L(a) / Omega_L0, with Omega_L(a) / Omega_L0 = H0^2 / H(a)^2.

QUMOND (Sect. 2.3, Eqs. QUMOND_Poisson_Newton and QUMOND_Poisson_MOND; discretised as in
Sect. 3.10, Eq. QUMOND_Poisson_MOND_discrete): the Newtonian potential phi_N solves the
seven-point system with the usual source; the MOND potential solves the seven-point
system with the source (1/h) sum_i [nu_B g_{B,i} - nu_A g_{A,i}], where B and A are the
faces at +-h/2 along axis i, g_{F,i} the two-point normal difference of phi_N across
the face, the two transverse components the four-point averages of the paper, and
nu = nu(|g_F| / g0) with g0 -> a^N g0.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import quad

from . import pm


def hubble2(a, omega_m, omega_l):
    """H(a)^2 / H0^2 for matter, curvature and a cosmological constant."""
    omega_k = 1.0 - omega_m - omega_l
    return omega_m * a ** -3 + omega_k * a ** -2 + omega_l


def dadt(a, omega_m, omega_l):
    """da / dt~ in supercomoving time."""
    return a ** 3 * np.sqrt(hubble2(a, omega_m, omega_l))


def tau(a0, a1, omega_m=1.0, omega_l=0.0):
    """Supercomoving time from a0 to a1 (numerical quadrature)."""
    val, _ = quad(lambda a: 1.0 / dadt(a, omega_m, omega_l), a0, a1, epsabs=0.0, epsrel=1e-13,
                  limit=200)
    return val


def mu_of_a(a, mu0, omega_m, omega_l):
    """mu(a) = 1 + mu0 Omega_L(a) / Omega_L0 = 1 + mu0 H0^2 / H(a)^2 (Omega_L0 > 0)."""
    if mu0 != 0.0 and omega_l <= 0.0:
        raise ValueError("mu(a) needs a cosmological constant")
    return 1.0 + mu0 / hubble2(a, omega_m, omega_l)


# --------------------------------------------------------------------------- MOND

def nu_function(y, family="simple", param=1.0):
    """The QUMOND interpolating functions nu(y) of Sect. 2.3."""
    y = np.asarray(y, dtype=np.float64)
    if family == "simple":
        return 0.5 + 0.5 * np.sqrt(1.0 + 4.0 / y)
    if family == "n":
        return (0.5 + 0.5 * np.sqrt(1.0 + 4.0 / y ** param)) ** (1.0 / param)
    if family == "beta":
        return (1.0 - np.exp(-y)) ** -0.5 + param * np.exp(-y)
    if family == "gamma":
        e = np.exp(-y ** (param / 2.0))
        return (1.0 - e) ** (-1.0 / param) + (1.0 - 1.0 / param) * e
    if family == "delta":
        return (1.0 - np.exp(-y ** (param / 2.0))) ** (-1.0 / param)
    raise ValueError(family)


def qumond_source(phin, h, g0, family="simple", param=1.0):
    """The MOND source (1/h) sum_i [nu_B g_{B,i} - nu_A g_{A,i}] of Eq.
    QUMOND_Poisson_MOND_discrete, from the Newtonian potential on the periodic grid."""
    phin = np.asarray(phin, dtype=np.float64)
    out = np.zeros_like(phin)
    for i in range(3):
        t1, t2 = [d for d in range(3) if d != i]
        up = np.roll(phin, -1, axis=i)                      # phi at +e_i
        gi = (up - phin) / h                                 # normal: across the face B_i
        # transverse components at B_i: the centred differences of both cells averaged
        gt = []
        for t in (t1, t2):
            dc = np.roll(phin, -1, axis=t) - np.roll(phin, 1, axis=t)
            du = np.roll(up, -1, axis=t) - np.roll(up, 1, axis=t)
            gt.append((du + dc) / (4.0 * h))
        mag = np.sqrt(gi * gi + gt[0] ** 2 + gt[1] ** 2)
        # nu_B g_{B,i} at face B_i; nu g -> 0 where the gradient vanishes (nu grows at
        # most as y^-1/2 for small y)
        safe = np.where(mag > 0.0, mag, 1.0)
        flux = np.where(mag > 0.0, nu_function(safe / g0, family, param) * gi, 0.0)
        out += (flux - np.roll(flux, 1, axis=i)) / h         # minus the face A_i = B_i of i-1
    return out


def qumond_accel(u, n, a, g0, g0_exponent=0.0, family="simple", param=1.0, mas="tsc",
                 omega_m=1.0, points=5, return_fields=False):
    """Particle accelerations in QUMOND: the Newtonian solve, the MOND source with
    g0 a^N, the second seven-point solve, the gradient and the interpolation."""
    h = 1.0 / n
    rho = pm.deposit(u, n, mas)
    f = pm.source(rho, a, omega_m)
    phin = pm.solve_exact7(f, h)
    s = qumond_source(phin, h, g0 * a ** g0_exponent, family, param)
    phi = pm.solve_exact7(s, h)
    acc = pm.interp(u, pm.gradient(phi, h, points), mas)
    if return_fields:
        return acc, dict(phin=phin, src=s, phi=phi)
    return acc


# --------------------------------------------------------------------------- runs

def accel(u, n, a, omega_m=1.0, omega_l=0.0, mu0=0.0, mas="tsc", solver="exact7"):
    """Accelerations with the parametrised coupling: the Newtonian chain with the source
    coefficient (3/2) Omega_m a mu(a)."""
    mu = mu_of_a(a, mu0, omega_m, omega_l)
    return pm.accel(u, n, a, solver, mas, omega_m * mu)


def run(x, v, a_list, n, omega_m=1.0, omega_l=0.0, mu0=0.0, g0=None, g0_exponent=0.0,
        family="simple", param=1.0, mas="tsc"):
    """Kick-drift-kick steps (Sect. 3.4) with the background's supercomoving time steps,
    parametrised gravity (mu0) or QUMOND (g0 given). Returns (x, v, acc)."""
    def force(xx, a):
        if g0 is not None:
            return qumond_accel(xx * n, n, a, g0, g0_exponent, family, param, mas, omega_m)
        return accel(xx * n, n, a, omega_m, omega_l, mu0, mas)
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    acc = force(x, a_list[0])
    for a0, a1 in zip(a_list[:-1], a_list[1:]):
        t = tau(a0, a1, omega_m, omega_l)
        v = v + 0.5 * t * acc
        x = pm.wrap01(x + t * v)
        acc = force(x, a1)
        v = v + 0.5 * t * acc
    return x, v, acc

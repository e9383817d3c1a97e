"""FP64 reference of f(R) gravity (Hu-Sawicki) with the non-linear multigrid.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model (paper Sect. 2.5): f_R = df/dR, with the background curvature
R_bar(a) = 3 m^2 (a^-3 + 4 Omega_L / Omega_m) and the background scalaron
f_R_bar(a) = (R_bar(1) / R_bar(a))^(n+1) f_R0.

Units. Lengths in box units (the grid spacing is h = 1/n), time in the supercomoving
time of the Poisson solver. Curvatures are in units of H0^2 / c^2, so m^2 = Omega_m and
R_bar = 3 (Omega_m a^-3 + 4 Omega_L). The scalaron in simulation units is
f~ = a^2 f_R and the speed of light c~ = c / (H0 L_box) (2997.92458 / L_box for a box
in Mpc/h): with these, the comoving f(R) field equations of Sect. 2.5 become the
supercomoving pair of Sect. 3.11 (Eqs. fr_sim_1, fr_sim_2):
    lap phi~ = (3/2) Omega_m a (rho~ - 1) - (c~^2 / 2) lap f~,
    lap f~   = -(Omega_m a / c~^2) (rho~ - 1) + (a^4 R_bar / (3 c~^2)) [(f~_bar / f~)^(1/(n+1)) - 1],
with f~_bar = a^2 f_R_bar. rho~ - 1 is taken as rho~ minus its measured mean.

Discretisation (Sect. 3.11). With u = (f~ / f~_bar)^(1/(n+1)) (u = 1 in the background)
and the seven-point Laplacian, the field equation at a cell reads
    N_h(u) = (f~_bar / h^2) [sum_nb u_nb^(n+1) - 6 u^(n+1)] - K / u = s,
    K = a^4 R_bar / (3 c~^2),  s = -(Omega_m a / c~^2)(rho~ - 1) - K.
For the cell value u given its six neighbours this is the depressed polynomial
u^(n+2) + p u + q = 0 (a cubic for n = 1, a quartic for n = 2) with
    p = -(1/6) sum_nb u_nb^(n+1) + h^2 s / (6 f~_bar),   q = h^2 K / (6 f~_bar) < 0,
which on the finest level is the p, q pair the paper prints. (The paper labels the
polynomial u^(n+1) + p u + q; its own cubic for n = 1 and quartic for n = 2 fix the
degree at n + 2.) The closed-form roots are those of Sect. 3.11, computed in FP64.

Non-linear multigrid (Sect. 3.7.2, full approximation storage): red-black non-linear
Gauss-Seidel (each cell set to the root of its polynomial), residual d = s - N_h(u),
coarse problem N_H(u_H) = N_H(R u) + R d from u_H = R u, correction
u += P(u_H - R u). R is the full weighting and P the trilinear prolongation of the linear
multigrid (oracle/mg.py); cycles V, F and W recurse as there. The coarsest grid gets a
fixed number of sweeps. The force is F = F_Newton + (c~^2 / 2) grad f~, i.e. the
gradient of phi_N - (c~^2 / 2) f~ with the usual stencil.
"""
from __future__ import annotations

import numpy as np

from . import mg as omg
from . import pm

C_KM_S = 299792.458


def c_tilde(box_mpc_h):
    """Speed of light in simulation units for a box of box_mpc_h Mpc/h."""
    return C_KM_S / (100.0 * box_mpc_h)


def r_bar(a, omega_m, omega_l):
    """Background curvature in units of H0^2 / c^2 (m^2 = Omega_m)."""
    return 3.0 * (omega_m * a ** -3 + 4.0 * omega_l)


def fr_bar(a, f_r0, n_exp, omega_m, omega_l):
    """Background scalaron f_R_bar(a) (Sect. 2.5)."""
    return (r_bar(1.0, omega_m, omega_l) / r_bar(a, omega_m, omega_l)) ** (n_exp + 1) * f_r0


class Coeffs:
    """The per-step constants of the discrete field equation."""

    def __init__(self, a, f_r0, n_exp, c2, omega_m=0.3, omega_l=0.7):
        if n_exp not in (1, 2):
            raise ValueError("Hu-Sawicki n must be 1 or 2")
        self.a, self.n_exp, self.c2 = a, n_exp, c2
        self.fbar = a * a * fr_bar(a, f_r0, n_exp, omega_m, omega_l)   # f~_bar
        self.K = a ** 4 * r_bar(a, omega_m, omega_l) / (3.0 * c2)
        self.cA = omega_m * a / c2

    def source(self, rho):
        rho = np.asarray(rho, dtype=np.float64)
        return -self.cA * (rho - rho.mean()) - self.K


# --------------------------------------------------------------------------- roots

def _stable_root_difference(d0, d1):
    """For Delta0 < 0: with B = (-Delta0)^(3/2), sqrt(disc) = sqrt(Delta1^2 + 4 B^2) and
    A = (|Delta1| + sqrt(disc)) / 2, returns (A^(1/3), A^(2/3) - (-Delta0)). The difference
    is formed as (A - B)(A + B) / (A^(4/3) + A^(2/3) B^(2/3) + B^(4/3)) with
    A - B = |Delta1| / 2 + Delta1^2 / (2 (sqrt(disc) + 2 B)): the same number, without the
    cancellation of subtracting two nearly equal terms."""
    B = (-d0) ** 1.5
    sq = np.sqrt(d1 * d1 + 4.0 * B * B)
    ad1 = np.abs(d1)
    A = 0.5 * (ad1 + sq)
    Q = np.cbrt(A)
    a_minus_b = 0.5 * ad1 + 0.5 * d1 * d1 / (sq + 2.0 * B)
    return Q, a_minus_b * (A + B) / (Q ** 4 - d0 * Q * Q + d0 * d0)


def root_cubic(p, q):
    """Root of u^3 + p u + q = 0 by the closed forms of Sect. 3.11 (q < 0: the largest
    real root, which is positive). Where one real root exists, the cube root C is taken
    from (Delta1 - sqrt(disc)) / 2 (Delta1 < 0): the paper's (Delta1 + sqrt(disc)) / 2
    gives Delta0 / C in place of C and so the same root. For p > 0 the root
    -(C + Delta0 / C) / 3 = (|C|^2 + Delta0) / (3 |C|) is evaluated without cancellation
    (_stable_root_difference); the printed form loses digits when the root is small."""
    p = np.asarray(p, dtype=np.float64)
    q = np.broadcast_to(np.asarray(q, dtype=np.float64), p.shape)
    d0 = -3.0 * p
    d1 = 27.0 * q
    disc = d1 * d1 - 4.0 * d0 ** 3
    out = np.empty_like(p)
    zero = p == 0.0
    pos = p > 0.0
    one = (~zero) & (~pos) & (disc > 0.0)
    three = ~(zero | pos | one)
    out[zero] = np.cbrt(-q[zero])
    C, diff = _stable_root_difference(d0[pos], d1[pos])
    out[pos] = diff / (3.0 * C)
    c = np.cbrt(0.5 * (d1[one] - np.sqrt(disc[one])))
    out[one] = -(c + d0[one] / c) / 3.0
    cos_t = np.clip(d1[three] / (2.0 * d0[three] ** 1.5), -1.0, 1.0)
    theta = np.arccos(cos_t)
    out[three] = -2.0 * np.sqrt(d0[three]) * np.cos(theta / 3.0 + 2.0 * np.pi / 3.0) / 3.0
    return out


def root_quartic(p, q):
    """Root of u^4 + p u + q = 0 by the closed forms of Sect. 3.11. Q + Delta0 / Q (Q^3 =
    (Delta1 + sqrt(disc)) / 2, Delta0 = 12 q < 0) is formed as (Q^2 + Delta0) / Q without
    cancellation (_stable_root_difference): the printed form loses up to 1e-2 of u where
    p is near 0. Where no real S remains (negative discriminant or Q + Delta0/Q <= 0) the
    root falls back to (-q)^(1/4), as the paper prescribes, and a slightly negative
    square-root argument is taken as zero."""
    p = np.asarray(p, dtype=np.float64)
    q = np.broadcast_to(np.asarray(q, dtype=np.float64), p.shape)
    d0 = 12.0 * q
    d1 = 27.0 * p * p
    disc = d1 * d1 - 4.0 * d0 ** 3
    fallback = np.sqrt(np.sqrt(-q))
    out = fallback.copy()
    ok = (p != 0.0) & (disc >= 0.0)
    Q, diff = _stable_root_difference(d0[ok], d1[ok])
    w = diff / Q
    good = w > 0.0
    S = 0.5 * np.sqrt(np.where(good, w, 1.0) / 3.0)
    pp = p[ok]
    arg = np.where(pp > 0.0, -4.0 * S * S + pp / S, -4.0 * S * S - pp / S)
    r = np.where(pp > 0.0, -S, S) + 0.5 * np.sqrt(np.maximum(arg, 0.0))
    sub = out[ok]
    sub[good] = r[good]
    out[ok] = sub
    return out


def root(p, q, n_exp):
    return root_cubic(p, q) if n_exp == 1 else root_quartic(p, q)


# --------------------------------------------------------------------------- operator

def operator(u, h, co):
    """N_h(u) = (f~_bar / h^2) lap7-numerator(u^(n+1)) - K / u."""
    w = u ** (co.n_exp + 1)
    return co.fbar * pm.laplacian7(w, h) - co.K / u


def nl_sweep(u, s, h, co, order=(0, 1)):
    """One red-black non-linear Gauss-Seidel sweep in place: every cell of a colour is
    set to the root of its depressed polynomial (red = (i+j+k) even, first)."""
    black = omg._colour_mask(u.shape[0])
    q = h * h * co.K / (6.0 * co.fbar)
    for colour in order:
        mask = black if colour == 1 else ~black
        nb = omg._neighbour_sum(u ** (co.n_exp + 1))
        p = -nb / 6.0 + h * h * s / (6.0 * co.fbar)
        u[mask] = root(p[mask], q, co.n_exp)
    return u


def is_coarsest(n):
    return n <= 4 or n % 4 != 0


def fas_cycle(u, s, h, co, pre=2, post=1, coarse_sweeps=32, cycle="F"):
    """One full-approximation-storage cycle in place (Sect. 3.7.2)."""
    n = u.shape[0]
    if is_coarsest(n):
        for _ in range(coarse_sweeps):
            nl_sweep(u, s, h, co, (0, 1))
        return u
    for _ in range(pre):
        nl_sweep(u, s, h, co, (0, 1))
    d = s - operator(u, h, co)
    H = 2.0 * h
    uH0 = omg.restrict(u, "fw")
    sH = operator(uH0, H, co) + omg.restrict(d, "fw")
    uH = uH0.copy()
    inner = {"V": ("V",), "W": ("W", "W"), "F": ("F", "V")}[cycle]
    for kind in inner:
        fas_cycle(uH, sH, H, co, pre, post, coarse_sweeps, kind)
    u += omg.prolong(uH - uH0)
    for _ in range(post):
        nl_sweep(u, s, h, co, (1, 0))
    return u


def residual_norm(u, s, h, co):
    return float(np.linalg.norm(s - operator(u, h, co)) / np.linalg.norm(s))


def solve(rho, co, u0=None, cycles=1, **kw):
    """`cycles` FAS cycles on the scalaron from u0 (default: the background u = 1).
    Returns (u, relative residual before each cycle and after the last)."""
    n = rho.shape[0]
    h = 1.0 / n
    s = co.source(rho)
    u = np.ones((n, n, n)) if u0 is None else np.array(u0, dtype=np.float64)
    hist = [residual_norm(u, s, h, co)]
    for _ in range(cycles):
        fas_cycle(u, s, h, co, **kw)
        hist.append(residual_norm(u, s, h, co))
    return u, hist


def scalaron(u, co):
    """f~ = f~_bar u^(n+1)."""
    return co.fbar * u ** (co.n_exp + 1)


# --------------------------------------------------------------------------- force, runs

def accel(x, n, a, f_r0, n_exp, c2, omega_m=0.3, omega_l=0.7, u0=None, cycles=1, mas="tsc",
          points=5, return_fields=False, **kw):
    """Particle accelerations in f(R): the Newtonian potential (exact seven-point solve,
    the multigrid's fixed point), the scalaron by `cycles` FAS cycles from u0, and the
    gradient of phi_N - (c~^2/2) f~ interpolated to the particles. x in grid units."""
    h = 1.0 / n
    rho = pm.deposit(x, n, mas)
    phin = pm.solve_exact7(pm.source(rho, a, omega_m), h)
    co = Coeffs(a, f_r0, n_exp, c2, omega_m, omega_l)
    u, hist = solve(rho, co, u0, cycles, **kw)
    phi = phin - 0.5 * c2 * scalaron(u, co)
    acc = pm.interp(x, pm.gradient(phi, h, points), mas)
    if return_fields:
        return acc, dict(rho=rho, phin=phin, u=u, phi=phi, hist=hist)
    return acc


def run(x, v, a_list, n, f_r0, n_exp, c2, omega_m=0.3, omega_l=0.7, **kw):
    """Kick-drift-kick steps (Sect. 3.4) with the LCDM background's time steps; the
    scalaron of each force evaluation starts from the previous one (the first from
    u = 1), without rescaling (Sect. 3.11). Returns (x, v, acc, u)."""
    from . import gravity as og
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    acc, fl = accel(x * n, n, a_list[0], f_r0, n_exp, c2, omega_m, omega_l, None,
                    return_fields=True, **kw)
    u = fl["u"]
    for a0, a1 in zip(a_list[:-1], a_list[1:]):
        t = og.tau(a0, a1, omega_m, omega_l)
        v = v + 0.5 * t * acc
        x = pm.wrap01(x + t * v)
        acc, fl = accel(x * n, n, a1, f_r0, n_exp, c2, omega_m, omega_l, u,
                        return_fields=True, **kw)
        u = fl["u"]
        v = v + 0.5 * t * acc
    return x, v, acc, u

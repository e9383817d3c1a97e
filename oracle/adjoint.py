"""FP64 vector-Jacobian products of the particle-mesh loop and the reverse leapfrog.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The forward map of one force evaluation is
    x -> rho(x) -> f = c (rho - mean rho) -> phi = L^+ f -> g = -D phi -> a = interp(x, g)
with c = (3/2) a Omega_m, L^+ the zero-mean inverse of the seven-point
Laplacian (symmetric), D the antisymmetric 5-point central difference, and the
same window W in deposit and interpolation. Its transpose, applied to a
cotangent lambda on the accelerations:
    g_bar   = interp^T(x) lambda            (a 3-component deposit)
    phi_bar = sum_d D_d g_bar_d             ((-D)^T = D)
    rho_bar = c L^+ (phi_bar - mean)        (L^+ symmetric, mean removal symmetric)
    x_bar   = sum_c grad W rho_bar_c  +  sum_c grad W (g_c . lambda_p)
The derivatives of the TSC window are continuous (C^1), so these are exact.
"""
from __future__ import annotations

import numpy as np

from . import pm


def dw_tsc(s):
    """d W_TSC / d s."""
    s = np.asarray(s, dtype=np.float64)
    a = np.abs(s)
    return np.where(a < 0.5, -2.0 * s, np.where(a < 1.5, -(1.5 - a) * np.sign(s), 0.0))


def dw_cic(s):
    s = np.asarray(s, dtype=np.float64)
    return np.where(np.abs(s) < 1.0, -np.sign(s), 0.0)


def _entries_with_grad(u, n, mas):
    """Yield (flat index, W, dW/du [np, 3]) over each particle's support."""
    firsts, ws, dws = [], [], []
    dfun = dw_tsc if mas == "tsc" else dw_cic
    for d in range(3):
        f, w = pm.axis_support(u[:, d], mas)
        cells = f[None] + np.arange(w.shape[0]).reshape(-1, 1)
        firsts.append(f)
        ws.append(w)
        dws.append(dfun(u[None, :, d] - (cells + 0.5)))
    s = ws[0].shape[0]
    for a in range(s):
        for b in range(s):
            for c in range(s):
                flat = ((((firsts[0] + a) % n) * n + (firsts[1] + b) % n) * n
                        + (firsts[2] + c) % n)
                w = ws[0][a] * ws[1][b] * ws[2][c]
                dw = np.stack([dws[0][a] * ws[1][b] * ws[2][c],
                               ws[0][a] * dws[1][b] * ws[2][c],
                               ws[0][a] * ws[1][b] * dws[2][c]], axis=-1)
                yield flat, w, dw


def deposit_vjp(x, n, rho_bar, mas="tsc", mass=None):
    """d<rho_bar, rho(x)>/dx for box-unit positions x [np, 3]."""
    u = np.asarray(x, dtype=np.float64) * n
    if mass is None:
        mass = n ** 3 / u.shape[0]
    rb = np.asarray(rho_bar, dtype=np.float64).reshape(-1)
    out = np.zeros_like(u)
    for flat, _, dw in _entries_with_grad(u, n, mas):
        out += dw * rb[flat][:, None]
    return mass * n * out


def interp_vjp(x, grid, lam, mas="tsc"):
    """Transpose of a = interp(x, grid): returns (grid_bar [n,n,n,3], x_bar [np, 3])."""
    n = grid.shape[0]
    u = np.asarray(x, dtype=np.float64) * n
    lam = np.asarray(lam, dtype=np.float64)
    g = grid.reshape(n ** 3, 3)
    gbar = np.zeros((n ** 3, 3), dtype=np.float64)
    xbar = np.zeros_like(u)
    for flat, w, dw in _entries_with_grad(u, n, mas):
        for d in range(3):
            gbar[:, d] += np.bincount(flat, weights=w * lam[:, d], minlength=n ** 3)
        xbar += dw * np.sum(g[flat] * lam, axis=1)[:, None]
    return gbar.reshape(n, n, n, 3), n * xbar


def gradient_vjp(gbar, h, points=5):
    """Transpose of g = -D phi: phi_bar = sum_d D_d g_bar_d."""
    return sum(pm.derivative(gbar[..., d], h, d, points) for d in range(3))


def solve_vjp(phi_bar, h, coef):
    """Transpose of phi = L^+ (c (rho - mean rho)): rho_bar = c L^+ (phi_bar - mean)."""
    return coef * pm.solve_exact7(phi_bar, h)


def accel_vjp(x, n, a, lam, mas="tsc", omega_m=1.0, points=5, g=None):
    """x_bar = (d accel(x) / d x)^T lam for box-unit x (exact7 solve)."""
    h = 1.0 / n
    x = np.asarray(x, dtype=np.float64)
    if g is None:
        _, fields = pm.accel(x * n, n, a, "exact7", mas, omega_m, points=points,
                             return_fields=True)
        g = fields["g"]
    gbar, xbar = interp_vjp(x, g, lam, mas)
    phibar = gradient_vjp(gbar, h, points)
    rhobar = solve_vjp(phibar, h, 1.5 * a * omega_m)
    return xbar + deposit_vjp(x, n, rhobar, mas)


def density_loss(x, n, weight, mas="tsc"):
    """L = sum_c w_c delta_c^2 with delta = rho~ - 1."""
    delta = pm.deposit(np.asarray(x, dtype=np.float64) * n, n, mas) - 1.0
    return float(np.sum(weight * delta * delta))


def density_loss_vjp(x, n, weight, mas="tsc"):
    delta = pm.deposit(np.asarray(x, dtype=np.float64) * n, n, mas) - 1.0
    return deposit_vjp(x, n, 2.0 * weight * delta, mas)


def forward_trajectory(x0, v0, a_list, n, mas="tsc"):
    """States (x_i, v_i, acc_i) at every a_i, exact7 solve."""
    x = np.asarray(x0, dtype=np.float64)
    v = np.asarray(v0, dtype=np.float64)
    acc = pm.accel(x * n, n, a_list[0], "exact7", mas)
    states = [(x, v, acc)]
    for a0, a1 in zip(a_list[:-1], a_list[1:]):
        x, v, acc = pm.kdk_step(x, v, acc, a0, a1, n, solver="exact7", mas=mas)
        states.append((x, v, acc))
    return states


def kdk_adjoint(states, a_list, n, xbar, vbar, mas="tsc"):
    """Reverse the leapfrog. For each step, from (x_bar, v_bar) at a_{i+1}:
        x_bar += (tau/2) J(x_{i+1})^T v_bar;  v_bar += tau x_bar;  x_bar += (tau/2) J(x_i)^T v_bar
    where J(x) = d accel(x) / dx at the step's scale factor.
    """
    xbar = np.array(xbar, dtype=np.float64)
    vbar = np.array(vbar, dtype=np.float64)
    for i in range(len(a_list) - 2, -1, -1):
        a0, a1 = a_list[i], a_list[i + 1]
        tau = pm.tau_eds(a0, a1)
        x0, x1 = states[i][0], states[i + 1][0]
        xbar = xbar + 0.5 * tau * accel_vjp(x1, n, a1, vbar, mas)
        vbar = vbar + tau * xbar
        xbar = xbar + 0.5 * tau * accel_vjp(x0, n, a0, vbar, mas)
    return xbar, vbar


def ic_gradient(psi, q, a_list, n, weight, mas="tsc"):
    """dL/dPsi for x0 = q + Psi, v0 = a0^{1/2} Psi, L = density_loss at a_list[-1]."""
    a0 = a_list[0]
    x0 = pm.wrap01(q + psi)
    v0 = np.sqrt(a0) * psi
    states = forward_trajectory(x0, v0, a_list, n, mas)
    xbar = density_loss_vjp(states[-1][0], n, weight, mas)
    xbar, vbar = kdk_adjoint(states, a_list, n, xbar, np.zeros_like(xbar), mas)
    loss = density_loss(states[-1][0], n, weight, mas)
    return loss, xbar + np.sqrt(a0) * vbar


def ic_loss(psi, q, a_list, n, weight, mas="tsc"):
    a0 = a_list[0]
    x0 = pm.wrap01(q + psi)
    v0 = np.sqrt(a0) * psi
    states = forward_trajectory(x0, v0, a_list, n, mas)
    return density_loss(states[-1][0], n, weight, mas)

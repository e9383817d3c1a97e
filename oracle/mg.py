"""FP64 linear multigrid for the periodic seven-point Poisson problem.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper's linear multigrid (Sect. 3.7.1) with red-black Gauss-Seidel
smoothing (Sect. 3.6). The paper's V-cycle listing is a figure that is not
available, so the cycle below is built from the prose:
  1. pre-smoothing: `pre` red-black sweeps, u <- (1-w) u + w (L(u) - h^2 f) / 6
     (Jacobi update on one colour at a time; red = (i+j+k) even, red first);
  2. residual d = f - laplacian7(u), restricted to the grid of size H = 2h;
  3. the coarse error equation L_H v = d_H is solved recursively, starting from
     the Jacobi guess v = -H^2 d_H / 6, until the grid has at most 16 cells per
     side (or cannot be halved to an even size);
  4. prolongation-correction u += P v with the 27/64, 9/64, 3/64, 1/64 weights
     (per axis 3/4 for the nearest coarse centre and 1/4 for the next);
  5. post-smoothing: `post` sweeps in mirrored colour order (black first).
Restriction "fw" is the full weighting R = P^T / 8 (per axis (1,3,3,1)/8 over
fine cells 2J-1 .. 2J+2); "avg" is the paper's mean of the 8 children.
The coarsest grid is smoothed until its residual drops by 1e-3 (at most 500
sweeps), with the mean removed from its right-hand side and solution.
"""
from __future__ import annotations

import numpy as np

from .pm import laplacian7


def _neighbour_sum(u):
    s = np.zeros_like(u)
    for ax in range(3):
        s += np.roll(u, 1, axis=ax) + np.roll(u, -1, axis=ax)
    return s


def _colour_mask(n):
    i = np.arange(n)
    return ((i[:, None, None] + i[None, :, None] + i[None, None, :]) % 2).astype(bool)


def rbgs_sweep(u, f, h, omega=1.0, order=(0, 1)):
    """One red-black Gauss-Seidel sweep in place; order (0, 1) = red then black."""
    black = _colour_mask(u.shape[0])
    for colour in order:
        mask = black if colour == 1 else ~black
        new = (_neighbour_sum(u) - h * h * f) / 6.0
        u[mask] = (1.0 - omega) * u[mask] + omega * new[mask]
    return u


def _restrict_axis(r, axis, kind):
    n = r.shape[axis]
    take = lambda idx: np.take(r, np.asarray(idx) % n, axis=axis)  # noqa: E731
    j2 = 2 * np.arange(n // 2)
    if kind == "fw":
        return (take(j2 - 1) + 3.0 * take(j2) + 3.0 * take(j2 + 1) + take(j2 + 2)) / 8.0
    if kind == "avg":
        return 0.5 * (take(j2) + take(j2 + 1))
    raise ValueError(kind)


def restrict(r, kind="fw"):
    """Fine -> coarse transfer (separable per axis)."""
    out = r
    for ax in range(3):
        out = _restrict_axis(out, ax, kind)
    return out


def _prolong_axis(v, axis):
    nc = v.shape[axis]
    take = lambda idx: np.take(v, np.asarray(idx) % nc, axis=axis)  # noqa: E731
    jc = np.arange(nc)
    even = 0.75 * take(jc) + 0.25 * take(jc - 1)   # fine 2J: centre (J + 1/4) H
    odd = 0.75 * take(jc) + 0.25 * take(jc + 1)    # fine 2J+1: centre (J + 3/4) H
    shape = list(v.shape)
    shape[axis] = 2 * nc
    out = np.empty(shape, dtype=np.float64)
    sl_e = [slice(None)] * v.ndim
    sl_o = [slice(None)] * v.ndim
    sl_e[axis] = slice(0, None, 2)
    sl_o[axis] = slice(1, None, 2)
    out[tuple(sl_e)] = even
    out[tuple(sl_o)] = odd
    return out


def prolong(v):
    """Coarse -> fine trilinear prolongation (paper Sect. 3.7.1 weights)."""
    out = v
    for ax in range(3):
        out = _prolong_axis(out, ax)
    return out


def is_coarsest(n, coarsest=16):
    return n <= coarsest or n % 4 != 0


def coarse_solve(u, f, h, tol=1e-3, max_sweeps=500):
    f = f - f.mean()
    r0 = np.linalg.norm(f - laplacian7(u, h))
    for _ in range(max_sweeps):
        rbgs_sweep(u, f, h)
        u -= u.mean()
        if np.linalg.norm(f - laplacian7(u, h)) <= tol * r0:
            break
    return u


def vcycle(u, f, h, pre=2, post=2, omega=1.0, restriction="fw", coarsest=16, cycle="V"):
    """One multigrid cycle in place. The paper names V, F and W cycles (Sect. 3.7.1,
    App. C) without spelling out F and W; they follow the usual definitions: the coarse
    error equation is treated by one V cycle (V), by two W cycles in a row (W), or by
    an F cycle followed by a V cycle (F), the second recursion continuing from the
    first one's coarse iterate."""
    n = u.shape[0]
    if is_coarsest(n, coarsest):
        return coarse_solve(u, f, h)
    for _ in range(pre):
        rbgs_sweep(u, f, h, omega, (0, 1))
    d = f - laplacian7(u, h)
    dH = restrict(d, restriction)
    H = 2.0 * h
    vH = -(H * H) * dH / 6.0
    inner = {"V": ("V",), "W": ("W", "W"), "F": ("F", "V")}[cycle]
    for kind in inner:
        vcycle(vH, dH, H, pre, post, omega, restriction, coarsest, kind)
    u += prolong(vH)
    for _ in range(post):
        rbgs_sweep(u, f, h, omega, (1, 0))
    return u


def truncation_error(u, h, restriction="fw"):
    """Estimate of the truncation error on the coarse grid (paper Sect. 3.7.1, the
    estimate it takes from the literature): tau = L_H(R u) - R(L_h u), H = 2h, with R
    the restriction of the cycle."""
    return laplacian7(restrict(u, restriction), 2.0 * h) - restrict(laplacian7(u, h), restriction)


def solve(f, h, u0=None, tol=1e-10, max_cycles=50, alpha=None, **kw):
    """V-cycles until ||f - L u|| / ||f|| < tol, or, with alpha, until the residual is
    below alpha times the truncation-error estimate (Eq. multigrid_threshold): with
    both norms the square root of the sum of squares over their own grid (the
    residual over the fine cells, the estimate over the coarse cells),
    ||f - L u|| < alpha ||truncation_error(u)||. Returns (u, list of relative residuals).

    The starting guess is the Jacobi step u = -h^2 f / 6 (paper Sect. 3.7.1)
    unless u0 (a warm start, paper Sect. 3.9) is given.
    """
    f = np.asarray(f, dtype=np.float64)
    u = -(h * h) * f / 6.0 if u0 is None else np.array(u0, dtype=np.float64)
    fn = np.linalg.norm(f)
    hist = []
    restriction = kw.get("restriction", "fw")
    for _ in range(max_cycles + 1):
        dn = np.linalg.norm(f - laplacian7(u, h))
        rel = dn / fn if fn > 0 else 0.0
        hist.append(rel)
        if alpha is not None:
            done = dn < alpha * np.linalg.norm(truncation_error(u, h, restriction))
        else:
            done = rel < tol
        if done or len(hist) > max_cycles:
            break
        vcycle(u, f, h, **kw)
    return u - u.mean(), hist

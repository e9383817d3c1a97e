"""Seeded synthetic initial conditions for the particle-mesh loop.

This module generates inputs only. It holds none of the particle-mesh
arithmetic (no mass assignment, no Poisson stencil, no gradient stencil, no
integrator); both the FP64 oracle and the HIP path consume what it returns.

Recipe (paper Sect. 3.3, initial conditions):
  * Gaussian white noise. The paper draws W(k) = A e^{i theta} with Rayleigh
    amplitudes and Hermitian symmetry. The real-space construction used here
    (rfftn of real N(0,1) noise) has exactly that distribution and is Hermitian
    by construction.
  * Linear density  delta(k) = sqrt(P(k)) W(k),  P(k) = k^n  (optionally times
    exp(-k^2/k_c^2)); the k = 0 mode and the Nyquist planes are set to zero.
  * First-order LPT (Zel'dovich): Psi = -grad(nabla^-2 delta), i.e.
    Psi(k) = i k delta(k) / k^2, evaluated spectrally (the paper computes IC
    derivatives in Fourier space).
  * The amplitude is fixed by rescaling so that sqrt(<|Psi|^2>) equals the
    requested rms displacement in cells (the paper's (2 pi)^{3/2} factor then
    drops out).
  * Particles start at cell centres (paper App. B.2): q = (idx + 1/2) h.
    x = q + Psi, and in an Einstein-de Sitter background the growing-mode
    velocity in supercomoving time (dt~ = H0 dt / a^2, paper Sect. 3.1) is
    v = dx/dt~ = a^{1/2} Psi, since D = a and da/dt~ = a^{3/2}.

Units: box length 1, positions in [0, 1), velocities in box units per unit of
supercomoving time.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np
import scipy.fft as sfft

__all__ = [
    "displacement_field",
    "zeldovich_particles",
    "to_cell_offset",
    "ensemble_draw",
    "unit_directions",
    "ParticleSet",
]


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def displacement_field(n: int, spectral_index: float, rms_cells: float, seed: int,
                       cutoff_k: float | None = None, precision: str = "f64") -> np.ndarray:
    """Zel'dovich displacement Psi on the n^3 lattice, shape [n, n, n, 3], box units.

    spectral_index: n_s in P(k) ~ k^{n_s}.  cutoff_k: k_c of exp(-k^2/k_c^2) or None.
    precision: "f64" (default) or "f32" (used for 512^3 to bound memory and time).
    """
    if n < 2 or n % 2:
        raise ValueError("n must be even and >= 2")
    rdt = np.float64 if precision == "f64" else np.float32
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.standard_normal((n, n, n), dtype=rdt)
    wk = sfft.rfftn(noise, workers=_workers())
    del noise
    m_full = np.fft.fftfreq(n, d=1.0 / n).astype(rdt)
    m_half = np.arange(n // 2 + 1, dtype=rdt)
    k_full = (2.0 * np.pi) * m_full
    k_half = (2.0 * np.pi) * m_half
    kx = k_full[:, None, None]
    ky = k_full[None, :, None]
    kz = k_half[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    amp = np.power(k2, 0.25 * spectral_index)  # sqrt(P) = k^{n/2} = (k^2)^{n/4}
    if cutoff_k is not None:
        amp *= np.exp(-0.5 * k2 / (cutoff_k * cutoff_k))
    amp[0, 0, 0] = 0.0
    # zero the Nyquist planes (their modes have no well-defined gradient sign)
    amp[n // 2, :, :] = 0.0
    amp[:, n // 2, :] = 0.0
    amp[:, :, n // 2] = 0.0
    dk = wk * amp
    del wk, amp
    inv_k2 = 1.0 / k2
    inv_k2[0, 0, 0] = 0.0
    psi = np.empty((n, n, n, 3), dtype=rdt)
    for d, kd in enumerate((kx, ky, kz)):
        comp = (1j * kd) * dk * inv_k2
        psi[..., d] = sfft.irfftn(comp, s=(n, n, n), workers=_workers())
        del comp
    rms = float(np.sqrt(np.mean(np.sum(psi.astype(np.float64) ** 2, axis=-1))))
    if rms == 0.0:
        raise ValueError("degenerate field")
    psi *= rdt(rms_cells / n / rms)
    return psi


@dataclass
class ParticleSet:
    """Particles in box units plus the lattice they started from (FP32 on output)."""
    pos: np.ndarray   # [np, 3] float32 in [0, 1)
    vel: np.ndarray   # [np, 3] float32, box units per supercomoving time
    n: int
    a: float


def _wrap01_f32(x64: np.ndarray) -> np.ndarray:
    x = np.mod(x64, 1.0).astype(np.float32)
    x[x >= np.float32(1.0)] = np.float32(0.0)
    return x


def zeldovich_particles(n: int, spectral_index: float, rms_cells: float, a: float, seed: int,
                        cutoff_k: float | None = None, precision: str = "f64") -> ParticleSet:
    """One particle per cell, displaced from the cell centres by Psi; v = a^{1/2} Psi."""
    psi = displacement_field(n, spectral_index, rms_cells, seed, cutoff_k, precision)
    h = 1.0 / n
    idx = (np.arange(n, dtype=np.float64) + 0.5) * h
    pos = np.empty((n, n, n, 3), dtype=np.float32)
    pos[..., 0] = _wrap01_f32(idx[:, None, None] + psi[..., 0])
    pos[..., 1] = _wrap01_f32(idx[None, :, None] + psi[..., 1])
    pos[..., 2] = _wrap01_f32(idx[None, None, :] + psi[..., 2])
    vel = (np.sqrt(a) * psi).astype(np.float32)
    return ParticleSet(pos.reshape(-1, 3), vel.reshape(-1, 3), n, a)


def to_cell_offset(pos: np.ndarray, n: int):
    """Box-unit FP32 positions -> (int32 linear cell index [np], FP32 in-cell offset [np, 3]).

    u = x n (cell units) is split into floor(u) and u - floor(u) in FP64; an
    offset that rounds up to 1.0 in FP32 is carried into the cell index.
    """
    u = pos.astype(np.float64) * n
    c = np.floor(u)
    off = (u - c).astype(np.float32)
    carry = off >= np.float32(1.0)
    off[carry] = 0.0
    c = (c.astype(np.int64) + carry) % n
    cell = (c[:, 0] * n + c[:, 1]) * n + c[:, 2]
    return cell.astype(np.int32), off


def from_cell_offset(cell: np.ndarray, off: np.ndarray, n: int) -> np.ndarray:
    """Inverse of to_cell_offset, exact in FP64: box-unit positions [np, 3]."""
    c = cell.astype(np.int64)
    ci = np.stack([c // (n * n), (c // n) % n, c % n], axis=-1).astype(np.float64)
    return (ci + off.astype(np.float64)) / n


def ensemble_draw(master_seed: int, boxes: int, sizes=(32, 48, 64, 96, 128),
                  index_range=(-2.5, -1.0)):
    """Per-box (grid size, spectral index, seed) for an ensemble of independent boxes."""
    rng = np.random.Generator(np.random.PCG64(master_seed))
    ns = rng.choice(np.asarray(sizes), size=boxes)
    idx = rng.uniform(index_range[0], index_range[1], size=boxes)
    return [(int(ns[b]), float(idx[b]), 1000 + b) for b in range(boxes)]


def lattice_points(n: int) -> np.ndarray:
    """Cell centres ((i, j, k) + 1/2) / n as FP32 [n^3, 3], the unperturbed particle lattice."""
    idx = ((np.arange(n, dtype=np.float64) + 0.5) / n).astype(np.float32)
    q = np.empty((n, n, n, 3), dtype=np.float32)
    q[..., 0] = idx[:, None, None]
    q[..., 1] = idx[None, :, None]
    q[..., 2] = idx[None, None, :]
    return q.reshape(-1, 3)


def weight_grid(n: int, seed: int) -> np.ndarray:
    """Seeded uniform [0, 1) FP32 weights on the n^3 grid (loss weights of a density objective)."""
    return np.random.default_rng(seed).random((n, n, n), dtype=np.float64).astype(np.float32)


def direction_fields(n: int, count: int, seed: int, smooth_index: float = -1.5) -> list:
    """Seeded perturbation directions of a displacement field, FP32 [n^3, 3] each, unit rms
    per component: even entries are smooth Gaussian random fields (P ~ k^smooth_index), odd
    entries white noise."""
    out = []
    rng = np.random.default_rng(seed)
    for i in range(count):
        if i % 2 == 0:
            d = displacement_field(n, smooth_index, 1.0, seed + 7919 * (i + 1)).reshape(-1, 3)
        else:
            d = rng.standard_normal((n ** 3, 3))
        d = d / np.sqrt(np.mean(d * d))
        out.append(d.astype(np.float32))
    return out


def unit_directions(npart: int, count: int, seed: int) -> list:
    """Seeded Gaussian white-noise directions of a displacement field, FP64 [npart, 3] each,
    normalised to unit L2 norm over all particles and components."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        d = rng.standard_normal((npart, 3))
        out.append(d / np.linalg.norm(d))
    return out

"""FP64 reference of the initial conditions and the power-spectrum estimator.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Initial conditions (paper Sect. 3.3, App. A): a Gaussian density field from a
given white-noise realisation and a linear power spectrum, displaced from the
lattice of cell centres by Lagrangian perturbation theory to first, second or
third order, with every derivative taken in Fourier space. Conventions:
  * unit periodic box, n cells per side, N = n^3; Fourier series
    delta(x) = sum_k delta_k e^{i k.x}, k = 2 pi m, <|delta_k|^2> = P(k) (box
    volume 1); the white noise w(x) ~ N(0, 1) per cell gives unit-variance modes
    DFT[w] / sqrt(N), so DFT[delta] = sqrt(N) sqrt(P(k)) DFT[w];
  * P(k) is given at a = 1 as a table, interpolated linearly in log k - log P
    and held constant beyond its ends;
  * the k = 0 mode and the Nyquist planes of every field whose derivatives are
    taken are zero (an odd derivative has no real image there);
  * Einstein-de Sitter growth: D = a, and the higher-order growth factors of the
    paper's App. A closed forms, D2 = -3/7 D^2, D3a = -1/3 D^3, D3b = 10/21 D^3,
    D3c = -1/7 D^3, each growing as a^order, so the supercomoving velocity of an
    order-k term is k a^(1/2) D^(k) Psi^(k);
  * dealias: products of fields are formed on a grid of 2n cells per side from
    zero-padded spectra and truncated back (free of aliasing for the quadratic and
    cubic terms; the paper's 3/2 rule is the same for quadratic terms).
Power spectrum (the estimator of Sect. 4): delta = rho / mean(rho) - 1, modes
deconvolved by the window W = prod_d sinc(k_d h / 2)^p, P in shells of
round(|m|) = 1, 2, ...
"""
from __future__ import annotations

import numpy as np

LPT_GROWTH = {"2": -3.0 / 7.0, "3a": -1.0 / 3.0, "3b": 10.0 / 21.0, "3c": -1.0 / 7.0}


def _modes(n):
    """Wavevector components (k = 2 pi m) on the rfftn layout, and a mask of the modes
    that are kept (not on a Nyquist plane)."""
    m = np.fft.fftfreq(n, d=1.0 / n)
    mh = np.arange(n // 2 + 1, dtype=np.float64)
    kx = (2 * np.pi * m)[:, None, None]
    ky = (2 * np.pi * m)[None, :, None]
    kz = (2 * np.pi * mh)[None, None, :]
    keep = ((np.abs(m) != n // 2)[:, None, None] & (np.abs(m) != n // 2)[None, :, None]
            & (mh != n // 2)[None, None, :])
    return (kx, ky, kz), keep


def power_law_table(amplitude, index, kmin=1.0, kmax=1e4, points=64):
    """A table of P(k) = amplitude k^index (log-spaced k)."""
    k = np.geomspace(kmin, kmax, points)
    return k, amplitude * k ** index


def interp_pk(k, k_tab, p_tab):
    """Log-log linear interpolation of the table, constant beyond its ends."""
    lk = np.log(np.clip(k, k_tab[0], k_tab[-1]))
    return np.exp(np.interp(lk, np.log(k_tab), np.log(p_tab)))


def linear_density_spectrum(noise, k_tab, p_tab):
    """rfftn of the linear density at a = 1: sqrt(N) sqrt(P(k)) rfftn(w), with the k = 0
    mode and the Nyquist planes set to zero."""
    noise = np.asarray(noise, dtype=np.float64)
    n = noise.shape[0]
    (kx, ky, kz), keep = _modes(n)
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    kk[0, 0, 0] = 1.0
    dk = np.sqrt(noise.size) * np.sqrt(interp_pk(kk, k_tab, p_tab)) * np.fft.rfftn(noise)
    dk[0, 0, 0] = 0.0
    return np.where(keep, dk, 0.0)


class _Spectral:
    """Fourier-space derivatives on an n^3 grid and products formed on n or 2n."""

    def __init__(self, n, dealias):
        self.n = n
        self.k, self.keep = _modes(n)
        k2 = sum(c * c for c in self.k)
        k2[0, 0, 0] = 1.0
        self.inv_k2 = 1.0 / k2
        self.inv_k2[0, 0, 0] = 0.0
        self.m = 2 * n if dealias else n

    def to_real(self, spec):
        """Real field on the product grid (zero-padded when it is finer)."""
        n, m = self.n, self.m
        if m == n:
            return np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2))
        big = np.zeros((m, m, m // 2 + 1), dtype=complex)
        h = n // 2
        idx = np.r_[0:h, m - h:m]
        big[np.ix_(idx, idx, np.arange(h + 1))] = spec
        return np.fft.irfftn(big, s=(m, m, m), axes=(0, 1, 2)) * (m / n) ** 3

    def from_real(self, field):
        """Spectrum on the n grid of a real field on the product grid (truncated), with
        the Nyquist planes dropped."""
        n, m = self.n, self.m
        full = np.fft.rfftn(field)
        if m != n:
            h = n // 2
            idx = np.r_[0:h, m - h:m]
            full = full[np.ix_(idx, idx, np.arange(h + 1))] * (n / m) ** 3
        return np.where(self.keep, full, 0.0)

    def second_derivatives(self, phik):
        """phi_,ij for i <= j as real fields on the product grid."""
        out = {}
        for i in range(3):
            for j in range(i, 3):
                out[(i, j)] = self.to_real(-self.k[i] * self.k[j] * phik)
        return out

    def gradient(self, phik):
        """grad phi on the n grid, [n, n, n, 3]."""
        return np.stack([np.fft.irfftn(1j * self.k[d] * phik, s=(self.n,) * 3, axes=(0, 1, 2))
                         for d in range(3)], axis=-1)

    def inverse_laplacian(self, spec):
        return -spec * self.inv_k2


def _sym(d, i, j):
    return d[(min(i, j), max(i, j))]


def lpt_displacements(noise, k_tab, p_tab, order=3, dealias=True):
    """The displacement fields Psi^(1), Psi^(2), Psi^(3a), Psi^(3b), Psi^(3c) at a = 1
    (paper Sect. 3.3), each [n, n, n, 3] in box units, as a dict keyed '1', '2', '3a',
    '3b', '3c' (up to the given order)."""
    noise = np.asarray(noise, dtype=np.float64)
    dk = linear_density_spectrum(noise, k_tab, p_tab)
    return lpt_from_density(dk, noise.shape[0], order, dealias)


def lpt_sources(dk, n, order=3, dealias=True):
    """The real-space sources of the higher orders on the product grid, from the
    spectrum dk of the linear density: second derivatives of phi(1) (and of phi(2)),
    the second-order source lap phi(2), and at third order det phi(1)_ij, lap phi(3b)
    and the three components of lap A(3c) (the paper's explicit forms). Returns
    (spectral helper, phi(1) spectrum, phi(2) spectrum or None, dict of fields)."""
    sp = _Spectral(n, dealias)
    phi1 = sp.inverse_laplacian(dk)                       # phi(1) = lap^-1 delta
    fields = {}
    if order < 2:
        return sp, phi1, None, fields
    d1 = sp.second_derivatives(phi1)
    a = lambda i, j: _sym(d1, i, j)  # noqa: E731
    # lap phi(2) = (1/2) [phi_ii phi_jj - phi_ij phi_ij] (sums over i, j)
    fields["s2"] = (a(0, 0) * (a(1, 1) + a(2, 2)) + a(1, 1) * a(2, 2)
                    - a(0, 1) ** 2 - a(0, 2) ** 2 - a(1, 2) ** 2)
    phi2 = sp.inverse_laplacian(sp.from_real(fields["s2"]))
    fields["d1"] = d1
    if order < 3:
        return sp, phi1, phi2, fields
    fields["det"] = (a(0, 0) * a(1, 1) * a(2, 2) + 2 * a(0, 1) * a(0, 2) * a(1, 2)
                     - a(1, 2) ** 2 * a(0, 0) - a(0, 2) ** 2 * a(1, 1) - a(0, 1) ** 2 * a(2, 2))
    d2 = sp.second_derivatives(phi2)
    fields["d2"] = d2
    b = lambda i, j: _sym(d2, i, j)  # noqa: E731
    fields["s3b"] = (0.5 * a(0, 0) * (b(1, 1) + b(2, 2)) + 0.5 * a(1, 1) * (b(0, 0) + b(2, 2))
                     + 0.5 * a(2, 2) * (b(0, 0) + b(1, 1))
                     - a(0, 1) * b(0, 1) - a(0, 2) * b(0, 2) - a(1, 2) * b(1, 2))
    fields["rx"] = (b(0, 1) * a(0, 2) - b(0, 2) * a(0, 1) + a(1, 2) * (b(1, 1) - b(2, 2))
                    - b(1, 2) * (a(1, 1) - a(2, 2)))
    fields["ry"] = (b(1, 2) * a(0, 1) - b(0, 1) * a(1, 2) + a(0, 2) * (b(2, 2) - b(0, 0))
                    - b(0, 2) * (a(2, 2) - a(0, 0)))
    fields["rz"] = (b(0, 2) * a(1, 2) - b(1, 2) * a(0, 2) + a(0, 1) * (b(0, 0) - b(1, 1))
                    - b(0, 1) * (a(0, 0) - a(1, 1)))
    return sp, phi1, phi2, fields


def lpt_from_density(dk, n, order=3, dealias=True):
    """The LPT displacement fields of a linear density given by its rfftn dk (Nyquist
    planes zero), as lpt_displacements."""
    sp, phi1, phi2, f = lpt_sources(dk, n, order, dealias)
    out = {"1": -sp.gradient(phi1)}                       # Psi(1) = -grad phi(1)
    if order < 2:
        return out
    out["2"] = sp.gradient(phi2)                          # Psi(2) = grad phi(2)
    if order < 3:
        return out
    out["3a"] = sp.gradient(sp.inverse_laplacian(sp.from_real(f["det"])))
    out["3b"] = sp.gradient(sp.inverse_laplacian(sp.from_real(f["s3b"])))
    ak = [sp.inverse_laplacian(sp.from_real(f[r])) for r in ("rx", "ry", "rz")]
    k = sp.k
    curl = [1j * (k[1] * ak[2] - k[2] * ak[1]), 1j * (k[2] * ak[0] - k[0] * ak[2]),
            1j * (k[0] * ak[1] - k[1] * ak[0])]
    out["3c"] = np.stack([np.fft.irfftn(c, s=(n,) * 3, axes=(0, 1, 2)) for c in curl],
                         axis=-1)                         # Psi(3c) = curl A(3c)
    return out


def lpt_state(noise, k_tab, p_tab, a, order=3, dealias=True):
    """Positions x = q + sum D^(k)(a) Psi^(k) (wrapped into [0, 1)) and supercomoving
    velocities v = a^(1/2) sum k D^(k)(a) Psi^(k) of the particles of the lattice of
    cell centres (row-major), Einstein-de Sitter (Eqs. x_ini_LPT, v_ini_LPT)."""
    n = np.asarray(noise).shape[0]
    psi = lpt_displacements(noise, k_tab, p_tab, order, dealias)
    growth = {"1": (a, 1), "2": (LPT_GROWTH["2"] * a ** 2, 2),
              "3a": (LPT_GROWTH["3a"] * a ** 3, 3), "3b": (LPT_GROWTH["3b"] * a ** 3, 3),
              "3c": (LPT_GROWTH["3c"] * a ** 3, 3)}
    disp = np.zeros((n, n, n, 3))
    vel = np.zeros((n, n, n, 3))
    for key, field in psi.items():
        d, kord = growth[key]
        disp += d * field
        vel += np.sqrt(a) * kord * d * field
    c = (np.arange(n) + 0.5) / n
    q = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1)
    x = np.mod(q + disp, 1.0)
    x[x >= 1.0] = 0.0
    return x.reshape(-1, 3), vel.reshape(-1, 3)


def power_spectrum(rho, deconv=3, nbins=None):
    """P(k) of delta = rho / mean - 1 in shells round(|m|) = 1 .. nbins: returns
    (P, mean |k| per shell, modes per shell), counting the full sphere of modes. Each
    mode is delta_k = DFT[delta] / N divided by W(k) = prod_d sinc(k_d h / 2)^deconv."""
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape[0]
    if nbins is None:
        nbins = n // 2
    delta = rho / rho.mean() - 1.0
    fk = np.fft.rfftn(delta) / rho.size
    m = np.fft.fftfreq(n, d=1.0 / n)
    mh = np.arange(n // 2 + 1, dtype=np.float64)
    mx, my, mz = m[:, None, None], m[None, :, None], mh[None, None, :]
    w = np.ones_like(fk.real)
    for md in (mx, my, mz):
        x = np.pi * md / n
        w = w * np.where(x == 0.0, 1.0, np.sin(x) / np.where(x == 0.0, 1.0, x)) ** deconv
    power = np.abs(fk) ** 2 / w ** 2
    weight = np.where((mz == 0) | (mz == n // 2), 1.0, 2.0) * np.ones_like(power)
    kmag = np.sqrt(mx * mx + my * my + mz * mz)
    b = np.rint(kmag).astype(np.int64)
    sel = (b >= 1) & (b <= nbins)
    cnt = np.bincount(b[sel], weights=weight[sel], minlength=nbins + 1)[1:]
    pk = np.bincount(b[sel], weights=(weight * power)[sel], minlength=nbins + 1)[1:]
    ks = np.bincount(b[sel], weights=(weight * 2 * np.pi * kmag)[sel], minlength=nbins + 1)[1:]
    with np.errstate(invalid="ignore", divide="ignore"):
        return pk / cnt, ks / cnt, cnt.astype(np.int64)

"""Seeded synthetic particle realisations (inputs only: no solver arithmetic).

These generators stand in for the paper's galaxies, whose observed surface
densities are not available: disks with the shapes the paper uses.

* Kuzmin disk (Sec. 3.1): enclosed-mass fraction f = 1 - a/sqrt(R^2+a^2),
  so R = a sqrt((1-f)^-2 - 1) for uniform f, uniform azimuth, zero thickness.
* Exponential disk with a sech^2 vertical profile (Sec. 3.3-3.5): radius
  from the inverse of the enclosed fraction 1 - (1+x) e^-x (x = R/Rd) via the
  lower real branch of the Lambert W function, z = z0 artanh(2u - 1), which
  samples rho ~ sech^2(z/z0).
* Two-component galaxy (Sec. 3.4): half of the particles are stars and half
  are gas, each component with equal particle masses summing to its mass.

All draws use NumPy's PCG64 with seed 31851201 + 100 * config + realisation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import lambertw

SEED_BASE = 31851201


def seed_for(config: int, realisation: int = 0) -> int:
    return SEED_BASE + 100 * int(config) + int(realisation)


@dataclass
class Particles:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def total_mass(self) -> float:
        return float(self.m.sum())

    def shuffled(self, seed: int) -> "Particles":
        p = np.random.Generator(np.random.PCG64(seed)).permutation(self.n)
        return Particles(self.x[p].copy(), self.y[p].copy(), self.z[p].copy(), self.m[p].copy())


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def kuzmin_disk(n: int, a: float, M: float, seed: int) -> Particles:
    rng = _rng(seed)
    f = rng.random(n)
    R = a * np.sqrt((1.0 - f) ** -2 - 1.0)
    phi = 2.0 * np.pi * rng.random(n)
    x = R * np.cos(phi)
    y = R * np.sin(phi)
    z = np.zeros(n)
    m = np.full(n, M / n)
    return Particles(x, y, z, m)


def kuzmin_disk_stratified(n: int, a: float, M: float) -> Particles:
    """The Kuzmin disk with its inverse-CDF radii taken at the stratified mass
    fractions f = (i + 1/2) / n and azimuths from the golden-ratio sequence:
    the same distribution as kuzmin_disk with far less sampling noise, for
    measuring the solver's own accuracy."""
    i = np.arange(n, dtype=np.float64)
    f = (i + 0.5) / n
    R = a * np.sqrt((1.0 - f) ** -2 - 1.0)
    phi = 2.0 * np.pi * np.mod(i * 0.6180339887498949, 1.0)
    return Particles(R * np.cos(phi), R * np.sin(phi), np.zeros(n), np.full(n, M / n))


def _radical_inverse(i: np.ndarray, base: int) -> np.ndarray:
    """Van der Corput sequence in the given base (low-discrepancy points in [0, 1))."""
    out = np.zeros(i.shape, dtype=np.float64)
    f = 1.0 / base
    k = i.astype(np.int64).copy()
    while np.any(k > 0):
        out += f * (k % base)
        k //= base
        f /= base
    return out


def exponential_disk_stratified(n: int, Rd: float, M: float, z0: float) -> Particles:
    """Exponential disk with sech^2(z/z0) heights (razor thin for z0 = 0) from
    stratified mass fractions (i + 1/2) / n, golden-ratio azimuths and base-3
    van der Corput height fractions: the distribution of exponential_disk with
    far less sampling noise."""
    i = np.arange(n, dtype=np.float64)
    f = (i + 0.5) / n
    w = lambertw(-(1.0 - f) / np.e, k=-1).real
    R = Rd * (-1.0 - w)
    phi = 2.0 * np.pi * np.mod(i * 0.6180339887498949, 1.0)
    if z0 > 0.0:
        u = np.clip(_radical_inverse(np.arange(1, n + 1), 3), 1e-300, 1.0 - 1e-16)
        z = z0 * np.arctanh(2.0 * u - 1.0)
    else:
        z = np.zeros(n)
    return Particles(R * np.cos(phi), R * np.sin(phi), z, np.full(n, M / n))


def _exp_radii(rng: np.random.Generator, n: int, Rd: float) -> np.ndarray:
    u = rng.random(n)
    # 1 - (1 + x) e^-x = u  <=>  x = -1 - W_{-1}(-(1 - u)/e)
    w = lambertw(-(1.0 - u) / np.e, k=-1).real
    return Rd * (-1.0 - w)


def _sech2_heights(rng: np.random.Generator, n: int, z0: float) -> np.ndarray:
    if z0 <= 0.0:
        return np.zeros(n)
    u = rng.random(n)
    u = np.clip(u, 1e-300, 1.0 - 1e-16)
    return z0 * np.arctanh(2.0 * u - 1.0)


def exponential_disk(n: int, Rd: float, M: float, z0: float, rng: np.random.Generator) -> Particles:
    R = _exp_radii(rng, n, Rd)
    phi = 2.0 * np.pi * rng.random(n)
    z = _sech2_heights(rng, n, z0)
    return Particles(R * np.cos(phi), R * np.sin(phi), z, np.full(n, M / n))


def two_component_disk(n: int, seed: int, Md=5e10, Rd=3.0, zd=0.3, Mg=1e10, Rg=6.0, zg=0.15) -> Particles:
    """Stellar plus gas exponential disks, n//2 + (n - n//2) particles."""
    rng = _rng(seed)
    ns = n // 2
    s = exponential_disk(ns, Rd, Md, zd, rng)
    g = exponential_disk(n - ns, Rg, Mg, zg, rng)
    return Particles(np.concatenate([s.x, g.x]), np.concatenate([s.y, g.y]),
                     np.concatenate([s.z, g.z]), np.concatenate([s.m, g.m]))


@dataclass
class DiskParams:
    ml: float           # stellar mass-to-light ratio
    z_star: float       # kpc
    z_gas: float        # kpc
    dist: float         # distance factor
    n_particles: int
    n_grid: int
    seed: int

    def particles(self) -> Particles:
        # Distances scale lengths linearly and masses quadratically; scale heights stay.
        d = self.dist
        return two_component_disk(self.n_particles, self.seed, Md=self.ml * 5e10 * d * d, Rd=3.0 * d,
                                  zd=self.z_star, Mg=1e10 * d * d, Rg=6.0 * d, zg=self.z_gas)


def fit_grid(count: int = 64, config: int = 4, n_choices=(129, 257)) -> list:
    """Seeded Latin-hypercube draw of the batched rotation-curve fit parameters:
    M/L in [0.3, 1.2], z* in [0.1, 0.6], z_g in [0.05, 0.5], distance factor in
    [0.8, 1.2], particle count log-uniform in [2e5, 2e6], grid 129^3 or 257^3."""
    rng = _rng(seed_for(config))
    lo = np.array([0.3, 0.1, 0.05, 0.8, np.log(2e5)])
    hi = np.array([1.2, 0.6, 0.5, 1.2, np.log(2e6)])
    u = np.empty((count, 5))
    for d in range(5):
        u[:, d] = (rng.permutation(count) + rng.random(count)) / count
    v = lo + u * (hi - lo)
    grids = rng.choice(np.asarray(n_choices), size=count)
    out = []
    for r in range(count):
        out.append(DiskParams(ml=float(v[r, 0]), z_star=float(v[r, 1]), z_gas=float(v[r, 2]),
                              dist=float(v[r, 3]), n_particles=int(round(np.exp(v[r, 4]))),
                              n_grid=int(grids[r]), seed=seed_for(config, r + 1)))
    return out


# ------------------------------------------------ device-side realisations

def _exp_radii_torch(u, Rd):
    """Invert 1 - (1 + x) e^-x = u by safeguarded Newton steps (x = R/Rd)."""
    import torch
    lo = torch.zeros_like(u)
    hi = torch.full_like(u, 60.0)
    x = torch.sqrt(2.0 * u).clamp(max=50.0)
    for _ in range(40):
        F = 1.0 - (1.0 + x) * torch.exp(-x) - u
        lo = torch.where(F < 0, x, lo)
        hi = torch.where(F >= 0, x, hi)
        dF = x * torch.exp(-x)
        xn = x - F / torch.clamp(dF, min=1e-300)
        bad = (xn <= lo) | (xn >= hi) | ~torch.isfinite(xn)
        x = torch.where(bad, 0.5 * (lo + hi), xn)
    return Rd * x


def two_component_disk_torch(n, seed, Md=5e10, Rd=3.0, zd=0.3, Mg=1e10, Rg=6.0, zg=0.15, device="cuda"):
    """The two-component disk of two_component_disk, drawn on the GPU with
    torch's Philox generator (a different random stream, same distributions);
    returns (x, y, z, m) float64 device tensors."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    ns = n // 2
    parts = []
    for cnt, R0, M, z0 in ((ns, Rd, Md, zd), (n - ns, Rg, Mg, zg)):
        u = torch.rand(cnt, generator=gen, device=device, dtype=torch.float64)
        R = _exp_radii_torch(u, R0)
        phi = 2.0 * math.pi * torch.rand(cnt, generator=gen, device=device, dtype=torch.float64)
        w = torch.rand(cnt, generator=gen, device=device, dtype=torch.float64).clamp(1e-300, 1.0 - 1e-16)
        z = z0 * torch.atanh(2.0 * w - 1.0) if z0 > 0 else torch.zeros_like(w)
        parts.append((R * torch.cos(phi), R * torch.sin(phi), z, torch.full((cnt,), M / cnt, dtype=torch.float64,
                                                                           device=device)))
    return tuple(torch.cat([p[i] for p in parts]).contiguous() for i in range(4))

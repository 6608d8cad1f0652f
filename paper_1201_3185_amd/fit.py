"""Rotation-curve fitting on the batched solver (Sec. 4 of Angus et al.).

The paper fits each galaxy by an exhaustive search over four parameters --
distance D, stellar mass-to-light ratio M/L and the sech^2 scale heights of
the stellar and gas disks -- scoring every model by chi^2/n between its QUMOND
circular-speed curve and the observed one.  Here the galaxy is the synthetic
two-component disk (stars 5e10 Msun x M/L, R_d = 3 kpc; gas 1e10 Msun, R_g = 6
kpc; lengths scale with D, masses with D^2), the "observed" curve comes from a
realisation with known parameters and seeded Gaussian errors, and every batch
of parameter sets is one run of qumond_batch (one captured graph).

Distances enter as in the paper's figures: the observed radii are angular
radii placed at the model's distance, so a model at distance factor d is
compared at radii d R_obs (interpolated from a fine radial grid); speeds do
not depend on the distance.  Everything numerical that concerns the potential
runs in libqumond.so; this module draws particles (torch), marshals and
scores.
"""
from __future__ import annotations

import itertools
import time
from dataclasses import dataclass
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import qumond as Q
from . import synth


@dataclass(frozen=True)
class Params:
    dist: float     # distance factor (lengths x dist, masses x dist^2)
    ml: float       # stellar mass-to-light ratio
    z_star: float   # kpc
    z_gas: float    # kpc


def _disk(p: Params, n_particles: int, seed: int):
    d = p.dist
    return synth.two_component_disk_torch(n_particles, seed, Md=p.ml * 5e10 * d * d, Rd=3.0 * d, zd=p.z_star,
                                          Mg=1e10 * d * d, Rg=6.0 * d, zg=p.z_gas)


class CurveBatch:
    """QUMOND circular-speed curves of many parameter sets, 64 (or `size`) per
    run of one batch of single-box problems (n^3 grid, box_side kpc)."""

    def __init__(self, size: int = 64, n: int = 129, box_side: float = 120.0, r_max: float = 36.0, dr: float = 0.1,
                 n_particles: int = 500_000, refine_iters: int = 3, nu_n: float = 1.0, a0: float = 3600.0):
        """nu_n and a0 choose the MOND interpolating function (1: Eq. 2's nu,
        else the n-family) and acceleration constant of every model."""
        self.size = size
        self.n_particles = n_particles
        self.R = np.arange(dr, r_max + 0.5 * dr, dr)
        self.batch = Q.Batch(Q.BatchConfig(box_side=box_side, refine_iters=refine_iters, autotune=True, nu_n=nu_n,
                                           a0=a0), [n] * size, self.R)
        self.seconds = 0.0
        self.runs = 0

    def curves(self, params: Sequence[Params], seed: int = 1) -> np.ndarray:
        """v_c(R) [len(params), len(self.R)] in km/s (QUMOND, midplane).  Every
        model is drawn from the same random numbers (seed), so that the
        particles move smoothly with the parameters and chi^2 differences
        between models are not realisation noise."""
        out = np.empty((len(params), len(self.R)))
        for s in range(0, len(params), self.size):
            chunk = list(params[s:s + self.size])
            while len(chunk) < self.size:        # pad the last run with copies
                chunk.append(chunk[-1])
            t0 = time.perf_counter()
            for i, p in enumerate(chunk):
                x, y, z, m = _disk(p, self.n_particles, seed)
                self.batch.set_particles(i, x, y, z, m, float(m.sum().item()))
            self.batch.run(use_graph=True, allow_not_converged=True)
            vc2 = self.batch.rotation_curves(True).cpu().numpy()
            self.seconds += time.perf_counter() - t0
            self.runs += 1
            k = min(self.size, len(params) - s)
            out[s:s + k] = np.sqrt(np.maximum(vc2[:k], 0.0))
        return out

    def close(self):
        self.batch.close()


def observe(cb: CurveBatch, truth: Params, R_obs: np.ndarray, err_frac: float = 0.02, seed: int = 7,
            particle_seed: int = 424242) -> Tuple[np.ndarray, np.ndarray]:
    """A mock observed curve: the truth's QUMOND curve (its own realisation) at
    the angular radii R_obs (kpc at distance factor 1), with seeded Gaussian
    errors of err_frac times the speed; returns (v_obs, sigma_obs)."""
    v = cb.curves([truth], seed=particle_seed)[0]
    v_at = np.interp(truth.dist * R_obs, cb.R, v)
    sigma = err_frac * v_at
    rng = np.random.default_rng(seed)
    return v_at + sigma * rng.standard_normal(len(R_obs)), sigma


def chi2(cb: CurveBatch, params: Sequence[Params], R_obs: np.ndarray, v_obs: np.ndarray,
         sigma: np.ndarray) -> np.ndarray:
    """chi^2 / n of every parameter set against the observed curve."""
    v = cb.curves(params)
    out = np.empty(len(params))
    for i, p in enumerate(params):
        v_fit = np.interp(p.dist * R_obs, cb.R, v[i])
        out[i] = float(np.mean(((v_fit - v_obs) / sigma) ** 2))
    return out


def grid_search(cb: CurveBatch, axes: Dict[str, Sequence[float]], R_obs: np.ndarray, v_obs: np.ndarray,
                sigma: np.ndarray) -> Tuple[Params, float, List[Tuple[Params, float]]]:
    """Exhaustive search over the product of the axes (dist, ml, z_star, z_gas)."""
    grid = [Params(*v) for v in itertools.product(axes["dist"], axes["ml"], axes["z_star"], axes["z_gas"])]
    c = chi2(cb, grid, R_obs, v_obs, sigma)
    best = int(np.argmin(c))
    return grid[best], float(c[best]), list(zip(grid, c.tolist()))

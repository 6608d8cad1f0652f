"""Values the paper prints (tests/golden/paper_values.json, each entry cited) against
the oracle's constants, defaults and closed forms (CPU only)."""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle import analytic as A

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_a0_and_nu():
    assert O.A0_KPC == pytest.approx(GOLD["a0_kms2_per_pc"]["value"] * 1000.0)
    y = np.array([0.01, 0.5, 2.0, 40.0])
    assert np.allclose(O.nu(y), eval(GOLD["nu_form"]["value"], {"sqrt": np.sqrt, "y": y}), rtol=1e-15)


def test_oracle_defaults_follow_the_paper():
    cfg = O.OracleConfig(n=65, box_side=[100.0])
    assert cfg.npre == GOLD["pre_smoothing_sweeps"]["value"]
    assert cfg.npost == GOLD["post_smoothing_sweeps"]["value"]
    assert cfg.ncycle_fmg == GOLD["vcycles_per_level"]["value"]
    assert cfg.n in GOLD["grid_points_per_side"]["value"]
    # box choice: the paper's radii are one fifth of the box side
    for R, Lb in GOLD["box_choice_kpc"]["value"]:
        assert R == pytest.approx(cfg.gather_frac * Lb)


def test_paper_nesting_span():
    f = GOLD["box_halving"]["value"] ** GOLD["max_refinements"]["value"]
    assert 1.0 / f == GOLD["outer_box_factor"]["value"]
    assert GOLD["largest_box_kpc"]["value"] / GOLD["outer_box_factor"]["value"] == pytest.approx(
        GOLD["finest_box_kpc"]["value"], rel=0.03)


def test_kuzmin_mass_fraction_statement():
    g = GOLD["kuzmin_a1"]
    frac = 1.0 - A.kuzmin_enclosed(30.0, g["a_kpc"], g["M_msun"]) / g["M_msun"]
    assert frac == pytest.approx(GOLD["kuzmin_mass_beyond_30kpc_a1p5"]["value"], abs=0.001)


def test_coarsest_grid_centre_proportional_to_density():
    n = GOLD["coarsest_grid"]["value"]
    L = 4000.0
    vals = []
    for rho in (1.0, 2.0, 5.0):
        f = np.zeros((n,) * 3); f[1, 1, 1] = 4 * np.pi * O.G_KPC * rho
        u = np.zeros((n,) * 3)
        O.fmg(f, u, L, tol=0)
        vals.append(u[1, 1, 1] / rho)
    assert np.allclose(vals, vals[0], rtol=1e-15) and vals[0] < 0

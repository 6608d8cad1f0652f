"""Pins of the oracle's pointwise pieces and of the input samplers (CPU only).

nu(y) of Eq. 2 is pinned by the identity it must satisfy with the "simple"
mu-function the paper says it is the analogue of (mu(x) = x/(1+x), so
y = x mu(x) and nu(y) = 1/mu(x)); the point-mass QUMOND potential used as
the outer Dirichlet value is pinned by differentiating it numerically; the
Kuzmin fields (Sec. 3.1) by differentiation and quadrature; the samplers by
Kolmogorov-Smirnov tests against the enclosed-mass profiles.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle as O
from oracle import analytic as A
from paper_1201_3185_amd import synth


def test_nu_is_inverse_of_simple_mu():
    x = np.logspace(-4, 4, 81)
    y = x * x / (1.0 + x)            # y = x mu(x)
    assert np.allclose(O.nu(y), (1.0 + x) / x, rtol=1e-12, atol=0)


def test_nu_limits():
    assert O.nu(4.0 / 3.0) == pytest.approx(1.5, rel=1e-15)
    assert O.nu(1e12) == pytest.approx(1.0, rel=1e-11)
    y = 1e-10                        # deep MOND: nu ~ 1/sqrt(y)
    assert O.nu(y) * math.sqrt(y) == pytest.approx(1.0, rel=1e-4)


def test_units_a0():
    # Eq. 2: a0 = 3.6 (km/s)^2 / pc = 3600 (km/s)^2 / kpc (about 1.17e-10 m/s^2).
    assert O.A0_KPC == 3600.0
    si = O.A0_KPC * 1e6 / 3.0856775814913673e19
    assert si == pytest.approx(1.1667e-10, rel=1e-3)


def test_fixed_shift_rule():
    assert O.fixed_shift(1e10) == 27          # ceil(log2 1e10) = 34
    assert O.fixed_shift(2.0 ** 33) == 28     # exact power of two: ceil(log2) = 33
    assert O.fixed_shift(2.0 ** 33 + 1.0) == 27
    for M in (1.0, 3.7e9, 6e10, 1e12):
        s = O.fixed_shift(M)
        assert M * 2.0 ** s < 2.0 ** 62 and M * 2.0 ** (s + 1) >= 2.0 ** 61 * 0.999


@pytest.mark.parametrize("M", [1e9, 6e10])
def test_point_mond_potential_derivative(M):
    G, a0 = O.G_KPC, O.A0_KPC
    r = np.array([0.05, 0.5, 3.0, 30.0, 300.0])
    d = 1e-5 * r
    dphi = (O.phi_point_mond(r + d, G, M, a0) - O.phi_point_mond(r - d, G, M, a0)) / (2 * d)
    gN = G * M / r ** 2
    assert np.allclose(dphi, A.nu_closed(gN / a0) * gN, rtol=1e-7)


def test_point_mond_potential_limits():
    G, M = O.G_KPC, 1e10
    # a0 = 0 reduces to Newton; small r tends to -GM/r.
    r = np.array([0.1, 1.0, 10.0])
    assert np.allclose(O.phi_point_mond(r, G, M, 0.0), -G * M / r, rtol=1e-14)
    assert O.phi_point_mond(1e-6, G, M, O.A0_KPC) / (-G * M / 1e-6) == pytest.approx(1.0, rel=1e-5)
    # large r: logarithmic, slope sqrt(G M a0) / r
    r1, r2 = 1e5, 2e5
    slope = (O.phi_point_mond(r2, G, M, O.A0_KPC) - O.phi_point_mond(r1, G, M, O.A0_KPC)) / math.log(2.0)
    assert slope == pytest.approx(math.sqrt(G * M * O.A0_KPC), rel=1e-3)
    assert np.allclose(O.phi_point_mond(r, G, M, O.A0_KPC), A.phi_point_mond_closed(r, G, M, O.A0_KPC), rtol=1e-14)


def test_kuzmin_fields_consistent():
    a, M, G = 1.5, 1e10, O.G_KPC
    rng = np.random.default_rng(0)
    P = rng.uniform(-10, 10, (20, 3))
    P[:, 2] = np.where(np.abs(P[:, 2]) < 0.5, 0.7, P[:, 2])  # away from the plane's kink
    e = 1e-5
    for p in P:
        g = np.array(A.kuzmin_g_newton(*p, a, M, G))
        grad = np.zeros(3)
        for d in range(3):
            dp = np.zeros(3); dp[d] = e
            grad[d] = (A.kuzmin_phi_newton(*(p + dp), a, M, G) - A.kuzmin_phi_newton(*(p - dp), a, M, G)) / (2 * e)
        assert np.allclose(g, -grad, rtol=1e-6)
        gm = np.array(A.kuzmin_g_mond(*p, a, M, G))
        for d in range(3):
            dp = np.zeros(3); dp[d] = e
            grad[d] = (A.kuzmin_phi_mond(*(p + dp), a, M) - A.kuzmin_phi_mond(*(p - dp), a, M)) / (2 * e)
        assert np.allclose(gm, -grad, rtol=1e-6)
    # Midplane v_c^2 formulas agree with R |g_R| of the vector fields.
    R = np.array([0.5, 2.0, 8.0, 30.0])
    gx, _, _ = A.kuzmin_g_newton(R, 0 * R, 0 * R, a, M, G)
    assert np.allclose(-R * gx, A.kuzmin_vc2_newton(R, a, M, G), rtol=1e-13)
    gx, _, _ = A.kuzmin_g_mond(R, 0 * R, 0 * R, a, M, G)
    assert np.allclose(-R * gx, A.kuzmin_vc2_mond(R, a, M, G), rtol=1e-13)


def test_kuzmin_surface_density_integrates_to_enclosed_mass():
    a, M = 3.0, 1e10
    for R in (1.0, 5.0, 40.0):
        val, _ = integrate.quad(lambda s: 2 * np.pi * s * A.kuzmin_sigma(s, a, M), 0, R)
        assert val == pytest.approx(A.kuzmin_enclosed(R, a, M), rel=1e-10)
    # The Newtonian field jumps by 4 pi G Sigma across the plane (Gauss).
    R = 2.0
    _, _, gz_up = A.kuzmin_g_newton(R, 0.0, 1e-9, a, M)
    _, _, gz_dn = A.kuzmin_g_newton(R, 0.0, -1e-9, a, M)
    assert (gz_dn - gz_up) == pytest.approx(4 * np.pi * O.G_KPC * A.kuzmin_sigma(R, a, M), rel=1e-6)


def test_kuzmin_sampler_ks():
    a, M = 3.0, 1e10
    p = synth.kuzmin_disk(20000, a, M, 7)
    R = np.hypot(p.x, p.y)
    ks = stats.kstest(R, lambda r: A.kuzmin_enclosed(r, a, M) / M)
    assert ks.pvalue > 1e-3
    assert np.all(p.z == 0) and p.total_mass == pytest.approx(M, rel=1e-12)
    phi = np.arctan2(p.y, p.x)
    assert stats.kstest((phi + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3


def test_exponential_sech2_sampler_ks():
    rng = np.random.Generator(np.random.PCG64(3))
    Rd, z0, M = 3.0, 0.3, 5e10
    p = synth.exponential_disk(20000, Rd, M, z0, rng)
    R = np.hypot(p.x, p.y)
    assert stats.kstest(R, lambda r: A.exp_enclosed(r, Rd, M) / M).pvalue > 1e-3
    assert stats.kstest(p.z, lambda z: 0.5 * (1 + np.tanh(z / z0))).pvalue > 1e-3


def test_two_component_split():
    p = synth.two_component_disk(10001, 11)
    ms = np.unique(p.m)
    assert len(ms) == 2
    assert p.m[: 10001 // 2].sum() == pytest.approx(5e10, rel=1e-12)
    assert p.m[10001 // 2:].sum() == pytest.approx(1e10, rel=1e-12)


def test_fit_grid_ranges():
    g = synth.fit_grid()
    assert len(g) == 64
    ml = np.array([d.ml for d in g]); zs = np.array([d.z_star for d in g])
    zg = np.array([d.z_gas for d in g]); ds = np.array([d.dist for d in g])
    npart = np.array([d.n_particles for d in g]); ng = np.array([d.n_grid for d in g])
    assert ml.min() >= 0.3 and ml.max() <= 1.2 and zs.min() >= 0.1 and zs.max() <= 0.6
    assert zg.min() >= 0.05 and zg.max() <= 0.5 and ds.min() >= 0.8 and ds.max() <= 1.2
    assert npart.min() >= 2e5 * 0.999 and npart.max() <= 2e6 * 1.001
    assert set(ng.tolist()) == {129, 257}
    # Latin hypercube: every 1/64 stratum of each parameter holds exactly one draw.
    assert len(set(np.floor((ml - 0.3) / 0.9 * 64).astype(int).tolist())) == 64

"""Pins of the oracle's diagnostics (CPU only): the algebraic MOND relation of
Eq. 3 and the vertical velocity dispersion of Eq. 5.

* Eq. 3 on a point mass must give the radial derivative of the closed-form
  point-mass QUMOND potential (differentiated numerically here), reach the
  deep-MOND speed (G M a0)^(1/4) far out, keep the direction of g_N and
  reduce to g_N for a0 = 0; on the Kuzmin disk just above the plane it must
  give the midplane formula of Sec. 3.1, nu(|g_N,r| / a0) g_N,R.
* Eq. 5 for a sech^2(z/z0) disk: on a potential quadratic in z the gather is
  exact, so sigma^2 = k z z0 / (2 tanh(z/z0)) to rounding; on the potential of
  Spitzer's self-gravitating isothermal sheet, Phi = 2 pi G Sigma z0 ln cosh(z/z0),
  sigma^2 must be pi G Sigma z0 at every height (the textbook isothermal
  result); on the sampled Kuzmin potential it must converge at second order
  to the value from the closed-form vertical field.
"""
import numpy as np
import pytest

import oracle as O
from oracle import analytic as A
from tests.conftest import node_coords


def _point_field(x, y, z, M):
    r = np.sqrt(x * x + y * y + z * z)
    g = O.G_KPC * M / (r * r)
    return -g * x / r, -g * y / r, -g * z / r


def test_algebraic_point_mass_matches_potential_derivative():
    M = 3e10
    rng = np.random.default_rng(5)
    P = rng.normal(size=(40, 3)) * 20.0
    r = np.linalg.norm(P, axis=1)
    ax, ay, az = O.algebraic_field(*_point_field(P[:, 0], P[:, 1], P[:, 2], M))
    g = np.sqrt(ax * ax + ay * ay + az * az)
    # fourth-order central difference of the closed-form potential
    d = 1e-3 * r
    phi = lambda s: A.phi_point_mond_closed(s, O.G_KPC, M, O.A0_KPC)
    dphi = (-phi(r + 2 * d) + 8 * phi(r + d) - 8 * phi(r - d) + phi(r - 2 * d)) / (12 * d)
    assert np.allclose(g, dphi, rtol=1e-9)
    # direction unchanged: g parallel to -x
    assert np.allclose(ax * P[:, 1], ay * P[:, 0], rtol=1e-12, atol=1e-20)
    assert np.all(ax * P[:, 0] + ay * P[:, 1] + az * P[:, 2] < 0)


def test_algebraic_limits():
    M = 1e10
    x = np.array([1e6])
    ax, ay, az = O.algebraic_field(*_point_field(x, np.zeros(1), np.zeros(1), M))
    v2 = -ax[0] * x[0]
    assert v2 == pytest.approx((O.G_KPC * M * O.A0_KPC) ** 0.5, rel=1e-3)
    g = _point_field(np.array([2.0, 0.0]), np.array([0.0, 3.0]), np.array([1.0, -1.0]), M)
    out = O.algebraic_field(*g, a0=0.0)
    assert np.array_equal(np.stack(out), np.stack(g))
    zero = O.algebraic_field(np.zeros(3), np.zeros(3), np.zeros(3))
    assert np.all(np.stack(zero) == 0.0)


def test_algebraic_on_kuzmin_is_the_midplane_formula():
    a, M = 1.5, 1e10
    R = np.geomspace(0.1, 50.0, 30)
    eps = 1e-9
    gx, gy, gz = A.kuzmin_g_newton(R, np.zeros_like(R), np.full_like(R, eps), a, M)
    ax, _, _ = O.algebraic_field(gx, gy, gz)
    gr = O.G_KPC * M / (R * R + a * a)                       # |g_N,r| of Sec. 3.1
    gR = O.G_KPC * M * R * (R * R + a * a) ** -1.5           # |g_N,R| of Sec. 3.1
    expect = (0.5 + 0.5 * np.sqrt(1.0 + 4.0 * O.A0_KPC / gr)) * gR
    assert np.allclose(-ax, expect, rtol=1e-7)


def _sigma(phi, L, R, z, z0, naz=8, frac=0.45):
    x, y, zs = O.sigma_z_points(R, z, naz)
    _, _, az, used = O.gather([phi], [L], x, y, zs, frac=frac, mond=False)
    assert np.all(used == 0)
    return O.sigma_z2_from_az(zs, az, z0, len(R), naz)


def test_sigma_z_points_layout():
    x, y, zs = O.sigma_z_points(np.array([1.0, 2.0]), 0.3, naz=4)
    assert x.shape == (16,)
    assert np.allclose(zs.reshape(2, 8), [[0.3] * 4 + [-0.3] * 4] * 2)
    assert np.allclose(np.hypot(x, y).reshape(2, 8), [[1.0] * 8, [2.0] * 8])


def test_sigma_z_quadratic_potential_exact():
    n, L = 17, 8.0
    X, Y, Z = node_coords(n, L)
    k = 250.0
    phi = 0.5 * k * Z * Z + 3.0 * X - 1.0 * Y
    R = np.array([0.3, 1.1, 2.0])
    z0 = 0.4
    for z in (0.05, 0.4, 1.3):
        s2 = _sigma(phi, L, R, z, z0)
        assert np.allclose(s2, k * z * z0 / (2.0 * np.tanh(z / z0)), rtol=1e-12)
    # the z -> 0 limit of Eq. 5 for this profile: k z0^2 / 2
    s2 = _sigma(phi, L, R, 1e-6, z0)
    assert np.allclose(s2, 0.5 * k * z0 * z0, rtol=1e-10)


@pytest.mark.parametrize("z", [0.15, 0.5, 1.2])
def test_sigma_z_isothermal_sheet(z):
    Sigma, z0 = 5e7, 0.5                          # Msun / kpc^2, kpc
    spitzer = np.pi * O.G_KPC * Sigma * z0
    errs = []
    for n in (65, 129):
        L = 6.0
        X, Y, Z = node_coords(n, L)
        phi = 2.0 * np.pi * O.G_KPC * Sigma * z0 * np.log(np.cosh(Z / z0))
        s2 = _sigma(phi, L, np.array([0.2, 0.7]), z, z0)
        errs.append(np.max(np.abs(s2 / spitzer - 1.0)))
    assert errs[1] < 5e-3
    assert errs[0] / errs[1] > 3.0                # second order in the grid spacing


def test_sigma_z_kuzmin_second_order():
    a, M, z, z0 = 1.5, 1e10, 0.9, 0.3
    R = np.array([0.5, 1.5, 3.0])
    dphidz = O.G_KPC * M * (a + z) * (R * R + (a + z) ** 2) ** -1.5
    exact = dphidz * z0 / (2.0 * np.tanh(z / z0))
    errs = []
    for n in (33, 65):
        L = 16.0
        X, Y, Z = node_coords(n, L)
        phi = A.kuzmin_phi_newton(X, Y, Z, a, M)
        errs.append(np.max(np.abs(_sigma(phi, L, R, z, z0, frac=0.4) / exact - 1.0)))
    assert errs[1] < 0.02
    assert errs[0] / errs[1] > 3.0


# ------------------------------------------------------------ other nu forms

@pytest.mark.parametrize("nn", [1.0, 2.0, 3.0])
def test_nu_family_inverts_its_mu(nn):
    # the n-family is the inverse of mu_n(x) = x / (1 + x^n)^(1/n): y = x mu_n(x) <=> nu_n(y) = 1 / mu_n(x)
    x = np.logspace(-4, 4, 61)
    y = x * x / (1.0 + x ** nn) ** (1.0 / nn)
    assert np.allclose(O.nu(y, nn), (1.0 + x ** nn) ** (1.0 / nn) / x, rtol=1e-11, atol=0)


def test_nu_family_n1_is_eq2_nu():
    y = np.logspace(-6, 6, 25)
    assert np.array_equal(O.nu(y, 1.0), O.nu(y))
    assert np.allclose(np.vectorize(lambda v: O.lib().orc_nu_n(v, 1.0))(y), O.nu(y), rtol=0, atol=0)


def test_point_potential_family_n1_is_closed_form():
    r = np.geomspace(0.05, 5000.0, 23)
    for M in (1e6, 1e10, 3e11):
        closed = A.phi_point_mond_closed(r, O.G_KPC, M, O.A0_KPC)
        assert np.allclose(O.phi_point_mond_family(r, O.G_KPC, M, O.A0_KPC, 1.0), closed, rtol=1e-12)


@pytest.mark.parametrize("nn", [2.0, 4.0])
def test_point_potential_family_derivative_and_limits(nn):
    G, M, a0 = O.G_KPC, 2e10, O.A0_KPC
    r = np.array([0.3, 2.0, 4.7, 20.0, 300.0])
    d = 1e-3 * r
    phi = lambda s: O.phi_point_mond_family(s, G, M, a0, nn)
    dphi = (-phi(r + 2 * d) + 8 * phi(r + d) - 8 * phi(r - d) + phi(r - 2 * d)) / (12 * d)
    gN = G * M / (r * r)
    assert np.allclose(dphi, O.nu(gN / a0, nn) * gN, rtol=1e-8)
    # -GM/r at small r, logarithmic with slope sqrt(G M a0) far out
    assert phi(np.array([1e-4]))[0] == pytest.approx(-G * M / 1e-4, rel=1e-6)
    far = phi(np.array([1e5, 1e6]))
    assert (far[1] - far[0]) / np.log(10.0) == pytest.approx(np.sqrt(G * M * a0), rel=1e-4)


def test_source_family_converges_at_second_order():
    G, M, b, nn = O.G_KPC, 1e10, 2.0, 2.0
    L = 20.0
    c0 = np.array([0.11, -0.07, 0.05])

    def div(rr):                     # analytic (1/r^2) d/dr [r^2 nu_2(g/a0) g] for the Plummer Phi_N
        def flux(q):
            g = G * M * q / (q * q + b * b) ** 1.5
            nu2 = np.sqrt(0.5 * (1.0 + np.sqrt(1.0 + 4.0 * (O.A0_KPC / g) ** 2)))
            return q * q * nu2 * g
        d = 1e-4 * rr
        return (flux(rr + d) - flux(rr - d)) / (2 * d) / (rr * rr)

    errs = []
    for n in (33, 65):
        X, Y, Z = node_coords(n, L)
        r = np.sqrt((X - c0[0]) ** 2 + (Y - c0[1]) ** 2 + (Z - c0[2]) ** 2)
        S = O.mond_source(-G * M / np.sqrt(r * r + b * b), L, nu_n=nn)
        shell = (r > 3.0) & (r < 7.0)
        ex = div(r[shell])
        errs.append(np.abs(S[shell] - ex).max() / np.abs(ex).max())
    assert errs[0] < 0.05
    assert 3.3 < errs[0] / errs[1] < 4.7


def test_bc_outer_family_values():
    n, L, M = 9, 40.0, 5e10
    u = np.zeros((n,) * 3)
    O.bc_outer(u, L, 2, M=M, nu_n=2.0)
    X, Y, Z = node_coords(n, L)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    bmask = np.zeros_like(u, dtype=bool)
    bmask[0], bmask[-1], bmask[:, 0], bmask[:, -1], bmask[:, :, 0], bmask[:, :, -1] = (True,) * 6
    ref = O.phi_point_mond_family(r[bmask], O.G_KPC, M, O.A0_KPC, 2.0)
    assert np.allclose(u[bmask], ref, rtol=1e-14)
    assert np.all(u[~bmask] == 0)
    # n = 1 through the same call is the closed form of the C oracle
    u1 = np.zeros((n,) * 3)
    O.bc_outer(u1, L, 2, M=M, nu_n=1.0)
    assert np.allclose(u1[bmask], A.phi_point_mond_closed(r[bmask], O.G_KPC, M, O.A0_KPC), rtol=1e-13)

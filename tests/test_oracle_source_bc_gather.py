"""Pins of the oracle's Eq. 2 source, nested-box boundary values and force gather (CPU only).

* Source: with a0 = 0, nu is exactly 1 in IEEE arithmetic, so the face-flux
  divergence must equal the 7-point Laplacian of Phi_N; a uniform field has
  zero divergence; for a smooth spherical potential the discrete source
  converges at second order to the analytic div[nu grad Phi_N].
* Boundary interpolation from the coarser box (Sec. 2, nested refinement):
  exact for linear fields, second order for smooth ones.
* Gather: finite differences plus CIC weights reproduce a linear potential's
  field exactly; the box choice follows the R < L/5 rule of Sec. 3.1; points
  outside every box get the monopole field.
"""
import numpy as np
import pytest

import oracle as O
from tests.conftest import interior, node_coords


def laplacian(u, h):
    return -O.residual(np.zeros_like(u), u, h)


def test_source_with_a0_zero_is_the_laplacian():
    n, L = 17, 8.0
    h = L / (n - 1)
    X, Y, Z = node_coords(n, L)
    phin = -O.G_KPC * 1e10 / np.sqrt((X - 0.3) ** 2 + (Y + 0.2) ** 2 + (Z - 0.1) ** 2 + 1.0)
    S = O.mond_source(phin, L, a0=0.0)
    lap = laplacian(phin, h)
    assert np.abs(S - lap).max() <= 1e-12 * np.abs(lap).max()
    assert np.all(S[0] == 0) and np.all(S[:, -1] == 0)


def test_source_of_uniform_field_vanishes():
    n, L = 17, 8.0
    h = L / (n - 1)
    X, Y, Z = node_coords(n, L)
    g0 = np.array([120.0, -40.0, 75.0])
    phin = g0[0] * X + g0[1] * Y + g0[2] * Z
    S = O.mond_source(phin, L)
    flux = O.nu(np.linalg.norm(g0) / O.A0_KPC) * np.linalg.norm(g0)
    assert np.abs(interior(S)).max() < 1e-11 * flux / h


def _plummer_div(r, G, M, b, a0):
    """Analytic div[nu(|g|/a0) grad Phi_N] for Phi_N = -GM/sqrt(r^2+b^2)."""
    def flux(rr):
        g = G * M * rr / (rr * rr + b * b) ** 1.5
        return rr * rr * (0.5 + 0.5 * np.sqrt(1.0 + 4.0 * a0 / g)) * g
    d = 1e-4 * r
    return (flux(r + d) - flux(r - d)) / (2 * d) / (r * r)


def test_source_converges_at_second_order():
    G, M, b = O.G_KPC, 1e10, 2.0
    L = 20.0
    c0 = np.array([0.11, -0.07, 0.05])
    errs = []
    for n in (33, 65, 129):
        X, Y, Z = node_coords(n, L)
        r = np.sqrt((X - c0[0]) ** 2 + (Y - c0[1]) ** 2 + (Z - c0[2]) ** 2)
        S = O.mond_source(-G * M / np.sqrt(r * r + b * b), L)
        shell = (r > 3.0) & (r < 7.0)
        ex = _plummer_div(r[shell], G, M, b, O.A0_KPC)
        errs.append(np.abs(S[shell] - ex).max() / np.abs(ex).max())
    assert errs[0] < 0.05
    assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7


def test_bc_from_coarse_linear_exact_and_smooth_second_order():
    n, Lc = 17, 16.0
    Lf = Lc / 2
    Xc, Yc, Zc = node_coords(n, Lc)
    Xf, Yf, Zf = node_coords(n, Lf)
    lin = lambda X, Y, Z: 3.0 - X + 2 * Y + 0.25 * Z
    uf = np.zeros((n,) * 3)
    O.bc_from_coarse(lin(Xc, Yc, Zc), Lc, uf, Lf)
    bmask = np.ones((n,) * 3, bool); bmask[1:-1, 1:-1, 1:-1] = False
    assert np.abs(uf[bmask] - lin(Xf, Yf, Zf)[bmask]).max() < 1e-13
    assert np.all(interior(uf) == 0)
    errs = []
    for n in (17, 33, 65):
        Xc, Yc, Zc = node_coords(n, Lc)
        Xf, Yf, Zf = node_coords(n, Lf)
        pl = lambda X, Y, Z: -1.0 / np.sqrt(X * X + Y * Y + Z * Z + 9.0)
        uf = np.zeros((n,) * 3)
        O.bc_from_coarse(pl(Xc, Yc, Zc), Lc, uf, Lf)
        bmask = np.ones((n,) * 3, bool); bmask[1:-1, 1:-1, 1:-1] = False
        errs.append(np.abs(uf[bmask] - pl(Xf, Yf, Zf)[bmask]).max())
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_outer_bc_modes():
    n, L, M = 9, 40.0, 3e10
    u = np.full((n,) * 3, 5.0)
    O.bc_outer(u, L, 1, M=M)
    X, Y, Z = node_coords(n, L)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    bmask = np.ones((n,) * 3, bool); bmask[1:-1, 1:-1, 1:-1] = False
    assert np.allclose(u[bmask], -O.G_KPC * M / r[bmask], rtol=1e-15)
    assert np.all(interior(u) == 5.0)
    O.bc_outer(u, L, 2, M=M)
    from oracle.analytic import phi_point_mond_closed
    assert np.allclose(u[bmask], phi_point_mond_closed(r[bmask], O.G_KPC, M, O.A0_KPC), rtol=1e-13)
    O.bc_outer(u, L, 0)
    assert np.all(u[bmask] == 0)


def test_gather_linear_field_exact_everywhere():
    n, L = 17, 10.0
    X, Y, Z = node_coords(n, L)
    g = np.array([3.0, -2.0, 0.5])
    phi = -(g[0] * X + g[1] * Y + g[2] * Z) + 7.0
    rng = np.random.default_rng(0)
    P = rng.uniform(-4.99, 4.99, (300, 3))
    P[:5] = [[-5.0, 0, 0], [4.999999, 4.999999, -5.0], [0, 0, 0], [1.0, 1.0, 1.0], [-4.9, 3.3, 4.99]]
    ax, ay, az, used = O.gather([phi], [L], P[:, 0], P[:, 1], P[:, 2], frac=0.2)
    assert np.all(used == 0)
    assert np.allclose(ax, g[0], atol=1e-12) and np.allclose(ay, g[1], atol=1e-12)
    assert np.allclose(az, g[2], atol=1e-12)


def test_gather_quadratic_field_exact_on_nodes():
    n, L = 9, 8.0
    h = L / (n - 1)
    X, Y, Z = node_coords(n, L)
    phi = X * X - 2 * Y * Z + 0.5 * Z * Z
    pts = np.array([[-4, -4, -4], [4 - 1e-12, 0, 0], [-4 + h, 2 * h, -4], [1.0, -2.0, 3.0]], float)
    ax, ay, az, _ = O.gather([phi], [L], pts[:, 0], pts[:, 1], pts[:, 2], frac=0.45)
    x, y, z = pts.T
    assert np.allclose(ax, -2 * x, atol=1e-9)
    assert np.allclose(ay, 2 * z, atol=1e-9)
    assert np.allclose(az, 2 * y - z, atol=1e-9)


def test_gather_box_choice_and_monopole():
    n = 9
    Ls = [400.0, 200.0, 100.0, 50.0]
    phis = [np.zeros((n,) * 3) for _ in Ls]
    pts = np.array([
        [5.0, 0, 0],        # R < 10: finest box 3
        [15.0, 0, 0],       # R < 20: box 2
        [5.0, 0, 15.0],     # |z| >= 10 fails box 3 -> box 2
        [70.0, 0, 0],       # box 0 (R < 80)
        [85.0, 0, 0],       # no margin anywhere; outermost containing -> 0
        [300.0, 0, 0],      # outside every box: monopole
    ])
    M = 2e10
    ax, ay, az, used = O.gather(phis, Ls, pts[:, 0], pts[:, 1], pts[:, 2], M=M, mond=False)
    assert used.tolist() == [3, 2, 2, 0, 0, 255]
    assert ax[5] == pytest.approx(-O.G_KPC * M / 300.0 ** 2, rel=1e-14)
    ax, ay, az, used = O.gather(phis, Ls, pts[:, 0], pts[:, 1], pts[:, 2], M=M, mond=True)
    gN = O.G_KPC * M / 300.0 ** 2
    assert ax[5] == pytest.approx(-O.nu(gN / O.A0_KPC) * gN, rel=1e-14)

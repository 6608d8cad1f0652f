"""Pins of the oracle's multigrid (Sec. 2: FMG with red-black Gauss-Seidel), CPU only.

Each piece is tied to a property fixed by mathematics rather than by the
oracle's own formulas: Gauss-Seidel leaves zero residual on the colour it
just updated; the 7-point operator is exact on quadratics; full weighting
preserves constants and linear fields and is 1/8 times the adjoint of
trilinear prolongation; prolongation reproduces trilinear fields; the 3^3
grid with zero boundary gives centre value -h^2 f / 6 (Sec. 2: the centre
potential is proportional to the centre density).  The converged FMG is then
compared with the exact discrete solution from a type-I sine transform and
from a dense linear solve.
"""
import numpy as np
import pytest
from scipy.fft import dstn

import oracle as O
from tests.conftest import interior, node_coords


def _rand_problem(n, L, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, n, n))
    u = np.zeros((n, n, n))
    b = rng.standard_normal((n, n, n))
    mask = np.ones((n, n, n), bool)
    mask[1:-1, 1:-1, 1:-1] = False
    u[mask] = b[mask]
    return f, u


def _colour_mask(n, c):
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    m = ((i + j + k) % 2 == c)
    m[0, :, :] = m[-1, :, :] = m[:, 0, :] = m[:, -1, :] = m[:, :, 0] = m[:, :, -1] = False
    return m


def test_gauss_seidel_zeroes_residual_of_updated_colour():
    n, L = 17, 3.0
    h = L / (n - 1)
    f, u = _rand_problem(n, L, 0)
    u[1:-1, 1:-1, 1:-1] = np.random.default_rng(1).standard_normal((n - 2,) * 3)
    O.rbgs_colour(f, u, h, 0)
    r = O.residual(f, u, h)
    scale = np.abs(f).max()
    assert np.abs(r[_colour_mask(n, 0)]).max() < 1e-11 * scale
    assert np.abs(r[_colour_mask(n, 1)]).max() > 1e-3
    O.rbgs_colour(f, u, h, 1)
    r = O.residual(f, u, h)
    assert np.abs(r[_colour_mask(n, 1)]).max() < 1e-11
    # the sweep order is colour 0 then colour 1
    u2 = u.copy(); u3 = u.copy()
    O.rbgs_sweep(f, u2, h)
    O.rbgs_colour(f, u3, h, 0); O.rbgs_colour(f, u3, h, 1)
    assert np.array_equal(u2, u3)


def test_operator_exact_on_quadratics():
    n, L = 9, 2.0
    h = L / (n - 1)
    X, Y, Z = node_coords(n, L)
    u = X ** 2 + 2 * Y ** 2 + 3 * Z ** 2 + X * Y - 4 * Z + 1
    f = np.full((n, n, n), 12.0)     # Laplacian of u
    r = O.residual(f, u, h)
    assert np.abs(interior(r)).max() < 1e-11
    assert np.all(r[0] == 0) and np.all(r[:, :, -1] == 0)


def test_restriction_constants_linear_and_adjoint():
    nf = 17
    nc = 9
    c = O.restrict_fw(np.full((nf,) * 3, 2.5))
    assert np.allclose(interior(c), 2.5, rtol=1e-15) and np.all(c[0] == 0)
    Xf, Yf, Zf = node_coords(nf, 2.0)
    Xc, Yc, Zc = node_coords(nc, 2.0)
    lin = lambda X, Y, Z: 1.0 + 2 * X - 3 * Y + 0.5 * Z
    c = O.restrict_fw(lin(Xf, Yf, Zf))
    assert np.allclose(interior(c), interior(lin(Xc, Yc, Zc)), atol=1e-13)
    rng = np.random.default_rng(2)
    r = np.zeros((nf,) * 3); r[1:-1, 1:-1, 1:-1] = rng.standard_normal((nf - 2,) * 3)
    v = np.zeros((nc,) * 3); v[1:-1, 1:-1, 1:-1] = rng.standard_normal((nc - 2,) * 3)
    Pv = O.prolong_add(v, np.zeros((nf,) * 3))
    lhs = (O.restrict_fw(r) * v).sum()
    rhs = (r * Pv).sum() / 8.0
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_prolongation_reproduces_trilinear_fields():
    nc, nf = 5, 9
    Xc, Yc, Zc = node_coords(nc, 4.0)
    Xf, Yf, Zf = node_coords(nf, 4.0)
    tri = lambda X, Y, Z: 1 + X - 2 * Y + 3 * Z + X * Y - Y * Z + 0.5 * X * Y * Z
    uf = np.full((nf,) * 3, 7.0)
    O.interp(tri(Xc, Yc, Zc), uf)
    assert np.allclose(interior(uf), interior(tri(Xf, Yf, Zf)), atol=1e-13)
    assert np.all(uf[0] == 7.0)      # boundary untouched
    uc = np.random.default_rng(3).standard_normal((nc,) * 3)
    uf = O.prolong_add(uc, np.ones((nf,) * 3))
    assert np.allclose(uf[2:-2:2, 2:-2:2, 2:-2:2], 1 + uc[1:-1, 1:-1, 1:-1], rtol=1e-15)


def test_coarsest_grid_is_exact():
    n, L = 3, 6.0
    h = L / 2
    f = np.zeros((3, 3, 3)); f[1, 1, 1] = 0.7
    u = np.zeros((3, 3, 3))
    O.rbgs_sweep(f, u, h)
    assert u[1, 1, 1] == pytest.approx(-h * h * 0.7 / 6.0, rel=1e-15)
    st, rr, ex = O.fmg(f, np.zeros((3, 3, 3)), L, tol=1e-14)
    assert st == 0 and rr < 1e-14


def exact_discrete(f, u_bc, L):
    """Exact solution of the 7-point Dirichlet problem via the type-I DST."""
    n = f.shape[0]
    m = n - 2
    h = L / (n - 1)
    b = f[1:-1, 1:-1, 1:-1].copy()
    ub = u_bc.copy(); ub[1:-1, 1:-1, 1:-1] = 0.0
    nb = (ub[:-2, 1:-1, 1:-1] + ub[2:, 1:-1, 1:-1] + ub[1:-1, :-2, 1:-1] + ub[1:-1, 2:, 1:-1]
          + ub[1:-1, 1:-1, :-2] + ub[1:-1, 1:-1, 2:])
    b -= nb / h ** 2
    lam = (2 * np.cos(np.pi * np.arange(1, m + 1) / (m + 1)) - 2) / h ** 2
    den = lam[:, None, None] + lam[None, :, None] + lam[None, None, :]
    x = dstn(dstn(b, type=1, norm="ortho") / den, type=1, norm="ortho")
    out = u_bc.copy(); out[1:-1, 1:-1, 1:-1] = x
    return out


@pytest.mark.parametrize("n", [9, 17, 33, 65])
def test_fmg_matches_exact_discrete_solution(n):
    L = 10.0
    f, u = _rand_problem(n, L, n)
    ex = exact_discrete(f, u, L)
    st, rr, extra = O.fmg(f, u, L, tol=1e-13, max_extra=40)
    assert st == 0 and rr <= 1e-13
    assert np.abs(u - ex).max() <= 1e-12 * np.abs(ex).max()


@pytest.mark.parametrize("n", [5, 9])
def test_fmg_matches_dense_solve(n):
    L = 1.0
    h = L / (n - 1)
    f, u = _rand_problem(n, L, 100 + n)
    m = n - 2
    N = m ** 3
    A = np.zeros((N, N)); rhs = np.zeros(N)
    idx = lambda i, j, k: i + m * (j + m * k)
    for k in range(m):
        for j in range(m):
            for i in range(m):
                row = idx(i, j, k)
                A[row, row] = -6.0 / h ** 2
                rhs[row] = f[k + 1, j + 1, i + 1]
                for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    ii, jj, kk = i + di, j + dj, k + dk
                    if 0 <= ii < m and 0 <= jj < m and 0 <= kk < m:
                        A[row, idx(ii, jj, kk)] = 1.0 / h ** 2
                    else:
                        rhs[row] -= u[kk + 1, jj + 1, ii + 1] / h ** 2
    x = np.linalg.solve(A, rhs).reshape(m, m, m)
    O.fmg(f, u, L, tol=1e-14, max_extra=60)
    assert np.abs(interior(u) - x).max() <= 1e-12 * np.abs(x).max()


def test_vcycle_convergence_factor():
    n, L = 65, 1.0
    f, u = _rand_problem(n, L, 7)
    u[1:-1, 1:-1, 1:-1] = 0
    r0 = O.vcycles(f, u, L, 1)
    r1 = O.vcycles(f, u, L, 1)
    r2 = O.vcycles(f, u, L, 1)
    # V(2,2) red-black Gauss-Seidel for the 3D Poisson problem: textbook factor ~0.05-0.1
    assert r1 / r0 < 0.15 and r2 / r1 < 0.15


def test_fmg_error_tracks_discretisation_error():
    """FMG's defining property: after a fixed number of V-cycles per level the
    algebraic error is a fixed, h-independent fraction of the O(h^2)
    discretisation error (with trilinear FMG interpolation, about 3x after one
    cycle and well below it after two)."""
    L = 2.0
    ratio1, ratio2, errs = [], [], {}
    for n in (17, 33, 65):
        X, Y, Z = node_coords(n, L)
        k = np.pi / L
        s = np.sin(k * (X + 1)) * np.sin(k * (Y + 1)) * np.sin(k * (Z + 1))
        exact = s + X * Y
        f = -3 * k * k * s
        disc = exact_discrete(f, exact, L)
        e_disc = np.abs(disc - exact).max()
        for nc, store in ((1, ratio1), (2, ratio2)):
            u = exact.copy(); u[1:-1, 1:-1, 1:-1] = 0
            O.fmg(f, u, L, ncycle=nc, tol=0)
            store.append(np.abs(u - disc).max() / e_disc)
        errs[n] = e_disc
    assert max(ratio1) < 4.0 and max(ratio2) < 0.3
    assert max(ratio1) / min(ratio1) < 1.5
    assert 3.5 < errs[17] / errs[33] < 4.5 and 3.5 < errs[33] / errs[65] < 4.5


def test_source_free_box_solves_harmonic_field():
    """f = 0 with Dirichlet values from a harmonic quadratic: the 7-point scheme is
    exact on quadratics, so the converged solution is the field itself; the
    stopping test is then relative to the boundary-value contribution, whose norm
    equals that of the residual of the boundary-only field."""
    n, L = 33, 4.0
    h = L / (n - 1)
    X, Y, Z = node_coords(n, L)
    exact = X * X - Y * Y + 2 * X * Z - 3 * Y + 1.0
    u = exact.copy(); u[1:-1, 1:-1, 1:-1] = 0.0
    r0 = O.residual(np.zeros_like(u), u, h)
    bsum = O.lib().orc_boundary_coupling_sumsq(n, h, O._p(np.ascontiguousarray(u)))
    assert bsum == pytest.approx((interior(r0) ** 2).sum(), rel=1e-13)
    st, rr, extra = O.fmg(np.zeros_like(u), u, L, tol=1e-12, max_extra=40)
    assert st == 0 and rr <= 1e-12
    assert np.abs(u - exact).max() < 1e-11 * np.abs(exact).max()

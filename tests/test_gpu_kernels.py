"""Kernel-by-kernel parity of the gfx950 library against the FP64 oracle.

Each single-grid entry point of include/qumond_kernels.h is fed the same seeded
input as the oracle routine for the same step of Sec. 2, at sizes that span
one and several tiles with ragged tails (interior 3..255 points per side).
Tolerances: transfers with dyadic weights agree to rounding of the sums
(1e-15 of the field's scale); one Gauss-Seidel sweep, restriction and norms
to 1e-14..1e-13 (only the order of a handful of FP64 operations differs);
the face-flux source to 1e-12 of max|S| (a difference of fluxes).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1201_3185_amd import qumond as Q
from tests.conftest import node_coords

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def rand_state(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, n, n))
    u = rng.standard_normal((n, n, n))
    return f, u


SIZES = [5, 9, 17, 33, 65, 129, 257]


@pytest.mark.parametrize("n", SIZES)
def test_rbgs_sweep(n):
    L = 10.0
    h = L / (n - 1)
    f, u = rand_state(n, n)
    ref = u.copy()
    O.rbgs_sweep(f, ref, h)
    uin = dev(u)
    uout = dev(u)          # boundary preset
    Q.k_rbgs_sweep(dev(f), uin, uout, h)
    got = host(uout)
    assert rel(got, ref) < 1e-14
    assert np.array_equal(got[0], u[0]) and np.array_equal(got[:, :, -1], u[:, :, -1])


@pytest.mark.parametrize("n", [33, 129])
def test_rbgs_many_sweeps(n):
    L = 3.0
    h = L / (n - 1)
    f, u = rand_state(n, 100 + n)
    ref = u.copy()
    a, b = dev(u), dev(u)
    fd = dev(f)
    for s in range(6):
        O.rbgs_sweep(f, ref, h)
        Q.k_rbgs_sweep(fd, a, b, h)
        a, b = b, a
    assert rel(host(a), ref) < 1e-13


@pytest.mark.parametrize("n", SIZES)
def test_residual_restrict(n):
    L = 7.0
    h = L / (n - 1)
    f, u = rand_state(n, 200 + n)
    nc = (n + 1) // 2
    ref = O.restrict_fw(O.residual(f, u, h))
    fc = dev(np.full((nc,) * 3, 9.0))
    uc0 = dev(np.full((nc,) * 3, 9.0))
    uc1 = dev(np.full((nc,) * 3, 9.0))
    Q.k_residual_restrict(dev(f), dev(u), h, fc, uc0, uc1)
    assert rel(host(fc), ref) < 1e-13
    assert np.all(host(uc0) == 0)
    u1 = host(uc1)
    assert np.all(u1[0] == 0) and np.all(u1[-1] == 0) and np.all(u1[:, 0] == 0) and np.all(u1[:, :, -1] == 0)
    if nc > 2:
        assert np.all(u1[1:-1, 1:-1, 1:-1] == 9.0)


@pytest.mark.parametrize("n", [9, 17, 33, 65, 129, 257])
def test_residual_restrict_variants_bitwise(n):
    """The gather, LDS-tile (three tile sizes) and z-march (three chunk sizes;
    32x8 and 64x4 columns from coarse column 1 over the whole column, loading
    two to four steps ahead, 32x8 over 64-plane chunks) residual restrictions
    give the same bits."""
    L = 3.0
    h = L / (n - 1)
    f, u = rand_state(n, 400 + n)
    nc = (n + 1) // 2
    before = Q.tune_get_rr(n)
    outs = []
    try:
        for v in range(12):
            Q.tune_set_rr(n, v)
            fc, uc0, uc1 = (dev(np.full((nc,) * 3, 3.0)) for _ in range(3))
            Q.k_residual_restrict(dev(f), dev(u), h, fc, uc0, uc1)
            outs.append((host(fc), host(uc0), host(uc1)))
    finally:
        Q.tune_set_rr(n, before)
    for v in range(1, 12):
        for a, b in zip(outs[0], outs[v]):
            assert np.array_equal(a, b), v


def test_restrict_513():
    """At 513^3 the restriction of f gives the bits of the per-node gather of the
    residual restriction with a zero iterate (r = f exactly), and sampled coarse
    nodes equal the weighted sum written out in the same order."""
    n, nc = 513, 257
    g = torch.Generator(device="cuda")
    g.manual_seed(513)
    f = torch.randn((n,) * 3, dtype=torch.float64, device="cuda", generator=g)
    fc = torch.zeros((nc,) * 3, dtype=torch.float64, device="cuda")
    Q.k_restrict(f, fc)
    before = Q.tune_get_rr(n)
    try:
        Q.tune_set_rr(n, 0)
        u = torch.zeros_like(f)
        ref, c0 = (torch.zeros((nc,) * 3, dtype=torch.float64, device="cuda") for _ in range(2))
        Q.k_residual_restrict(f, u, 1.0, ref, c0)
        del u
    finally:
        Q.tune_set_rr(n, before)
    assert torch.equal(fc, ref)
    w = np.array([0.25, 0.5, 0.25])
    rng = np.random.default_rng(5)
    for _ in range(16):
        I, J, K = (int(x) for x in rng.integers(1, nc - 1, 3))
        blk = f[2 * K - 1:2 * K + 2, 2 * J - 1:2 * J + 2, 2 * I - 1:2 * I + 2].cpu().numpy()
        want = 0.0
        for c in range(3):
            for b in range(3):
                for a in range(3):
                    want += (w[a] * w[b] * w[c]) * blk[c, b, a]
        assert fc[K, J, I].item() == want
    assert torch.count_nonzero(fc[0]) == 0 and torch.count_nonzero(fc[:, :, -1]) == 0


@pytest.mark.parametrize("n", SIZES)
def test_restrict(n):
    src = rand_state(n, 300 + n)[0]
    nc = (n + 1) // 2
    dst = dev(np.full((nc,) * 3, 5.0))
    Q.k_restrict(dev(src), dst)
    assert rel(host(dst), O.restrict_fw(src)) < 1e-14


@pytest.mark.parametrize("nc", [3, 5, 9, 17, 33, 65, 129])
def test_prolong_add_and_interp(nc):
    nf = 2 * nc - 1
    rng = np.random.default_rng(nc)
    uc = rng.standard_normal((nc,) * 3)
    uf = rng.standard_normal((nf,) * 3)
    ref = O.prolong_add(uc, uf.copy())
    d = dev(uf)
    Q.k_prolong_add(dev(uc), d)
    assert rel(host(d), ref) < 1e-15
    ref = O.interp(uc, uf.copy())
    d = dev(uf)
    Q.k_interp(dev(uc), d)
    got = host(d)
    assert rel(got, ref) < 1e-15
    assert np.array_equal(got[0], uf[0])


@pytest.mark.parametrize("n", [5, 17, 33, 65, 129])
def test_mond_source(n):
    L = 20.0
    h = L / (n - 1)
    X, Y, Z = node_coords(n, L)
    r = np.sqrt((X - 0.3) ** 2 + (Y + 0.1) ** 2 + (Z - 0.05) ** 2)
    phin = -O.G_KPC * 3e10 / np.sqrt(r * r + 4.0)
    ref = O.mond_source(phin, L)
    S = dev(np.full((n,) * 3, 7.0))
    Q.k_mond_source(dev(phin), h, O.A0_KPC, S)
    got = host(S)
    assert rel(got, ref) < 1e-12
    assert np.all(got[0] == 0) and np.all(got[:, :, -1] == 0)
    # rough field (random) and the a0 = 0 special case
    rough = np.random.default_rng(n).standard_normal((n, n, n)) * 1e4
    rough[n // 2, :, :] = rough[n // 2, 0, 0]   # a plane with zero in-plane gradient components
    for a0 in (O.A0_KPC, 0.0):
        ref = O.mond_source(rough, L, a0=a0)
        Q.k_mond_source(dev(rough), h, a0, S)
        assert rel(host(S), ref) < 1e-12


def test_mond_source_zero_field_gives_zero_flux():
    n, L = 17, 4.0
    phin = np.full((n, n, n), -123.0)
    S = dev(np.full((n,) * 3, 7.0))
    Q.k_mond_source(dev(phin), L / (n - 1), O.A0_KPC, S)
    assert np.all(host(S) == 0.0)


@pytest.mark.parametrize("n", [5, 9, 33, 129])
def test_bc_from_coarse(n):
    Lc = 40.0
    Xc, Yc, Zc = node_coords(n, Lc)
    uc = np.sin(Xc / 7) * np.cos(Yc / 5) + Zc ** 2 / 100
    ref = O.bc_from_coarse(uc, Lc, np.zeros((n,) * 3), Lc / 2)
    d = dev(np.zeros((n,) * 3))
    Q.k_bc_from_coarse(dev(uc), d)
    assert rel(host(d), ref) < 1e-15


@pytest.mark.parametrize("n", [5, 33, 65, 129, 257])
def test_resid_norms(n):
    L = 2.0
    h = L / (n - 1)
    f, u = rand_state(n, 400 + n)
    r = O.residual(f, u, h)
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    Q.k_resid_norms(dev(f), dev(u), h, out)
    got = host(out)
    assert got[0] == pytest.approx((r[1:-1, 1:-1, 1:-1] ** 2).sum(), rel=1e-12)
    assert got[1] == pytest.approx((f[1:-1, 1:-1, 1:-1] ** 2).sum(), rel=1e-12)
    assert got[2] == pytest.approx(O.lib().orc_boundary_coupling_sumsq(n, h, O._p(np.ascontiguousarray(u))), rel=1e-12)
    # bitwise reproducible
    out2 = torch.zeros(3, dtype=torch.float64, device="cuda")
    Q.k_resid_norms(dev(f), dev(u), h, out2)
    assert np.array_equal(host(out2), got)


def _bc_problem(n, L, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, n, n))
    u = np.zeros((n, n, n))
    b = rng.standard_normal((n, n, n))
    mask = np.ones((n, n, n), bool)
    mask[1:-1, 1:-1, 1:-1] = False
    u[mask] = b[mask]
    return f, u


@pytest.mark.parametrize("n", [5, 9, 17, 33, 65, 129])
def test_fmg_fixed_schedule(n):
    L = 10.0
    f, u = _bc_problem(n, L, 500 + n)
    ref = u.copy()
    O.fmg(f, ref, L, ncycle=6, max_extra=0, tol=0.0)
    d = dev(u)
    rr, ex = Q.k_fmg(dev(f), d, L, ncycle=6, max_extra=0, tol=0.0)
    assert ex == 0
    assert rel(host(d), ref) < 1e-12


@pytest.mark.parametrize("n", [5, 9, 17])
def test_coarse_tail_repeatable(n):
    """The single-workgroup coarse tail gives the same bits on every run, for
    FMG and for V-cycles, and matches the oracle."""
    L = 7.0
    f, u = _bc_problem(n, L, 800 + n)
    outs = []
    for _ in range(3):
        d = dev(u)
        Q.k_fmg(dev(f), d, L, ncycle=3, max_extra=0, tol=0.0)
        Q.k_vcycles(dev(f), d, L, 2)
        outs.append(host(d))
    ref = u.copy()
    O.fmg(f, ref, L, ncycle=3, max_extra=0, tol=0.0)
    O.vcycles(f, ref, L, 2)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert rel(outs[0], ref) < 1e-12


@pytest.mark.parametrize("n", [17, 65])
def test_fmg_tolerance_stop_same_cycles(n):
    L = 1.0
    f, u = _bc_problem(n, L, 600 + n)
    ref = u.copy()
    st, rr_o, ex_o = O.fmg(f, ref, L, ncycle=1, max_extra=30, tol=1e-9)
    d = dev(u)
    rr_g, ex_g = Q.k_fmg(dev(f), d, L, ncycle=1, max_extra=30, tol=1e-9)
    assert ex_g == ex_o and rr_g <= 1e-9
    assert rr_g == pytest.approx(rr_o, rel=1e-3)
    assert rel(host(d), ref) < 1e-12


@pytest.mark.parametrize("n", [9, 33, 129])
def test_vcycles(n):
    L = 5.0
    f, u = _bc_problem(n, L, 700 + n)
    ref = u.copy()
    rr_o = O.vcycles(f, ref, L, 3)
    d = dev(u)
    rr_g = Q.k_vcycles(dev(f), d, L, 3)
    assert rr_g == pytest.approx(rr_o, rel=1e-8)
    assert rel(host(d), ref) < 1e-12


@pytest.mark.parametrize("n", [5, 17, 33, 65, 129])
def test_every_smoother_shape_is_bitwise_identical(n):
    """Launch shapes change only the schedule: each node's update is the same
    sum in the same order, so every shape gives the same bits."""
    L = 4.0
    h = L / (n - 1)
    f, u = rand_state(n, 800 + n)
    fd, ud = dev(f), dev(u)
    ref = dev(u)
    Q.k_rbgs_sweep(fd, ud, ref, h)
    ref = host(ref)
    assert rel(ref, O.rbgs_sweep(f, u.copy(), h)) < 1e-14
    for v in Q.SMOOTHER_VARIANTS:
        for kc in (2, 4, 16, 0):
            out = dev(u)
            Q.k_rbgs_sweep_shape(fd, ud, out, h, v, kc)
            assert np.array_equal(host(out), ref), (v, kc)


@pytest.mark.parametrize("n", [5, 9, 17, 33, 65, 129, 257])
def test_sweep_from_zero_is_bitwise_identical(n):
    """A sweep from a zero iterate that reads no iterate (null input) equals
    the sweep of a zero-filled iterate, in every single-sweep shape; only the
    interior of the output is written."""
    L = 3.5
    h = L / (n - 1)
    f = rand_state(n, 2100 + n)[0]
    fd = dev(f)
    ref = dev(np.zeros((n, n, n)))
    Q.k_rbgs_sweep(fd, dev(np.zeros((n, n, n))), ref, h)
    ref = host(ref)
    assert rel(ref, O.rbgs_sweep(f, np.zeros((n, n, n)), h)) < 1e-14
    start = np.full((n, n, n), 7.0)
    start[1:-1, 1:-1, 1:-1] = -3.0
    start[0] = start[-1] = start[:, 0] = start[:, -1] = start[:, :, 0] = start[:, :, -1] = 0.0
    out = dev(start)
    Q.k_rbgs_sweep_from_zero(fd, out, h)
    assert np.array_equal(host(out), ref)
    for v in Q.SMOOTHER_VARIANTS:
        for kc in ((0,) if v in (5, 9, 10) else (2, 4, 16, 0)):
            out = dev(start)
            Q.k_rbgs_sweep_shape(fd, None, out, h, v, kc)
            assert np.array_equal(host(out), ref), (v, kc)


@pytest.mark.parametrize("n", [5, 17, 33, 65])
def test_stacked_sweeps_are_bitwise_single_problem_sweeps(n):
    """Three problems stored back to back and swept in one launch (as the
    batched runner sweeps a size class), from a zero iterate (no input array)
    and from given iterates, give every problem the bits of its own
    single-problem sweep, in every single-sweep shape: a problem's offset is
    applied only to arrays that exist."""
    nb, L = 3, 2.5
    h = L / (n - 1)
    rng = np.random.default_rng(3300 + n)
    f = rng.standard_normal((nb, n, n, n))
    u = rng.standard_normal((nb, n, n, n))
    u[:, 0] = u[:, -1] = u[:, :, 0] = u[:, :, -1] = u[:, :, :, 0] = u[:, :, :, -1] = 0.0
    fd, ud = dev(f), dev(u)
    ref_zero, ref_u = [], []
    for p in range(nb):
        o = dev(np.zeros((n, n, n)))
        Q.k_rbgs_sweep_from_zero(dev(f[p]), o, h)
        ref_zero.append(host(o))
        o = dev(u[p])
        Q.k_rbgs_sweep(dev(f[p]), dev(u[p]), o, h)
        ref_u.append(host(o))
    start = np.full((nb, n, n, n), 5.0)
    start[:, 0] = start[:, -1] = start[:, :, 0] = start[:, :, -1] = start[:, :, :, 0] = start[:, :, :, -1] = 0.0
    for v in Q.SMOOTHER_VARIANTS:
        for kc in ((0,) if v in (5, 9, 10) else (2, 16, 0)):
            out = dev(start)
            Q.k_rbgs_sweep_stacked(fd, None, out, h, v, kc)
            got = host(out)
            out2 = dev(u)
            Q.k_rbgs_sweep_stacked(fd, ud, out2, h, v, kc)
            got2 = host(out2)
            for p in range(nb):
                assert np.array_equal(got[p], ref_zero[p]), (v, kc, p)
                assert np.array_equal(got2[p], ref_u[p]), (v, kc, p)


@pytest.mark.parametrize("n", [5, 17, 33, 65, 129, 257])
def test_single_sweep_with_correction_is_bitwise_identical(n):
    """A single sweep that applies the coarse correction on load equals
    prolong-add followed by a sweep, bit for bit, in every shape."""
    L = 4.5
    h = L / (n - 1)
    f, u = rand_state(n, 1900 + n)
    nc = (n + 1) // 2
    uc = np.random.default_rng(n + 3).standard_normal((nc, nc, nc))
    uc[0, :, :] = uc[-1, :, :] = uc[:, 0, :] = uc[:, -1, :] = uc[:, :, 0] = uc[:, :, -1] = 0.0
    fd, ucd = dev(f), dev(uc)
    pa = dev(u)
    Q.k_prolong_add(ucd, pa)
    ref = dev(u)
    Q.k_rbgs_sweep(fd, pa, ref, h)
    ref = host(ref)
    for v in Q.SMOOTHER_VARIANTS:
        for kc in ((0,) if v in (5, 9, 10) else (2, 4, 16, 0)):
            out = dev(u)
            Q.k_rbgs_sweep_shape(fd, dev(u), out, h, v, kc, uc=ucd)
            assert np.array_equal(host(out), ref), (v, kc)


@pytest.mark.parametrize("n", [9, 17, 33, 65, 129, 257])
def test_sweep_restrict_equals_sweep_then_restriction(n):
    """The fused last pre-smoothing sweep and residual restriction gives the
    bits of a sweep launch followed by a restriction launch: the swept u,
    the coarse right-hand side, the zeroed coarse iterate and the other coarse
    buffer zeroed on its boundary only (ring recomputation, several tiles at
    129^3 and 257^3, ragged edges)."""
    L = 5.5
    h = L / (n - 1)
    f, u = rand_state(n, 5100 + n)
    nc = (n + 1) // 2
    fd = dev(f)
    ref_u = dev(u)
    Q.k_rbgs_sweep(fd, dev(u), ref_u, h)
    ref = [dev(np.full((nc,) * 3, 3.0)) for _ in range(3)]
    Q.k_residual_restrict(fd, ref_u, h, *ref)
    out_u = dev(np.full((n,) * 3, -7.0))
    bnd = np.ones((n,) * 3, bool)
    bnd[1:-1, 1:-1, 1:-1] = False
    got = [dev(np.full((nc,) * 3, 3.0)) for _ in range(3)]
    Q.k_rbgs_sweep_restrict(fd, dev(u), out_u, h, *got)
    gu, ru = host(out_u), host(ref_u)
    assert np.array_equal(gu[~bnd], ru[~bnd])
    assert np.all(gu[bnd] == -7.0)   # boundary nodes are not written
    for a, b in zip(got, ref):
        assert np.array_equal(host(a), host(b))
    # and against the oracle's sweep and restriction
    uo = O.rbgs_sweep(f, u.copy(), h)
    assert rel(gu[~bnd], uo[~bnd]) < 1e-14
    assert rel(host(got[0]), O.restrict_fw(O.residual(f, uo, h))) < 1e-12


@pytest.mark.parametrize("n", [65, 129])
def test_fmg_with_fused_sweep_restrict_keeps_the_bits(n):
    """An FMG solve whose levels fuse the last pre-smoothing sweep with the
    residual restriction gives the bits of the solve without the fusion."""
    L = 9.0
    f, u = _bc_problem(n, L, 4300 + n)
    levels = [m for m in (9, 17, 33, 65, 129) if m <= n]
    saved = {m: Q.tune_get_sweep_restrict(m) for m in levels}
    outs = []
    try:
        for flag in (0, 1):
            for m in levels:
                Q.tune_set_sweep_restrict(m, flag)
            d = dev(u)
            Q.k_fmg(dev(f), d, L, ncycle=2, max_extra=0, tol=0.0)
            outs.append(host(d))
    finally:
        for m, v in saved.items():
            Q.tune_set_sweep_restrict(m, v)
    assert np.array_equal(outs[0], outs[1])


def test_correcting_sweep_shape_keeps_the_bits():
    """The correcting sweep's own launch shape, set apart from the plain
    sweep's, changes only the schedule: an FMG solve whose 129^3 level folds
    the correction into single sweeps gives the same bits in every shape."""
    n, L = 129, 10.0
    f, u = _bc_problem(n, L, 4242)
    saved = Q.tune_get_corr(n)
    outs = []
    try:
        for shape in ((-1, 0), (13, 32), (7, 16), (11, 0)):
            Q.tune_set_corr(n, *shape)
            d = dev(u)
            Q.k_fmg(dev(f), d, L, ncycle=2, max_extra=0, tol=0.0)
            outs.append(host(d))
    finally:
        Q.tune_set_corr(n, *saved)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("n", [5, 17, 33, 65, 129])
def test_every_fused_shape_is_bitwise_identical(n):
    """The fused two-sweep smoother in every shape (z-march tiles, 8^3, 6^3 and
    4^3 bricks, ragged at the far faces) equals two single sweeps bit for bit,
    from a zero iterate without an input array too, and with a coarse
    correction equals prolong-add then two sweeps."""
    L = 5.0
    h = L / (n - 1)
    f, u = rand_state(n, 1700 + n)
    fd = dev(f)
    a, b, c = dev(u), dev(u), dev(u)
    Q.k_rbgs_sweep(fd, a, b, h)
    Q.k_rbgs_sweep(fd, b, c, h)
    two = host(c)
    nc = (n + 1) // 2
    uc = np.random.default_rng(n).standard_normal((nc, nc, nc))
    uc[0, :, :] = uc[-1, :, :] = uc[:, 0, :] = uc[:, -1, :] = uc[:, :, 0] = uc[:, :, -1] = 0.0
    ucd = dev(uc)
    pa = dev(u)
    Q.k_prolong_add(ucd, pa)
    b2, c2 = dev(u), dev(u)
    Q.k_rbgs_sweep(fd, pa, b2, h)
    Q.k_rbgs_sweep(fd, b2, c2, h)
    two_p = host(c2)
    # from a zero iterate: no input array, only the output's interior written
    z = np.zeros((n, n, n))
    za, zb = dev(z), dev(z)
    Q.k_rbgs_sweep(fd, dev(z), za, h)
    Q.k_rbgs_sweep(fd, za, zb, h)
    two_z = host(zb)
    start = np.full((n, n, n), -5.0)
    start[0] = start[-1] = start[:, 0] = start[:, -1] = start[:, :, 0] = start[:, :, -1] = 0.0
    before = Q.tune_get_fused(n)
    try:
        for v in Q.FUSED_VARIANTS:
            for kc in ((0,) if v in (2, 3, 4, 8, 9) else (4, 16, 0)):
                Q.tune_set_fused(n, v, kc)
                out = dev(u)
                Q.k_rbgs_double_sweep(fd, dev(u), out, h)
                assert np.array_equal(host(out), two), (v, kc)
                out = dev(start)
                Q.k_rbgs_double_sweep(fd, None, out, h)
                assert np.array_equal(host(out), two_z), (v, kc, "zero iterate")
                out = dev(u)
                Q.k_rbgs_double_sweep(fd, dev(u), out, h, uc=ucd)
                assert np.array_equal(host(out), two_p), (v, kc, "prolong")
    finally:
        Q.tune_set_fused(n, *before)


@pytest.mark.parametrize("n", [257, 513])
def test_skewed_double_sweep_full_size(n):
    """The skewed two-sweep march (whole 64x16 columns, the four half-sweeps two
    planes apart) equals two single sweeps bit for bit at full size, from a
    given iterate and from a zero one, and with the coarse-grid correction
    applied in the same launch it equals a prolong-add and then two sweeps."""
    h = 1.0 / (n - 1)
    g = torch.Generator(device="cuda")
    g.manual_seed(n)
    f = torch.randn((n,) * 3, dtype=torch.float64, device="cuda", generator=g)
    u = torch.randn((n,) * 3, dtype=torch.float64, device="cuda", generator=g)
    u[0] = u[-1] = u[:, 0] = u[:, -1] = u[:, :, 0] = u[:, :, -1] = 0.0
    a, b = u.clone(), u.clone()
    Q.k_rbgs_sweep(f, u, a, h)
    Q.k_rbgs_sweep(f, a, b, h)
    z = torch.zeros_like(u)
    za, zb = z.clone(), z.clone()
    Q.k_rbgs_sweep(f, z, za, h)
    Q.k_rbgs_sweep(f, za, zb, h)
    before = Q.tune_get_fused(n)
    try:
        for v in (8, 9):
            Q.tune_set_fused(n, v, 0)
            out = torch.full_like(u, 3.0)
            out[0] = out[-1] = out[:, 0] = out[:, -1] = out[:, :, 0] = out[:, :, -1] = 0.0
            Q.k_rbgs_double_sweep(f, u, out, h)
            assert torch.equal(out, b), v
            out.fill_(-2.0)
            out[0] = out[-1] = out[:, 0] = out[:, -1] = out[:, :, 0] = out[:, :, -1] = 0.0
            Q.k_rbgs_double_sweep(f, None, out, h)
            assert torch.equal(out, zb), v
            nc = (n + 1) // 2
            uc = torch.randn((nc,) * 3, dtype=torch.float64, device="cuda", generator=g)
            uc[0] = uc[-1] = uc[:, 0] = uc[:, -1] = uc[:, :, 0] = uc[:, :, -1] = 0.0
            p = u.clone()
            Q.k_prolong_add(uc, p)
            pa, pb = p.clone(), p.clone()
            Q.k_rbgs_sweep(f, p, pa, h)
            Q.k_rbgs_sweep(f, pa, pb, h)
            out.fill_(5.0)
            out[0] = out[-1] = out[:, 0] = out[:, -1] = out[:, :, 0] = out[:, :, -1] = 0.0
            Q.k_rbgs_double_sweep(f, u, out, h, uc=uc)
            assert torch.equal(out, pb), (v, "prolong")
    finally:
        Q.tune_set_fused(n, *before)


def test_autotune_installs_a_table(tmp_path):
    before = Q.tune_get(65)
    best = Q.autotune(n_max=65, both=True, reps=3, json_path=str(tmp_path / "t.json"))
    assert set(best) == {33, 65} and all(v > 0 for v in best.values())
    txt = (tmp_path / "t.json").read_text()
    assert '"n": 65' in txt
    Q.tune_set(65, *before)
    Q.tune_load(str(tmp_path / "t.json"))
    assert Q.tune_get(65) in [(v, k) for v in Q.SMOOTHER_VARIANTS for k in (2, 4, 8, 16, 32, 64, 128, 0)]
    assert '"split_prolong"' in txt and all(Q.tune_get_split(n, fp32=fp) in (0, 1) for n in (33, 65)
                                            for fp in (False, True))


@pytest.mark.parametrize("n", [5, 9, 17, 33, 65, 129, 257])
def test_double_sweep_equals_two_sweeps_bitwise(n):
    """The fused two-sweep kernel (four stages of one z-march) gives the same
    bits as two single sweeps, and with a coarse correction the same bits as
    prolong-add followed by two sweeps; both agree with the oracle."""
    L = 6.0
    h = L / (n - 1)
    f, u = rand_state(n, 900 + n)
    fd = dev(f)
    a, b = dev(u), dev(u)
    Q.k_rbgs_sweep(fd, a, b, h)
    c = dev(u)
    Q.k_rbgs_sweep(fd, b, c, h)
    two = host(c)
    out = dev(u)
    Q.k_rbgs_double_sweep(fd, dev(u), out, h)
    assert np.array_equal(host(out), two)
    ref = u.copy()
    O.rbgs_sweep(f, ref, h)
    O.rbgs_sweep(f, ref, h)
    assert rel(two, ref) < 1e-13
    nc = (n + 1) // 2
    uc = np.random.default_rng(n).standard_normal((nc,) * 3)
    ucd = dev(uc)
    p = dev(u)
    Q.k_prolong_add(ucd, p)
    q, r = dev(u), dev(u)
    Q.k_rbgs_sweep(fd, p, q, h)
    Q.k_rbgs_sweep(fd, q, r, h)
    out = dev(u)
    Q.k_rbgs_double_sweep(fd, dev(u), out, h, uc=ucd)
    assert np.array_equal(host(out), host(r))
    ref = O.prolong_add(uc, u.copy())
    O.rbgs_sweep(f, ref, h)
    O.rbgs_sweep(f, ref, h)
    assert rel(host(out), ref) < 1e-13

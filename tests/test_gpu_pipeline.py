"""End-to-end parity of the C-ABI pipeline (deposit -> Newton FMG -> Eq. 2
source -> QUMOND FMG -> gather) against the FP64 oracle, on the same seeded
particles.

* The int64 fixed-point density grid is bit-exact (integer work), including
  after shuffling the particles (order independence, no lost atomics).
* Potentials on every node of every box agree to 1e-10 of max|Phi| (the
  FP64 tolerance: both sides run the same schedule, and rounding differences
  are damped by the iteration), and so do gathered forces, with the same
  V-cycle counts under the tolerance stop.
Workloads: the Kuzmin disk in one 65^3 box, and the two-component disk with
1e6 particles in four nested 129^3 boxes (400/200/100/50 kpc), plus edge
cases (no particles, every particle outside, the smallest grids, zero outer
boundary, a0 = 0).
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import analytic as A
from paper_1201_3185_amd import qumond as Q
from paper_1201_3185_amd import synth

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def run_gpu(cfg: Q.Config, p, total_mass=None):
    tm = p.total_mass if total_mass is None else total_mass
    ctx = Q.Context(cfg)
    x, y, z, m = dev(p.x), dev(p.y), dev(p.z), dev(p.m)
    out = {"n_outside": ctx.deposit(x, y, z, m, tm)}
    out["newton"] = ctx.solve_newton()
    ctx.mond_source()
    out["mond"] = ctx.solve_mond()
    nb = len(cfg.box_side)
    for key, fld in (("q", Q.FIELD_RHO_FIXED), ("f", Q.FIELD_RHS), ("phin", Q.FIELD_PHI_N), ("S", Q.FIELD_SOURCE),
                     ("phi", Q.FIELD_PHI)):
        out[key] = [ctx.get_field(b, fld).cpu().numpy() for b in range(nb)]
    out["ctx"] = ctx
    return out


def run_oracle(cfg: Q.Config, p, total_mass=None):
    tm = p.total_mass if total_mass is None else total_mass
    oc = O.OracleConfig(n=cfg.n, box_side=list(cfg.box_side), G=cfg.G, a0=cfg.a0, npre=cfg.npre, npost=cfg.npost,
                        ncycle_fmg=cfg.ncycle_fmg, max_vcycles=cfg.max_vcycles, tol_rel=cfg.tol_rel,
                        outer_bc=cfg.outer_bc, gather_frac=cfg.gather_frac, fixed_shift=cfg.fixed_shift)
    return O.run_pipeline(oc, p.x, p.y, p.z, p.m, tm), oc


def compare(g, o, cfg, check_cycles=True, s_tol=1e-10):
    nb = len(cfg.box_side)
    for b in range(nb):
        assert np.array_equal(g["q"][b], o.q[b]), f"int64 density differs in box {b}"
        assert rel(g["f"][b], o.f[b]) <= 1e-15
        assert rel(g["phin"][b], o.phin[b]) <= 1e-10
        # The source kernel on the GPU's own Phi_N (cross-fed) agrees to rounding.
        h = cfg.box_side[b] / (cfg.n - 1)
        assert rel(g["S"][b], O.mond_source(g["phin"][b], cfg.box_side[b], cfg.a0)) <= 1e-12
        # Directly: S is a second difference of Phi_N, so where |S| is tiny (no
        # matter) the solve-tolerance differences of Phi_N are amplified ~1/h^2.
        assert rel(g["S"][b], o.S[b]) <= s_tol
        assert rel(g["phi"][b], o.phi[b]) <= 1e-10
        if check_cycles:
            assert g["newton"]["vcycles"][b] == o.info_newton[b][2]
            assert g["mond"]["vcycles"][b] == o.info_mond[b][2]
    assert g["n_outside"] == o.n_outside


def compare_forces(ctx, o, oc, pts, total_mass):
    xd, yd, zd = dev(pts[0]), dev(pts[1]), dev(pts[2])
    for which, phis in ((0, o.phin), (1, o.phi)):
        ax, ay, az, used = ctx.gather_forces(xd, yd, zd, which)
        rx, ry, rz, ru = O.gather(phis, oc.box_side, *pts, frac=oc.gather_frac, G=oc.G, a0=oc.a0, M=total_mass,
                                  mond=bool(which))
        assert np.array_equal(used.cpu().numpy(), ru)
        ga = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()])
        ra = np.stack([rx, ry, rz])
        assert rel(ga, ra) <= 1e-10


@pytest.fixture(scope="module")
def kuzmin_run():
    p = synth.kuzmin_disk(100000, 3.0, 1e10, synth.seed_for(1))
    cfg = Q.Config(n=65, box_side=[100.0])
    return p, cfg, run_gpu(cfg, p), run_oracle(cfg, p)


def test_config1_kuzmin_parity(kuzmin_run):
    p, cfg, g, (o, oc) = kuzmin_run
    compare(g, o, cfg)
    assert all(r <= 1e-10 for r in g["newton"]["relres"] + g["mond"]["relres"])
    rng = np.random.default_rng(5)
    pts = (np.concatenate([p.x[:2000], rng.uniform(-80, 80, 300)]),
           np.concatenate([p.y[:2000], rng.uniform(-80, 80, 300)]),
           np.concatenate([p.z[:2000], rng.uniform(-80, 80, 300)]))
    compare_forces(g["ctx"], o, oc, pts, p.total_mass)


def test_config1_rotation_curve(kuzmin_run):
    p, cfg, g, (o, oc) = kuzmin_run
    R = np.arange(8.0, 37.0, 2.0)
    ctx = g["ctx"]
    for which, phis, exact in ((0, o.phin, A.kuzmin_vc2_newton), (1, o.phi, A.kuzmin_vc2_mond)):
        vc2 = ctx.rotation_curve(dev(R), 16, which).cpu().numpy()
        x, y, z = O.rotation_curve_points(R, 16)
        ax, ay, _, _ = O.gather(phis, oc.box_side, x, y, z, M=p.total_mass, mond=bool(which))
        ref = O.vc2_from_acc(x, y, ax, ay, len(R))
        assert rel(vc2, ref) <= 1e-10
        # context: the analytic Kuzmin curves (shot noise, monopole boundary)
        assert np.abs(np.sqrt(vc2 / exact(R, 3.0, 1e10)) - 1).max() < 0.03


def test_deposit_shuffle_invariant(kuzmin_run):
    p, cfg, g, _ = kuzmin_run
    ps = p.shuffled(99)
    ctx = Q.Context(cfg)
    ctx.deposit(dev(ps.x), dev(ps.y), dev(ps.z), dev(ps.m), p.total_mass)
    assert np.array_equal(ctx.get_field(0, Q.FIELD_RHO_FIXED).cpu().numpy(), g["q"][0])
    # and the deterministic solve reproduces the potential bit for bit
    ctx.solve_newton()
    assert np.array_equal(ctx.get_field(0, Q.FIELD_PHI_N).cpu().numpy(), g["phin"][0])


@pytest.mark.slow
def test_config2_nested_parity():
    p = synth.two_component_disk(1000000, synth.seed_for(2))
    cfg = Q.Config(n=129, box_side=[400.0, 200.0, 100.0, 50.0])
    g = run_gpu(cfg, p)
    o, oc = run_oracle(cfg, p)
    compare(g, o, cfg)
    rng = np.random.default_rng(6)
    idx = rng.choice(p.n, 5000, replace=False)
    pts = (np.concatenate([p.x[idx], rng.uniform(-250, 250, 500)]),
           np.concatenate([p.y[idx], rng.uniform(-250, 250, 500)]),
           np.concatenate([p.z[idx], rng.uniform(-250, 250, 500)]))
    compare_forces(g["ctx"], o, oc, pts, p.total_mass)


@pytest.mark.parametrize("n,sides", [(5, [10.0]), (9, [40.0, 20.0]), (17, [60.0, 30.0, 15.0]), (33, [80.0, 40.0])])
def test_small_grids_and_nesting(n, sides):
    p = synth.two_component_disk(20000, 77 + n)
    cfg = Q.Config(n=n, box_side=sides)
    g = run_gpu(cfg, p)
    o, oc = run_oracle(cfg, p)
    compare(g, o, cfg)


def test_zero_outer_bc_and_a0_zero():
    p = synth.kuzmin_disk(30000, 3.0, 1e10, 1234)
    cfg = Q.Config(n=33, box_side=[120.0, 60.0], outer_bc=Q.QUMOND_BC_ZERO, a0=0.0)
    g = run_gpu(cfg, p)
    o, oc = run_oracle(cfg, p)
    compare(g, o, cfg)
    for b in range(2):   # nu = 1 exactly: the QUMOND potential is the Newtonian one
        assert rel(g["phi"][b], g["phin"][b]) <= 1e-10


def test_no_particles_and_all_outside():
    cfg = Q.Config(n=17, box_side=[10.0])
    empty = synth.Particles(np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    g = run_gpu(cfg, empty, total_mass=1e9)
    o, oc = run_oracle(cfg, empty, total_mass=1e9)
    compare(g, o, cfg, check_cycles=False, s_tol=1e-7)
    assert np.all(g["q"][0] == 0) and g["n_outside"] == 0
    far = synth.Particles(np.array([50.0, -60.0, 5.0]), np.array([0.0, 0.0, 5.0]), np.array([0.0, 0.0, 0.0]),
                          np.array([1e9, 1e9, 1e9]))
    g = run_gpu(cfg, far)
    o, oc = run_oracle(cfg, far)
    compare(g, o, cfg, check_cycles=False, s_tol=1e-7)
    assert g["n_outside"] == 3 and np.all(g["q"][0] == 0)
    # forces fall back to the monopole outside the box
    ax, ay, az, used = g["ctx"].gather_forces(dev([100.0]), dev([0.0]), dev([0.0]), 0)
    assert used.cpu().numpy()[0] == 255
    assert ax.cpu().numpy()[0] == pytest.approx(-O.G_KPC * 3e9 / 1e4, rel=1e-14)


def test_call_order_state_machine():
    cfg = Q.Config(n=17, box_side=[10.0])
    ctx = Q.Context(cfg)
    with pytest.raises(Q.QumondError) as e:
        ctx.solve_newton()
    assert e.value.status == Q.QUMOND_ERR_STATE
    x = dev([0.1])
    with pytest.raises(Q.QumondError) as e:
        ctx.gather_forces(x, x, x, 0)
    assert e.value.status == Q.QUMOND_ERR_STATE
    ctx.deposit(x, x, x, dev([1e9]), 1e9)
    with pytest.raises(Q.QumondError) as e:
        ctx.mond_source()
    assert e.value.status == Q.QUMOND_ERR_STATE
    ctx.solve_newton()
    ctx.gather_forces(x, x, x, 0)
    with pytest.raises(Q.QumondError) as e:
        ctx.gather_forces(x, x, x, 1)
    assert e.value.status == Q.QUMOND_ERR_STATE
    ctx.mond_source()
    ctx.solve_mond()
    ctx.gather_forces(x, x, x, 1)


def test_not_converged_reports_best_iterate():
    p = synth.kuzmin_disk(20000, 3.0, 1e10, 4321)
    cfg = Q.Config(n=33, box_side=[100.0], ncycle_fmg=1, max_vcycles=1, tol_rel=1e-14)
    ctx = Q.Context(cfg)
    ctx.deposit(dev(p.x), dev(p.y), dev(p.z), dev(p.m), p.total_mass)
    with pytest.raises(Q.QumondError) as e:
        ctx.solve_newton()
    assert e.value.status == Q.QUMOND_ERR_NOT_CONVERGED
    info = ctx.solve_newton(allow_not_converged=True)
    assert info["converged"] == [0] and info["vcycles"] == [1] and info["relres"][0] < info["relres0"][0]


def test_overlapped_solve_equals_separate_calls_bitwise():
    """qumond_solve runs the Newtonian and QUMOND chains on two streams; the
    kernels and schedules are the same, so every field matches bit for bit."""
    p = synth.two_component_disk(200000, 4242)
    cfg = Q.Config(n=65, box_side=[200.0, 100.0, 50.0])
    g = run_gpu(cfg, p)
    ctx = Q.Context(cfg)
    ctx.deposit(dev(p.x), dev(p.y), dev(p.z), dev(p.m), p.total_mass)
    i_n, i_m = ctx.solve()
    assert i_n["vcycles"] == g["newton"]["vcycles"] and i_m["vcycles"] == g["mond"]["vcycles"]
    for b in range(3):
        for key, fld in (("phin", Q.FIELD_PHI_N), ("S", Q.FIELD_SOURCE), ("phi", Q.FIELD_PHI)):
            assert np.array_equal(ctx.get_field(b, fld).cpu().numpy(), g[key][b]), (key, b)
    # repeated calls reuse the second chain and stay identical
    ctx.solve()
    assert np.array_equal(ctx.get_field(2, Q.FIELD_PHI).cpu().numpy(), g["phi"][2])
    x = dev([1.0, 10.0, 60.0])
    ax, _, _, _ = ctx.gather_forces(x, x, x, 1)
    ax2, _, _, _ = g["ctx"].gather_forces(x, x, x, 1)
    assert np.array_equal(ax.cpu().numpy(), ax2.cpu().numpy())

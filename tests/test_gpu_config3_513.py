"""Parity at the full size of the 513^3 workload: the two-component disk
(stars 5e10 Msun, R_d 3 kpc, sech^2 0.3 kpc; gas 1e10 Msun, 6 kpc, 0.15 kpc),
1e7 particles, one 513^3 box of 120 kpc with a monopole outer boundary,
against the FP64 oracle run once on the same particles (Sec. 2's pipeline:
deposit, Newtonian FMG, Eq. 2 source, QUMOND FMG, gather).

* Plain FP64 to a 1e-10 relative residual, in the launch shapes of the
  committed MI355X table the benchmark uses: the int64 density is bit-exact,
  Phi_N and
  Phi agree to 1e-10 of max|Phi| at every node with the same V-cycle counts,
  the source agrees to 1e-12 when the oracle forms it from the GPU's own
  Phi_N, and forces at 1e5 particles plus points outside the disk agree to
  1e-10 with the same box choice.
* Mixed precision (FP32 multigrid inside FP64 refinement): refined to a
  1e-7 FP64 residual the potentials are within 1e-6 of the oracle's (the
  accuracy bar); stopped at the timed 1e-6 residual within 3e-6 (a residual
  bounds the field error only up to the operator's conditioning, which grows
  with the grid -- about 1.2x the residual at 129^3, 2.2x at 513^3 -- and the
  QUMOND potential also carries the Newtonian error through the source).
The oracle runs its node-parallel loops on several host threads (same bits
as one thread); its deposit and sums stay serial.
"""
import os
import time

import numpy as np
import pytest
import torch

import oracle as O
from paper_1201_3185_amd import qumond as Q
from paper_1201_3185_amd import synth

pytestmark = pytest.mark.gpu

N, L = 513, 120.0


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


TABLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1201_3185_amd",
                     "launch_shapes_mi355x.json")


@pytest.fixture(scope="module")
def config3():
    # the launch shapes the benchmark times at this size (the committed MI355X table)
    if os.path.exists(TABLE):
        Q.tune_load(TABLE)
    p = synth.two_component_disk(10_000_000, synth.seed_for(3))
    prev = O.set_threads(max(1, min(16, os.cpu_count() or 1)))
    try:
        t0 = time.perf_counter()
        o = O.run_pipeline(O.OracleConfig(n=N, box_side=[L], tol_rel=1e-10), p.x, p.y, p.z, p.m, p.total_mass)
        print(f"\noracle 513^3: {time.perf_counter() - t0:.1f} s on {O.set_threads(1)} threads", flush=True)
    finally:
        O.set_threads(prev)
    return p, o


def gpu_solve(p, **kw):
    ctx = Q.Context(Q.Config(n=N, box_side=[L], **kw))
    x, y, z, m = dev(p.x), dev(p.y), dev(p.z), dev(p.m)
    ctx.deposit(x, y, z, m, p.total_mass)
    i_n, i_m = ctx.solve()
    return ctx, i_n, i_m


def test_config3_fp64_against_oracle(config3):
    p, o = config3
    ctx, i_n, i_m = gpu_solve(p, tol_rel=1e-10)
    assert np.array_equal(ctx.get_field(0, Q.FIELD_RHO_FIXED).cpu().numpy(), o.q[0])
    assert rel(ctx.get_field(0, Q.FIELD_RHS).cpu().numpy(), o.f[0]) <= 1e-15
    phin = ctx.get_field(0, Q.FIELD_PHI_N).cpu().numpy()
    e_phin = rel(phin, o.phin[0])
    S = ctx.get_field(0, Q.FIELD_SOURCE).cpu().numpy()
    e_s_fed = rel(S, O.mond_source(phin, L))
    e_s = rel(S, o.S[0])
    phi = ctx.get_field(0, Q.FIELD_PHI).cpu().numpy()
    e_phi = rel(phi, o.phi[0])
    print(f"513^3 FP64: Phi_N {e_phin:.2e}, S cross-fed {e_s_fed:.2e}, S direct {e_s:.2e}, Phi {e_phi:.2e}; "
          f"cycles {i_n['vcycles'][0]}/{i_m['vcycles'][0]} (oracle {o.info_newton[0][2]}/{o.info_mond[0][2]})",
          flush=True)
    assert e_phin <= 1e-10 and e_phi <= 1e-10
    assert e_s_fed <= 1e-12
    # directly, S is a second difference of Phi_N: the two solves' rounding
    # differences (~1e-14 of max|Phi_N|) come back multiplied by ~(L/h)^2
    assert e_s <= 1e-8
    assert i_n["vcycles"][0] == o.info_newton[0][2] and i_m["vcycles"][0] == o.info_mond[0][2]
    assert i_n["relres"][0] <= 1e-10 and i_m["relres"][0] <= 1e-10
    del phin, S, phi
    # forces: 1e5 particles of the disk and points beyond it (monopole outside the box)
    rng = np.random.default_rng(31)
    pts = tuple(np.concatenate([c[:100_000], rng.uniform(-75.0, 75.0, 2000)]) for c in (p.x, p.y, p.z))
    xd, yd, zd = (dev(c) for c in pts)
    for which, phis in ((0, o.phin), (1, o.phi)):
        ax, ay, az, used = ctx.gather_forces(xd, yd, zd, which)
        rx, ry, rz, ru = O.gather(phis, [L], *pts, M=p.total_mass, mond=bool(which))
        assert np.array_equal(used.cpu().numpy(), ru)
        g = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()])
        assert rel(g, np.stack([rx, ry, rz])) <= 1e-10
    ctx.close()
    del ctx
    torch.cuda.empty_cache()


def test_config3_mixed_against_oracle(config3):
    p, o = config3
    errs = {}
    for tol in (1e-6, 1e-7):
        ctx, i_n, i_m = gpu_solve(p, tol_rel=tol, precision=Q.QUMOND_MIXED)
        for info in (i_n, i_m):
            assert info["converged"] == [1] and info["relres"][0] <= tol and info["refine_iters"][0] >= 1
        assert np.array_equal(ctx.get_field(0, Q.FIELD_RHO_FIXED).cpu().numpy(), o.q[0])
        errs[tol] = (rel(ctx.get_field(0, Q.FIELD_PHI_N).cpu().numpy(), o.phin[0]),
                     rel(ctx.get_field(0, Q.FIELD_PHI).cpu().numpy(), o.phi[0]))
        print(f"513^3 mixed to {tol:g}: Phi_N {errs[tol][0]:.2e}, Phi {errs[tol][1]:.2e}", flush=True)
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    # the accuracy bar: refined to a 1e-7 residual, both potentials within 1e-6
    assert max(errs[1e-7]) <= 1e-6
    # stopped at the timed 1e-6 residual, the field error is a few times the
    # residual: the residual bounds the error only through the operator's
    # conditioning, which grows with the grid, and Phi also carries Phi_N's
    # error through the source
    assert max(errs[1e-6]) <= 3e-6


def test_config3_deposit_conserves_mass(config3):
    """Integer mass of the fixed-point grid equals the mass of the particles
    inside the box to within the 8 corner roundings of each particle."""
    p, o = config3
    s = O.fixed_shift(p.total_mass)
    u = lambda c: (c + 0.5 * L) * ((N - 1) / L)
    ins = np.ones(p.n, bool)
    for c in (p.x, p.y, p.z):
        ins &= (u(c) >= 0) & (u(c) < N - 1)
    m_in = p.m[ins].sum() * 2.0 ** s
    assert abs(int(o.q[0].sum()) - m_in) <= 4 * p.n + 1e-12 * m_in

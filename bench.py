#!/usr/bin/env python3
"""Throughput of the particle-mesh QUMOND solve on one MI355X.

One step is one pass of the whole path over one synthetic galaxy already
resident in HBM: CIC deposit -> Newtonian FMG -> Eq. 2 source -> QUMOND FMG ->
force gather at every particle, all through the C ABI of libqumond.so
(qumond_deposit, qumond_solve -- the source and both FMG solves, the QUMOND
chain on a second stream -- and qumond_gather_forces).

Headline workload (the largest single-GPU configuration): two-component
exponential disk (stars Md = 5e10 Msun, Rd = 3 kpc, sech^2 height 0.3 kpc; gas
Mg = 1e10 Msun, Rg = 6 kpc, height 0.15 kpc), 1e7 particles, one 513^3 box of
120 kpc with a monopole outer boundary, 2+2 red-black sweeps and 6 V-cycles per
FMG level, both solves to a 1e-10 relative residual, plain FP64.

value = 513^3 grid points / wall time of one step (host syncs of the stopping
tests included).  The roofline object reports the red-black smoother on the
finest (513^3) level, the dominant kernel: algorithmic bytes (read u, read f,
write u: 24 B per node per launch, of one sweep or, where the launch table
fuses the pre-smoothing pair, of two) of those launches over their average
duration, from hipEvents the library records around each of them, on the
stream it runs on, during the timed steps; with fused pairs it also reports
the single plain sweep timed on its own.  cpu_baseline runs the CPU oracle on the full headline
workload (its node-parallel loops on the stated number of host threads), and
its potentials are the reference for every error figure of the 513^3 legs.

Further legs (same JSON line, not the headline value): the 513^3 disk to 1e-6
in FP64 (the paper's schedule and a 2-cycle one) and in mixed precision; the
nested 129^3 step (four boxes); the batched fit (64 disks of 129^3/257^3 in one
captured graph); the learned initial guess on held-out 129^3 disks; the paper's
Kuzmin and exponential-disk experiments.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
METRIC = "QUMOND solve grid-pts/s & wall time to 1e-6 rel residual: plain FP64 vs mixed+learned"
HBM_PEAK_GBS = 8000.0
LAUNCH_TABLE = os.path.join(HERE, "paper_1201_3185_amd", "launch_shapes_mi355x.json")
N3, L3, NP3 = 513, 120.0, 10_000_000


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def rel(a, b):
    import numpy as np
    return float(np.abs(a - b).max() / np.abs(b).max())


def host_cpu():
    """CPU model and logical core count of this host (from /proc/cpuinfo)."""
    model, cores = platform.processor() or "unknown", os.cpu_count() or 1
    try:
        with open("/proc/cpuinfo") as fh:
            lines = fh.read().splitlines()
        names = [ln.split(":", 1)[1].strip() for ln in lines if ln.startswith("model name")]
        if names:
            model, cores = names[0], len(names)
    except OSError:
        pass
    return model, cores


def smoother_traffic(key, sweeps):
    """HBM traffic per launch of the finest-level smoother from the committed
    rocprofv3 counter runs (copy-calibrated FETCH_SIZE + WRITE_SIZE), valid only
    for the same kind of launch (sweeps per launch) while the kernel's source
    file is unchanged (null otherwise)."""
    path = os.path.join(HERE, "profiles", "smoother_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(key)
    if not rec or rec.get("sweeps_per_launch", 1) != sweeps:
        return None
    src = open(os.path.join(HERE, rec.get("kernel_source", "paper_1201_3185_amd/csrc/grid_kernels.hip")), "rb").read()
    if rec.get("source_sha256", rec.get("grid_kernels_sha256")) != hashlib.sha256(src).hexdigest():
        return None
    return rec.get("bytes_per_launch")


def single_sweep_roofline(Q, torch, n=513, reps=15):
    """The single plain sweep at n^3 with the loaded launch shape, timed on its
    own (hipEvents around each launch, median of reps): the kernel of the
    levels that sweep once per launch, reported beside the two-sweep launch."""
    h = 1.0 / (n - 1)
    f = torch.ones((n,) * 3, dtype=torch.float64, device="cuda")
    u = [torch.full_like(f, 0.5), torch.full_like(f, 0.5)]
    for r in range(3):
        Q.k_rbgs_sweep(f, u[r & 1], u[1 - (r & 1)], h)
    ts = []
    for r in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        Q.k_rbgs_sweep(f, u[r & 1], u[1 - (r & 1)], h)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    del f, u
    torch.cuda.empty_cache()
    med_ms = sorted(ts)[len(ts) // 2]
    achieved = 24.0 * n ** 3 / (med_ms * 1e-3) / 1e9
    return {"median_launch_us": round(med_ms * 1e3, 2), "achieved": round(achieved, 1),
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "timed": f"median of {reps} launches on {n}^3 fields, apart from the step",
            "traffic": smoother_traffic("fp64_513_single", 1)}


def load_shapes(Q, args, n_max):
    if args.autotune or not os.path.exists(args.tune_table):
        log(f"autotuning launch shapes up to {n_max}^3 (setup, not timed)")
        Q.autotune(n_max=n_max, both=True, reps=5, json_path=args.save_tune)
        return "autotuned on this GPU"
    Q.tune_load(args.tune_table)
    return os.path.relpath(args.tune_table, HERE)


class Oracle513:
    """The CPU oracle on the headline workload: timed, and kept as the
    reference potentials of the 513^3 legs."""

    def __init__(self, p, threads):
        import oracle as O
        self.threads = threads
        prev = O.set_threads(threads)
        try:
            c0 = time.perf_counter()
            r = O.run_pipeline(O.OracleConfig(n=N3, box_side=[L3], tol_rel=1e-10), p.x, p.y, p.z, p.m, p.total_mass)
            c1 = time.perf_counter()
            O.gather(r.phi, [L3], p.x, p.y, p.z, M=p.total_mass, mond=True)
            c2 = time.perf_counter()
        finally:
            O.set_threads(prev)
        self.seconds = c2 - c0
        self.gather_seconds = c2 - c1
        self.phin, self.phi = r.phin[0], r.phi[0]
        self.cycles = (r.info_newton[0][2], r.info_mond[0][2])


def headline(Q, torch, np, x, y, z, m, M, steps, warmup, orc):
    """The 513^3 FP64 step to 1e-10: timed steps with the finest-level
    smoother's launches bracketed by hipEvents, then one step with events
    between its phases (deposit, solves, gather)."""
    ctx = Q.Context(Q.Config(n=N3, box_side=[L3], tol_rel=1e-10), stream=torch.cuda.current_stream())
    infos = {}

    def step():
        ctx.deposit(x, y, z, m, M, count_outside=False)
        infos["newton"], infos["mond"] = ctx.solve()
        ctx.gather_forces(x, y, z, 1, with_box=False)

    log(f"513^3 FP64: warmup {warmup}")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile_enable(True, level_n=N3)
    log(f"513^3 FP64: timing {steps} steps")
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    st = ctx.profile_read()
    ctx.profile_enable(False)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    ctx.deposit(x, y, z, m, M, count_outside=False)
    ev[1].record()
    ctx.solve()
    ev[2].record()
    ctx.gather_forces(x, y, z, 1, with_box=False)
    ev[3].record()
    torch.cuda.synchronize()
    phase = [ev[i].elapsed_time(ev[i + 1]) for i in range(3)]
    npart = x.numel()
    rec = {"ms": ms, "relres_newton": infos["newton"]["relres"][0], "relres_mond": infos["mond"]["relres"][0],
           "vcycles_after_fmg": [infos["newton"]["vcycles"][0], infos["mond"]["vcycles"][0]],
           "phases_ms": {"deposit": phase[0], "solves": phase[1], "gather": phase[2]},
           "deposit_particles_per_s": npart / (phase[0] * 1e-3), "gather_particles_per_s": npart / (phase[2] * 1e-3)}
    if orc is not None:
        rec["err_vs_oracle"] = {"phi_n": rel(ctx.get_field(0, Q.FIELD_PHI_N).cpu().numpy(), orc.phin),
                                "phi": rel(ctx.get_field(0, Q.FIELD_PHI).cpu().numpy(), orc.phi)}
        rec["oracle_vcycles_after_fmg"] = list(orc.cycles)
    ctx.close()
    torch.cuda.empty_cache()
    return rec, st


def to_1e6_513(Q, torch, np, x, y, z, m, M, orc, reps=3):
    """The metric's second part on the 513^3 workload: wall time of deposit +
    both solves to a 1e-6 FP64 relative residual + gather, for plain FP64 with
    the paper's 6 cycles per FMG level, plain FP64 with 2 cycles per level (a
    plain baseline that does no more than the target needs) and mixed
    precision (FP32 multigrid, FP64 refinement); each with its error against
    the oracle's FP64 potentials."""
    out = {"workload": "two-component disk, 1e7 particles, one 513^3 box of 120 kpc, solves to 1e-6"}
    for name, prec, ncyc in (("fp64", Q.QUMOND_FP64, 6), ("fp64_2cyc", Q.QUMOND_FP64, 2),
                             ("mixed", Q.QUMOND_MIXED, 2)):
        ctx = Q.Context(Q.Config(n=N3, box_side=[L3], precision=prec, tol_rel=1e-6, ncycle_fmg=ncyc))
        times = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.deposit(x, y, z, m, M, count_outside=False)
            i_n, i_m = ctx.solve()
            ctx.gather_forces(x, y, z, 1, with_box=False)
            torch.cuda.synchronize()
            if r:
                times.append((time.perf_counter() - t0) * 1e3)
        rec = {"ms": float(np.median(times)), "ncycle_fmg": ncyc,
               "relres_newton": i_n["relres"][0], "relres_mond": i_m["relres"][0],
               "cycles_newton": i_n["vcycles"][0], "cycles_mond": i_m["vcycles"][0]}
        if orc is not None:
            rec["err_vs_oracle"] = {"phi_n": rel(ctx.get_field(0, Q.FIELD_PHI_N).cpu().numpy(), orc.phin),
                                    "phi": rel(ctx.get_field(0, Q.FIELD_PHI).cpu().numpy(), orc.phi)}
        out[name] = rec
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    out["speedup_mixed_vs_fp64"] = out["fp64"]["ms"] / out["mixed"]["ms"]
    out["speedup_mixed_vs_fp64_2cyc"] = out["fp64_2cyc"]["ms"] / out["mixed"]["ms"]
    log(f"513^3 to 1e-6: fp64 {out['fp64']['ms']:.1f} ms, fp64 2-cycle {out['fp64_2cyc']['ms']:.1f} ms, "
        f"mixed {out['mixed']['ms']:.1f} ms")
    return out


def nested_129(Q, synth, torch, np, steps, warmup):
    """The nested 129^3 step: the same disk with 1e6 particles in four 129^3
    boxes of 400/200/100/50 kpc, FP64 to 1e-10; smoother launches of all
    levels timed with hipEvents in a second pass of the same steps."""
    n, sides = 129, [400.0, 200.0, 100.0, 50.0]
    p = synth.two_component_disk(1_000_000, synth.seed_for(2))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x, y, z, m = dev(p.x), dev(p.y), dev(p.z), dev(p.m)
    ctx = Q.Context(Q.Config(n=n, box_side=sides, tol_rel=1e-10), stream=torch.cuda.current_stream())

    def step():
        ctx.deposit(x, y, z, m, p.total_mass, count_outside=False)
        ctx.solve()
        ctx.gather_forces(x, y, z, 1, with_box=False)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ctx.profile_enable(True)
    for _ in range(steps):
        step()
    st = ctx.profile_read()
    ctx.profile_enable(False)
    ctx.close()
    avg = st["total_ms"] / max(st["launches"], 1)
    per = st["alg_bytes"] / max(st["launches"], 1)
    out = {"workload": "two-component disk, 1e6 particles, 4 nested 129^3 boxes (400/200/100/50 kpc), monopole "
                       "outer BC, FP64 FMG to 1e-10",
           "ms_per_step": ms, "grid_pts_per_s": 4 * n ** 3 / (ms * 1e-3),
           "smoother_all_levels": {"launches_per_step": st["launches"] // steps, "avg_launch_us": avg * 1e3,
                                   "alg_bytes_per_launch": per,
                                   "achieved_GBs": per / (avg * 1e-3) / 1e9 if avg > 0 else None}}
    log(f"nested 129^3 step: {ms:.2f} ms")
    torch.cuda.empty_cache()
    return out


def batched_fit(Q, synth, torch, np, reps=3, refine_iters=3):
    """The batched rotation-curve fit: 64 two-component disks on the seeded
    parameter grid (M/L 0.3-1.2, z* 0.1-0.6 kpc, z_g 0.05-0.5 kpc, distance
    +-20%, 2e5-2e6 particles), grids 129^3 or 257^3 in a 120 kpc box, mixed
    precision to 1e-6, one captured hipGraph per run (plus the tail check),
    smoother shapes autotuned on the batch's own grids.  Particles are drawn
    on the GPU and resident before timing."""
    params = synth.fit_grid(64, config=4)
    ns = [dp.n_grid for dp in params]
    R = [0.5 * k for k in range(1, 61)]
    b = Q.Batch(Q.BatchConfig(box_side=120.0, refine_iters=refine_iters, tol_rel=1e-6, autotune=True), ns, R)
    keep, npart = [], 0
    for i, dp in enumerate(params):
        d = dp.dist
        x, y, z, m = synth.two_component_disk_torch(dp.n_particles, dp.seed, Md=dp.ml * 5e10 * d * d, Rd=3.0 * d,
                                                    zd=dp.z_star, Mg=1e10 * d * d, Rg=6.0 * d, zg=dp.z_gas)
        b.set_particles(i, x, y, z, m, float(m.sum().item()))
        keep.append((x, y, z, m))
        npart += dp.n_particles
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = b.run(use_graph=True)            # autotune + capture + first replay (setup)
    t_setup = (time.perf_counter() - t0) * 1e3
    time.sleep(0.5)                         # a host pause that marks the timed replays in a kernel trace
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = b.run(use_graph=True)
        times.append((time.perf_counter() - t0) * 1e3)
    time.sleep(0.5)                         # ... and their end
    t0 = time.perf_counter()
    b.run(use_graph=False)
    t_eager = (time.perf_counter() - t0) * 1e3
    pts = sum(n ** 3 for n in ns)
    ms = float(np.median(times))
    d = b.describe()
    out = {"workload": "64 two-component disks (seeded fit grid), 129^3/257^3 boxes of 120 kpc, mixed precision "
                       f"({refine_iters} FP64 refinement steps in the graph, tail to 1e-6)",
           "problems": 64, "n_257": ns.count(257), "n_129": ns.count(129), "grid_pts": pts, "particles": npart,
           "ms_per_run": ms, "grid_pts_per_s": pts / (ms * 1e-3), "particles_per_s": npart / (ms * 1e-3),
           "ms_eager": t_eager, "ms_first_run_with_tune_and_capture": t_setup, "graph_nodes": d["graph_nodes"],
           "converged": int(sum(i["converged"] for i in info)),
           "max_relres_newton": max(i["relres_newton"] for i in info),
           "max_relres_mond": max(i["relres_mond"] for i in info),
           "tail_steps": int(sum(i["steps_newton"] + i["steps_mond"] - 2 * refine_iters for i in info)),
           "device_gb": d["device_bytes"] / 1e9}
    log(f"batched fit: {ms:.1f} ms per run of 64 disks ({pts / (ms * 1e-3):.3g} grid-pts/s), "
        f"eager {t_eager:.1f} ms, {out['converged']}/64 converged")
    b.close()
    del keep
    torch.cuda.empty_cache()
    return out


def kuzmin_paper_mode(Q, synth, torch, np, dev):
    """The paper's accuracy experiment (Sec. 3.1): stratified Kuzmin disks,
    nested 257^3 boxes halving from 2^10 times the finest box, zero outer
    potential, box choice R < L/5; largest relative error of the midplane
    circular speed against the closed-form curves, and the wall time of
    deposit + both solves."""
    G, a0 = 4.300917270e-6, 3600.0

    def vc2_newton(R, a, M):   # Sec. 3.1: |g_N,R| = G M R (R^2 + a^2)^-3/2 in the midplane
        return G * M * R * R * (R * R + a * a) ** -1.5

    def vc2_qumond(R, a, M):   # Sec. 3.1: nu(|g_N,r| / a0) |g_N,R| with |g_N,r| = G M / (R^2 + a^2)
        y = G * M / (R * R + a * a) / a0
        return (0.5 + 0.5 * np.sqrt(1.0 + 4.0 / y)) * vc2_newton(R, a, M)

    out = {}
    for name, a, M, finest, nbox in (("a1.5kpc_M1e10_boxes4096to4kpc", 1.5, 1e10, 4.0, 11),
                                     ("a150pc_M1e9_boxes4096to0.5kpc", 0.15, 1e9, 0.5, 14)):
        p = synth.kuzmin_disk_stratified(20_000_000, a, M)
        sides = [finest * 2 ** k for k in range(nbox - 1, -1, -1)]
        ctx = Q.Context(Q.Config(n=257, box_side=sides, outer_bc=Q.QUMOND_BC_ZERO, tol_rel=1e-10))
        x, y, z, m = dev(p.x), dev(p.y), dev(p.z), dev(p.m)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.deposit(x, y, z, m, M, count_outside=False)
        ctx.solve()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        R = np.geomspace(0.03, 30.0, 48)
        rec = {"boxes": nbox, "n": 257, "particles": 20_000_000, "ms": ms}
        for which, fn, tag in ((0, vc2_newton, "newton"), (1, vc2_qumond, "qumond")):
            vc2 = ctx.rotation_curve(dev(R), 64, which).cpu().numpy()
            err = np.abs(np.sqrt(vc2 / fn(R, a, M)) - 1.0)
            for r0 in (0.05, 0.3, 1.0):
                rec[f"{tag}_max_err_R_ge_{r0}kpc"] = float(err[R >= r0].max())
        out[name] = rec
        ctx.close()
        del ctx, x, y, z, m
        torch.cuda.empty_cache()
    log("Kuzmin paper mode: " + ", ".join(f"{k}: qumond {v['qumond_max_err_R_ge_0.3kpc']:.1e} (R>=0.3), "
                                          f"{v['qumond_max_err_R_ge_1.0kpc']:.1e} (R>=1)" for k, v in out.items()))
    return out


def disk_experiments(Q, synth, torch, np, dev):
    """The exponential-disk experiments in the paper's nesting (eleven 257^3
    boxes, 4096 kpc down to 4 kpc, zero outer potential): Sec. 3.3's thin
    versus 1 kpc sech^2 disk (R_d = 1.5 kpc, 1e10 Msun) with QUMOND against the
    algebraic relation of Eq. 3, and the Eq. 5 vertical dispersion at one
    scale height of a stellar disk (R_d = 3 kpc, 5e10 Msun, z0 = 0.3 kpc)."""
    sides = [4.0 * 2 ** k for k in range(10, -1, -1)]
    R = np.array([0.5, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 8.0, 10.0, 15.0])

    def solve(p, M):
        ctx = Q.Context(Q.Config(n=257, box_side=sides, outer_bc=Q.QUMOND_BC_ZERO, tol_rel=1e-10))
        x, y, z, m = dev(p.x), dev(p.y), dev(p.z), dev(p.m)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.deposit(x, y, z, m, M, count_outside=False)
        ctx.solve()
        torch.cuda.synchronize()
        return ctx, (time.perf_counter() - t0) * 1e3

    out = {"R_kpc": R.tolist(), "boxes": len(sides), "n": 257, "particles": 20_000_000}
    v = {}
    for z0 in (0.0, 1.0):
        ctx, ms = solve(synth.exponential_disk_stratified(20_000_000, 1.5, 1e10, z0), 1e10)
        for w, tag in ((Q.WHICH_NEWTON, "newton"), (Q.WHICH_QUMOND, "qumond"), (Q.WHICH_ALGEBRAIC, "algebraic")):
            v[(z0, tag)] = np.sqrt(ctx.rotation_curve(dev(R), 64, w).cpu().numpy())
        out[f"ms_deposit_and_solves_z0_{z0:g}"] = ms
        ctx.close()
        torch.cuda.empty_cache()
    out["thin_vc_kms"] = {t: v[(0.0, t)].round(3).tolist() for t in ("newton", "qumond", "algebraic")}
    out["thick_1kpc_vc_kms"] = {t: v[(1.0, t)].round(3).tolist() for t in ("newton", "qumond", "algebraic")}
    out["qumond_minus_algebraic_thin_kms"] = (v[(0.0, "qumond")] - v[(0.0, "algebraic")]).round(3).tolist()
    out["thin_minus_thick_qumond_kms"] = (v[(0.0, "qumond")] - v[(1.0, "qumond")]).round(3).tolist()

    ctx, ms = solve(synth.exponential_disk_stratified(20_000_000, 3.0, 5e10, 0.3), 5e10)
    sig = {}
    for w, tag in ((Q.WHICH_NEWTON, "newton"), (Q.WHICH_QUMOND, "qumond")):
        sig[tag] = np.sqrt(ctx.sigma_z(dev(R), 0.3, 0.3, naz=32, which=w).cpu().numpy()).round(3).tolist()
    ctx.close()
    torch.cuda.empty_cache()
    out["sigma_z_at_z0_kms"] = sig
    out["sigma_z_disk"] = "exponential, R_d = 3 kpc, 5e10 Msun, sech^2 z0 = 0.3 kpc, evaluated at |z| = z0"
    d = out["thin_minus_thick_qumond_kms"]
    log(f"disk experiments: thin - thick up to {max(d):.1f} km/s, {d[6]:.1f} at 6 kpc; QUMOND - algebraic "
        f"{min(out['qumond_minus_algebraic_thin_kms']):.1f} km/s at most; sigma_z(0.5 kpc) "
        f"{sig['qumond'][0]:.1f} km/s QUMOND, {sig['newton'][0]:.1f} Newton")
    return out


def learned_leg(Q, torch, np, count=8, oracle_threads=1):
    """Wall time and V-cycles of the QUMOND solve to 1e-6 on held-out disks
    (seed family 6, 129^3, 120 kpc) for the plain FP64 FMG with 6, 2 and 1
    cycles per level, FP64 V-cycles from zero / Phi_N / the trained network's
    prediction, the mixed FMG and the network's prediction followed by
    mixed-precision refinement (inference time included where the prediction
    is used); each variant's potential against the FP64 oracle's (deposit,
    both solves to 1e-10) on the same particles, when oracle_threads > 0."""
    from paper_1201_3185_amd import learned
    ckpt = os.path.join(HERE, "paper_1201_3185_amd", "weights", "unet129.npy")
    if not os.path.exists(ckpt):
        return None
    net = Q.UNet(129, seed=0)
    net.set_params(np.load(ckpt))
    params = learned.disk_set(count, config=6)
    judge = None
    if oracle_threads > 0:
        import oracle as O
        refs = {}

        def judge(i, phi):
            if i not in refs:
                x, y, z, m = (t.cpu().numpy() for t in learned._disk_tensors(params[i]))
                prev = O.set_threads(oracle_threads)
                try:
                    o = O.run_pipeline(O.OracleConfig(n=129, box_side=[120.0], tol_rel=1e-10), x, y, z, m,
                                       float(m.sum()))
                finally:
                    O.set_threads(prev)
                refs[i] = o.phi[0]
            return rel(phi.cpu().numpy(), refs[i])

    g = learned.gain(net, params, judge=judge)
    g["workload"] = (f"{count} held-out two-component disks (fit parameter ranges), one 129^3 box of 120 kpc, "
                     "QUMOND solve to 1e-6 from the same Phi_N and source")
    g["speedup_vs_fmg"] = {k: g["fmg"]["ms"] / g[k]["ms"] for k in learned.VARIANTS}
    g["speedup_vs_fmg2"] = {k: g["fmg2"]["ms"] / g[k]["ms"] for k in learned.VARIANTS}
    log("learned guess: " + ", ".join(f"{k} {g[k]['ms']:.2f} ms" for k in learned.VARIANTS) +
        f", inference {g['infer_ms']:.2f} ms")
    net = None
    torch.cuda.empty_cache()
    return g


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the oracle's node-parallel loops (0: min(16, logical cores))")
    ap.add_argument("--no-mixed", action="store_true", help="skip the 513^3 legs to 1e-6")
    ap.add_argument("--no-nested", action="store_true", help="skip the nested 129^3 step")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-disk batched fit")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-guess comparison")
    ap.add_argument("--no-kuzmin", action="store_true", help="skip the paper-mode Kuzmin accuracy run")
    ap.add_argument("--no-disks", action="store_true",
                    help="skip the paper-mode thickness, algebraic-MOND and sigma_z experiments")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the 513^3 FP64 steps (no oracle, no other legs): the command the kernel traces and "
                         "counter runs profile")
    ap.add_argument("--tune-table", default=LAUNCH_TABLE,
                    help="launch-shape table to load (default: the committed MI355X table)")
    ap.add_argument("--autotune", action="store_true", help="autotune the launch shapes instead of loading a table")
    ap.add_argument("--save-tune", default=None, help="with --autotune: write the table to this JSON file")
    ap.add_argument("--mixed-only", action="store_true",
                    help="only the 513^3 legs to 1e-6 (FP64 6- and 2-cycle, mixed; no oracle) and print their record")
    ap.add_argument("--nested-only", action="store_true",
                    help="only the nested 129^3 step (after loading the launch table) and print its record")
    ap.add_argument("--batch-profile", action="store_true",
                    help="run only the batched-fit leg (for a kernel trace of its replays) and print its record")
    ap.add_argument("--learned-profile", action="store_true",
                    help="run only the learned-guess leg on 4 held-out disks without the oracle (for a kernel "
                         "trace of the U-Net inference) and print its record")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device to device three times (a known-size copy that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--calibrate-own", action="store_true",
                    help="only run the library's prolong-add kernel three times on a 513^3 grid (reads 9 B and "
                         "writes 8 B per fine node: a second, own-kernel scale for the counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): this build has no multi-GPU path; "
              "sharding the boxes or the batch over GPUs is a design that is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    sys.path.insert(0, HERE)
    from paper_1201_3185_amd import qumond as Q
    from paper_1201_3185_amd import synth

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        ms = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.copy_(a)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        t = min(ms)
        print(json.dumps({"calibration_copy_bytes": a.numel() * 8, "copies": 3, "best_ms": t,
                          "read_plus_write_GBs": 2 * a.numel() * 8 / (t * 1e-3) / 1e9}), flush=True)
        return
    if args.calibrate_own:
        nc = (N3 + 1) // 2
        uc = torch.ones((nc, nc, nc), dtype=torch.float64, device="cuda")
        uf = torch.zeros((N3, N3, N3), dtype=torch.float64, device="cuda")
        for _ in range(3):
            Q.k_prolong_add(uc, uf)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_kernel": "prolong_k<double, true>", "fine_interior_nodes": (N3 - 2) ** 3,
                          "coarse_nodes": nc ** 3, "launches": 3}), flush=True)
        return
    if args.batch_profile:
        print(json.dumps(batched_fit(Q, synth, torch, np, reps=2)), flush=True)
        return
    if args.learned_profile:
        load_shapes(Q, args, 129)
        print(json.dumps(learned_leg(Q, torch, np, count=4, oracle_threads=0)), flush=True)
        return
    if args.nested_only:
        load_shapes(Q, args, 129)
        print(json.dumps(nested_129(Q, synth, torch, np, args.steps, args.warmup)), flush=True)
        return

    shapes_from = load_shapes(Q, args, N3)
    log(f"generating {NP3} particles")
    p = synth.two_component_disk(NP3, synth.seed_for(3))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x, y, z, m = dev(p.x), dev(p.y), dev(p.z), dev(p.m)
    M = p.total_mass
    if args.mixed_only:
        print(json.dumps(to_1e6_513(Q, torch, np, x, y, z, m, M, None)), flush=True)
        return

    orc, cpu = None, None
    model, ncores = host_cpu()
    threads = args.cpu_threads if args.cpu_threads > 0 else max(1, min(16, ncores))
    if not args.no_cpu_baseline and not args.headline_only:
        log(f"CPU oracle on the full 513^3 workload ({threads} threads)")
        orc = Oracle513(p, threads)
        cpu = {"value": N3 ** 3 / orc.seconds, "unit": "grid-pts/s", "cores": threads, "kind": "oracle",
               "sample": f"the full headline workload (deposit of 1e7 particles, both FMG solves to 1e-10, source, "
                         f"gather at all particles) in {orc.seconds:.1f} s; node-parallel loops on {threads} threads, "
                         f"deposit and sums serial",
               "cpu_model": model, "host_logical_cores": ncores}
        log(f"oracle: {orc.seconds:.1f} s")

    head, st = headline(Q, torch, np, x, y, z, m, M, args.steps, args.warmup, orc)
    ms = head["ms"]
    value = N3 ** 3 / (ms * 1e-3)
    avg_ms = st["total_ms"] / max(st["launches"], 1)
    per_launch = st["alg_bytes"] / max(st["launches"], 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    sweeps = st.get("sweeps_per_launch", 1) or 1
    if sweeps == 2:
        kern = ("red-black smoother, finest (513^3) level: the skewed two-sweep launches (rbgs2_skew_k: the "
                "pre-smoothing pair of each V-cycle in one pass; the post-smoothing pair, which also applies the "
                "coarse-grid correction in its launch, is left out; 24 B per node per launch of two sweeps), FP64")
    else:
        kern = ("red-black smoother, finest (513^3) level, plain sweeps (one per launch; the first "
                "post-smoothing sweep, which also applies the coarse-grid correction, is left out), FP64 "
                "(24 B per node)")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": smoother_traffic("fp64_513", sweeps),
            "kernel": kern, "sweeps_per_launch": sweeps,
            "launches_per_step": st["launches"] // args.steps, "avg_launch_us": round(avg_ms * 1e3, 2),
            "alg_bytes_per_launch": per_launch}
    if sweeps == 2:
        roof["single_sweep"] = single_sweep_roofline(Q, torch)
    log(f"513^3 FP64 step {ms:.2f} ms, {value:.4g} grid-pts/s; finest smoother {st['launches']} launches, "
        f"avg {avg_ms * 1e3:.1f} us, {achieved:.0f} GB/s algorithmic")

    legs = {}
    if not args.headline_only:
        if not args.no_mixed:
            legs["to_1e-6_513"] = to_1e6_513(Q, torch, np, x, y, z, m, M, orc)
        del x, y, z, m
        torch.cuda.empty_cache()
        orc_threads = threads if not args.no_cpu_baseline else 0
        orc = None
        if not args.no_nested:
            legs["nested_129"] = nested_129(Q, synth, torch, np, args.steps, args.warmup)
        if not args.no_batch:
            legs["batched_fit_64"] = batched_fit(Q, synth, torch, np)
        if not args.no_learned:
            legs["learned_guess_129"] = learned_leg(Q, torch, np, oracle_threads=orc_threads)
        if not args.no_kuzmin:
            legs["kuzmin_paper_mode_257"] = kuzmin_paper_mode(Q, synth, torch, np, dev)
        if not args.no_disks:
            legs["exponential_disks_paper_mode_257"] = disk_experiments(Q, synth, torch, np, dev)

    out = {
        "metric": METRIC, "value": value, "unit": "grid-pts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "two-component exponential disk, 1e7 particles, one 513^3 box of 120 kpc, monopole "
                               "outer BC, FP64 FMG (2+2 RB-GS, 6 V-cycles per level) to 1e-10, deposit + both "
                               "solves + gather at all particles",
                   "n": N3, "box_kpc": L3, "particles": NP3, "tol_rel": 1e-10, "ncycle_fmg": 6, "npre": 2,
                   "npost": 2, "precision": "fp64", "launch_shapes": shapes_from},
        "headline_513": head,
        "roofline": roof, "cpu_baseline": cpu,
    }
    out.update(legs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

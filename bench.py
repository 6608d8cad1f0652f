#!/usr/bin/env python3
"""Throughput of the particle-mesh QUMOND solve on one MI355X.

One step is one pass of the whole path over one synthetic galaxy already
resident in HBM: CIC deposit -> Newtonian FMG -> Eq. 2 source -> QUMOND FMG ->
force gather at every particle, all through the C ABI of libqumond.so
(qumond_deposit, qumond_solve -- which overlaps the QUMOND chain of box b with
the Newtonian solve of box b+1 -- and qumond_gather_forces).

Workload: two-component exponential disk (stars Md = 5e10 Msun, Rd = 3 kpc,
sech^2 height 0.3 kpc; gas Mg = 1e10 Msun, Rg = 6 kpc, height 0.15 kpc),
1e6 particles, four nested 129^3 boxes of 400/200/100/50 kpc with a monopole
outer boundary, 2+2 red-black sweeps and 6 V-cycles per FMG level, both solves
to 1e-10 relative residual, in FP64.

value = grid points of all boxes / wall time of one step (host syncs of the
stopping tests included).  The roofline object reports the red-black
smoother (the dominant kernel): algorithmic bytes (read u, read f, write u)
of its launches divided by their summed durations, from hipEvents recorded by
the library around each launch on the solve's stream during a second pass of
the same K steps.  cpu_baseline times the CPU oracle (single thread) on one
full step of the same workload.

Further legs (same JSON line, not the headline value): the 513^3 disk to 1e-6
in FP64 and in mixed precision; the batched fit (64 disks of 129^3/257^3 in one
captured graph); the learned initial guess on held-out 129^3 disks.
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
METRIC = "QUMOND solve grid-pts/s & wall time to 1e-6 rel residual: plain FP64 vs mixed+learned"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def smoother_traffic(per_launch_alg_bytes):
    """HBM traffic per smoother launch from committed rocprofv3 counter runs,
    valid only while the kernel source is unchanged (null otherwise)."""
    path = os.path.join(HERE, "profiles", "smoother_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(HERE, "paper_1201_3185_amd", "csrc", "grid_kernels.hip"), "rb").read()
    if rec.get("grid_kernels_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return rec.get("bytes_per_launch")


def mixed_vs_fp64(Q, synth, torch, np, dev, reps=3, profile=False):
    """The metric's second part on the 513^3 workload (two-component disk,
    1e7 particles, 120 kpc box, monopole boundary): wall time of deposit +
    both solves (to 1e-6 FP64 relative residual) + gather, plain FP64 against
    FP32 multigrid with FP64 refinement, and the 513^3 smoother's HBM roofline
    from the FP64 run's smoother launches.  With profile=True only the mixed
    case runs, its timed repetitions between two 0.5 s host pauses (for a
    kernel trace of them)."""
    n, L = 513, 120.0
    log("513^3 workload: 1e7 particles")
    p = synth.two_component_disk(10_000_000, synth.seed_for(3))
    x, y, z, m = dev(p.x), dev(p.y), dev(p.z), dev(p.m)
    out = {"workload": "two-component disk, 1e7 particles, one 513^3 box of 120 kpc, solves to 1e-6"}
    fields = {}
    Q.autotune(n_max=n, both=True, reps=3)
    # plain: the paper's 6 V-cycles per FMG level in FP64; same short schedule in FP64
    # for comparison; mixed: 2 FP32 cycles per FMG level, then FP64 refinement
    cases = (("fp64", Q.QUMOND_FP64, 6), ("fp64_2cyc", Q.QUMOND_FP64, 2), ("mixed", Q.QUMOND_MIXED, 2))
    for name, prec, ncyc in (cases[2:] if profile else cases):
        ctx = Q.Context(Q.Config(n=n, box_side=[L], precision=prec, tol_rel=1e-6, ncycle_fmg=ncyc))
        times = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            if profile and r == 1:
                time.sleep(0.5)
            t0 = time.perf_counter()
            ctx.deposit(x, y, z, m, p.total_mass, count_outside=False)
            i_n, i_m = ctx.solve()
            ctx.gather_forces(x, y, z, 1, with_box=False)
            torch.cuda.synchronize()
            if r:
                times.append((time.perf_counter() - t0) * 1e3)
        if profile:
            time.sleep(0.5)
        rec = {"ms": float(np.median(times)), "ncycle_fmg": ncyc,
               "relres_newton": i_n["relres"][0], "relres_mond": i_m["relres"][0],
               "cycles_newton": i_n["vcycles"][0], "cycles_mond": i_m["vcycles"][0]}
        if name == "fp64":
            ctx.profile_enable(True)
            ctx.deposit(x, y, z, m, p.total_mass, count_outside=False)
            ctx.solve()
            st = ctx.profile_read()
            ctx.profile_enable(False)
            gbs = st["alg_bytes"] / (st["total_ms"] * 1e-3) / 1e9
            rec["smoother_roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                        "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                                        "launches": st["launches"],
                                        "avg_launch_us": round(1e3 * st["total_ms"] / max(st["launches"], 1), 2)}
        fields[name] = ctx.get_field(0, Q.FIELD_PHI).cpu().numpy()
        out[name] = rec
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    if profile:
        log(f"513^3 mixed: {out['mixed']['ms']:.1f} ms per run")
        return out
    out["mixed_err_vs_fp64"] = float(np.abs(fields["mixed"] - fields["fp64"]).max() / np.abs(fields["fp64"]).max())
    out["mixed_err_vs_fp64_2cyc"] = float(np.abs(fields["mixed"] - fields["fp64_2cyc"]).max() /
                                          np.abs(fields["fp64_2cyc"]).max())
    out["speedup_mixed"] = out["fp64"]["ms"] / out["mixed"]["ms"]
    out["speedup_mixed_same_schedule"] = out["fp64_2cyc"]["ms"] / out["mixed"]["ms"]
    log(f"513^3: fp64 {out['fp64']['ms']:.1f} ms, mixed {out['mixed']['ms']:.1f} ms, "
        f"err {out['mixed_err_vs_fp64']:.2e}")
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
           "device_gb": d["device_bytes"] / 1e9, "shapes": d["classes"]}
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


def learned_leg(Q, torch, np, count=8):
    """Wall time and V-cycles of the QUMOND solve to 1e-6 on held-out disks
    (seed family 6, 129^3, 120 kpc) for the plain FP64 FMG, FP64 V-cycles from
    zero / Phi_N / the trained network's prediction, the mixed FMG and the
    network's prediction followed by mixed-precision refinement; inference
    time is included where the prediction is used."""
    from paper_1201_3185_amd import learned
    ckpt = os.path.join(HERE, "paper_1201_3185_amd", "weights", "unet129.npy")
    if not os.path.exists(ckpt):
        return None
    net = Q.UNet(129, seed=0)
    net.set_params(np.load(ckpt))
    g = learned.gain(net, learned.disk_set(count, config=6))
    g["workload"] = (f"{count} held-out two-component disks (fit parameter ranges), one 129^3 box of 120 kpc, "
                     "QUMOND solve to 1e-6 from the same Phi_N and source")
    g["speedup_vs_fmg"] = {k: g["fmg"]["ms"] / g[k]["ms"] for k in learned.VARIANTS}
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
    ap.add_argument("--no-profile-pass", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the 513^3 FP64-vs-mixed comparison")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-disk batched fit")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-guess comparison")
    ap.add_argument("--no-kuzmin", action="store_true", help="skip the paper-mode Kuzmin accuracy run")
    ap.add_argument("--no-disks", action="store_true",
                    help="skip the paper-mode thickness, algebraic-MOND and sigma_z experiments")
    ap.add_argument("--save-tune", default=None, help="write the autotuned smoother table to this JSON file")
    ap.add_argument("--tune-table", default=None, help="load the smoother table from this JSON file instead of "
                                                       "autotuning (to replay the same launches under a profiler)")
    ap.add_argument("--graphs", type=int, default=0,
                    help="1: the nested step replays its FMG schedules from captured HIP graphs (use_graphs); 0: eager")
    ap.add_argument("--batch-profile", action="store_true",
                    help="run only the batched-fit leg (for a kernel trace of its replays) and print its record")
    ap.add_argument("--mixed-profile", action="store_true",
                    help="run only the 513^3 mixed-precision case (timed runs between host pauses) and print its "
                         "record")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device to device three times (the known-size kernel that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
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
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": a.numel() * 8, "copies": 3}), flush=True)
        return
    if args.batch_profile:
        print(json.dumps(batched_fit(Q, synth, torch, np, reps=2)), flush=True)
        return
    if args.mixed_profile:
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        print(json.dumps(mixed_vs_fp64(Q, synth, torch, np, dev, reps=2, profile=True)), flush=True)
        return
    n, sides, npart = 129, [400.0, 200.0, 100.0, 50.0], 1_000_000
    log(f"generating {npart} particles")
    p = synth.two_component_disk(npart, synth.seed_for(2))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x, y, z, m = dev(p.x), dev(p.y), dev(p.z), dev(p.m)
    M = p.total_mass
    if args.tune_table:
        log(f"loading smoother launch shapes from {args.tune_table}")
        Q.tune_load(args.tune_table)
    else:
        log("autotuning smoother launch shapes (setup, not timed)")
        Q.autotune(n_max=n, both=False, reps=5, json_path=args.save_tune)
    shapes = {str(k): {"single": Q.tune_get(k), "fused": Q.tune_get_fused(k)} for k in (33, 65, 129)}
    cfg = Q.Config(n=n, box_side=sides, tol_rel=1e-10, use_graphs=args.graphs)
    # graphs need a stream of the step's own (the null stream cannot be captured)
    stream = torch.cuda.Stream() if args.graphs else torch.cuda.current_stream()
    stream.wait_stream(torch.cuda.current_stream())
    ctx = Q.Context(cfg, stream=stream)
    infos = {}

    def step():
        with torch.cuda.stream(stream):
            ctx.deposit(x, y, z, m, M, count_outside=False)
            infos["newton"], infos["mond"] = ctx.solve()   # source + both FMG chains, overlapped
            return ctx.gather_forces(x, y, z, 1, with_box=False)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    pts = len(sides) * n ** 3
    value = pts / (ms * 1e-3)
    log(f"{ms:.3f} ms/step, {value:.4g} grid-pts/s")

    roof = None
    if not args.no_profile_pass:
        ctx.profile_enable(True)
        for _ in range(args.steps):
            step()
        st = ctx.profile_read()
        ctx.profile_enable(False)
        avg_ms = st["total_ms"] / max(st["launches"], 1)
        per_launch = st["alg_bytes"] / max(st["launches"], 1)
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        tr = smoother_traffic(per_launch)
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
                "kernel": "red-black smoother launches, all levels (z-march and brick kernels, one or two sweeps per launch; 24 B/pt per launch)", "launches_per_step": st["launches"] // args.steps,
                "avg_launch_us": round(avg_ms * 1e3, 3), "alg_bytes_per_launch": per_launch}
        log(f"smoother: {st['launches']} launches, avg {avg_ms * 1e3:.2f} us, {achieved:.1f} GB/s algorithmic")

    mixed = None
    if not args.no_mixed:
        mixed = mixed_vs_fp64(Q, synth, torch, np, dev)

    batch = None
    if not args.no_batch:
        batch = batched_fit(Q, synth, torch, np)

    kuz = None
    if not args.no_kuzmin:
        kuz = kuzmin_paper_mode(Q, synth, torch, np, dev)

    disks = None
    if not args.no_disks:
        disks = disk_experiments(Q, synth, torch, np, dev)

    learned_out = None
    if not args.no_learned:
        learned_out = learned_leg(Q, torch, np)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        log("timing the CPU oracle on one full step")
        oc = O.OracleConfig(n=n, box_side=sides, tol_rel=1e-10)
        c0 = time.perf_counter()
        res = O.run_pipeline(oc, p.x, p.y, p.z, p.m, M)
        O.gather(res.phi, sides, p.x, p.y, p.z, M=M, mond=True)
        c1 = time.perf_counter()
        cpu = {"value": pts / (c1 - c0), "unit": "grid-pts/s", "cores": 1, "kind": "oracle",
               "sample": "one full step of the same workload (deposit, both FMG solves to 1e-10, source, "
                         f"gather of all particles) in {c1 - c0:.1f} s, single-threaded C"}
        log(f"oracle: {c1 - c0:.2f} s")

    out = {
        "metric": METRIC, "value": value, "unit": "grid-pts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "two-component exponential disk, 1e6 particles, 4 nested 129^3 boxes "
                               "(400/200/100/50 kpc), monopole outer BC, FP64 FMG to 1e-10",
                   "n": n, "boxes_kpc": sides, "particles": npart, "tol_rel": 1e-10, "ncycle_fmg": 6,
                   "npre": 2, "npost": 2, "precision": "fp64", "graphs": bool(args.graphs)},
        "vcycles_after_fmg": {"newton": infos["newton"]["vcycles"], "mond": infos["mond"]["vcycles"]},
        "smoother_shapes": shapes,
        "mixed_vs_fp64_513": mixed,
        "batched_fit_64": batch,
        "learned_guess_129": learned_out,
        "kuzmin_paper_mode_257": kuz,
        "exponential_disks_paper_mode_257": disks,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

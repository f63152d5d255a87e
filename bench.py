"""Benchmark: particle-updates/s of the SediFoam particle step + plain
diffusion averaging on one MI355X.

A bench step is one pass of the hot path: 10 velocity-Verlet particle steps
(neighbour binning/re-sort when due, contact + lubrication + fluid forces,
integration) followed by one averaging (PCM deposition + implicit diffusion
smoothing), as in the 1M-sphere bed workload (averaging every 10 steps).
Inputs are seeded synthetic beds resident in HBM before the timed region.

Prints one JSON line.  Extra objects: "roofline" (force kernel against the
HBM peak, from HIP events on the library's stream), "cpu_baseline" (the FP64
oracle on the host, a few steps of the same bed), "averaging" (plain solve
timings) and "phases".
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-updates/s at 1M/10M particles; averaging ms plain vs surrogate"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6


def averaging_rooflines(n, ncell, dep_ms, smooth_ms, direct, mesh, nch=4):
    """Deposition against HBM: the method's algorithmic bytes, 60 B per
    particle (position and radius 32 B, drag 24 B, ID 4 B) plus 8 B per cell
    and channel written; with the solid volume flux (7 channels) also the
    velocity, 24 B per particle.
    The plain solve against the method's algorithmic minimum: read raw and
    write smooth, 16 B per cell and channel, at HBM peak.  The direct solve's
    own work, a forward and an inverse transform along each axis (4 (nx + ny
    + nz) FLOP per cell and channel on the FP64 matrix cores), is given
    beside it.  The solve time includes its full-field residual check."""
    dep_bytes = (60 + (24 if nch == 7 else 0)) * n + 8 * nch * ncell
    dep = {"ms": round(dep_ms, 5), "bytes": int(dep_bytes), "bound": "hbm",
           "achieved_GBps": round(dep_bytes / (dep_ms * 1e-3) / 1e9, 1),
           "frac": round(dep_bytes / (dep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    min_bytes = 16 * ncell * nch
    sol = {"ms": round(smooth_ms, 5), "bound": "hbm", "bytes": int(min_bytes),
           "hbm_minimum_ms": round(min_bytes / HBM_PEAK_GBS / 1e6, 5),
           "achieved_GBps": round(min_bytes / (smooth_ms * 1e-3) / 1e9, 1),
           "frac": round(min_bytes / (smooth_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if direct:
        flop = 4 * (mesh[0] + mesh[1] + mesh[2]) * ncell * nch
        tf = flop / (smooth_ms * 1e-3) / 1e12
        sol["transforms"] = {"bound": "mfma_fp64", "gflop": round(flop / 1e9, 3),
                             "achieved_tflops": round(tf, 2),
                             "peak_tflops": FP64_MFMA_PEAK_TFLOPS,
                             "frac": round(tf / FP64_MFMA_PEAK_TFLOPS, 4)}
    return dep, sol


# HBM traffic of the step-mode force kernel on the 1M-sphere bed (FP64), from
# two rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE; KiB
# per dispatch, mean over the profiled step-mode dispatches), scaled by what
# the same counters read for a 1 GiB device copy (--copy-calibration: the
# copy's FETCH_SIZE reads 0.5x the bytes read, WRITE_SIZE 1.0x the bytes
# written).  Valid only for the kernel sources it was measured on.
FORCE_PMC = {
    ("bed1m", "fp64"): {
        "fetch_kib": 290952.6, "write_kib": 280519.1, "fetch_scale": 2.0, "write_scale": 1.0,
        "sources_sha256": "a9a4c805a345f3170f926cc8cd1f646cb74b7d0c953bba65b7e68550a8c1e1db",
        "profile": "profiles/k_forces_bed1m_fp64.md"},
}
FORCE_SOURCES = ("k_forces.hip", "k_common.h", "sedimi_internal.h")


def force_sources_sha():
    """Hash of the force kernel's sources with comments and blank lines
    removed: the stored HBM counters stay valid across comment edits and
    lapse with any change to the code."""
    h = hashlib.sha256()
    for f in FORCE_SOURCES:
        with open(os.path.join(ROOT, "paper_1601_03801_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def copy_calibration():
    """Three copies of a 1 GiB device buffer (the reference for the PMC byte
    counters)."""
    import torch
    x = torch.empty(256 * 2 ** 20, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("bench: copied 1 GiB three times", flush=True)


def force_bytes_per_particle(mean_nbr, mean_contacts, mixed):
    """Algorithmic HBM bytes of one force-kernel launch per particle:
    own state read (pos, vel, omg, acc: 4 x 32 B; id, count, mask: 12 B),
    its neighbour indices (4 B each), read + write of the tangential history
    of its active contacts (3 components), the state written back (vel, omg,
    acc, alpha, drag: 5 x 32 B; mask 4 B).  Neighbour states are the same
    arrays already counted once."""
    hist = (12 if mixed else 24) * 2
    return 140 + 4 * mean_nbr + hist * mean_contacts + 164


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed bench steps")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bed1m")
    ap.add_argument("--substeps", type=int, default=10)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--drag", default="difelice", choices=["difelice", "syamlal", "stokes"],
                    help="drag law of the particle step")
    ap.add_argument("--bandwidth-z", type=float, default=0.0,
                    help="averaging bandwidth across the bed in particle diameters "
                         "(0: the same as along it)")
    ap.add_argument("--lift", type=float, default=0.0,
                    help="shear-lift coefficient C_l (0: no lift; the paper's value is 1.6)")
    ap.add_argument("--solid-velocity", action="store_true",
                    help="also average the solid velocity U_s (7 averaged channels)")
    ap.add_argument("--scheme", default="euler", choices=["euler", "bdf2"],
                    help="pseudo-time scheme of the averaging")
    ap.add_argument("--cpu-steps", type=int, default=3, help="oracle steps for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--nn-train-steps", type=int, default=2000,
                    help="surrogate training snapshots (0 skips the surrogate section)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 1 GiB copy used to scale the PMC byte counters")
    ap.add_argument("--nn-alpha", type=float, default=1.0,
                    help="leaky-ReLU slope of the surrogate (1 makes the network linear)")
    ap.add_argument("--nn-groups", type=int, default=4, choices=[1, 4],
                    help="channel groups of the surrogate (4: one group of 8 per field)")
    ap.add_argument("--nn-lr", type=float, default=3e-4,
                    help="peak of the surrogate's cosine learning-rate schedule")
    ap.add_argument("--rebuilds", type=int, default=5,
                    help="forced neighbour-list rebuilds timed on the main bed")
    ap.add_argument("--bed10m-steps", type=int, default=20,
                    help="timed bench steps of the 10M-sphere mixed-precision bed "
                         "(0 skips it)")
    ap.add_argument("--nn-steps", type=int, default=10,
                    help="coupled steps (averaging every step) per averaging mode")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path "
              "has no multi-GPU mode", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import torch

    main_run = particle_bench(args, args.workload, args.precision, args.steps, args.warmup,
                              rebuilds=args.rebuilds, cpu_steps=0 if args.no_cpu_baseline
                              else args.cpu_steps)
    value, elapsed, n = main_run["value"], main_run["elapsed"], main_run["n"]
    K, W, S, prm = args.steps, args.warmup, args.substeps, main_run["prm"]
    mixed = args.precision == "mixed"
    torch.cuda.empty_cache()

    bed10m = None
    if args.workload == "bed1m" and args.bed10m_steps > 0:
        r = particle_bench(args, "bed10m", "mixed", args.bed10m_steps, 2, rebuilds=0,
                           cpu_steps=0)
        bed10m = {"workload": "bed10m", "particles": r["n"], "mesh": r["mesh"],
                  "precision": "mixed", "dtype": "f64-state/f32-forces",
                  "value": round(r["value"], 1), "unit": "particle-updates/s",
                  "steps": r["steps"], "particle_steps": r["steps"] * S,
                  "ms_per_step": round(1000 * r["elapsed"] / r["steps"], 4),
                  "roofline": r["roofline"], "averaging_ms": r["averaging"]["plain_ms"],
                  "averaging": r["averaging"], "particle_step_only": r["particle_step_only"],
                  "stats": r["stats"]}
        print(f"bench: bed10m mixed {bed10m['value']:.4e} particle-updates/s", file=sys.stderr,
              flush=True)
        torch.cuda.empty_cache()

    surrogate = None
    if args.nn_train_steps > 0:
        surrogate = surrogate_section(args)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "particle-updates/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(1000 * elapsed / K, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if not mixed else "f64-state/f32-forces", "data": "synthetic",
        "config": {"workload": args.workload, "particles": n, "mesh": main_run["mesh"],
                   "substeps_per_step": S, "average_every": S, "dt": prm["dt"],
                   "precision": args.precision, "drag": args.drag, "lift_c": args.lift,
                   "solid_velocity": args.solid_velocity, "scheme": args.scheme,
                   "avg_bandwidth_m": prm["avg_bandwidth"],
                   "avg_bandwidth_z_m": prm["avg_bandwidth_z"] or prm["avg_bandwidth"],
                   "bed_seed": main_run["meta"].get("bed_seed"),
                   "field_seed": main_run["meta"].get("field_seed")},
        "roofline": main_run["roofline"],
        "cpu_baseline": main_run["cpu"],
        "averaging": main_run["averaging"],
        "phases": main_run["phases"],
        "particle_step_only": main_run["particle_step_only"],
        "rebuild": main_run["rebuild"],
        "bed10m_mixed": bed10m,
        "surrogate": surrogate,
        "stats": main_run["stats"],
    }
    print(json.dumps(out))


def rebuild_bytes_per_particle(mean_nbr, mean_contacts, mixed):
    """Algorithmic HBM bytes of one neighbour-list rebuild per particle:
    bin key from the position (32 B read, key + rank 8 B written), the
    scatter (8 B read, 4 B written), the re-sort of the particle state (pos,
    vel, omg, acc, alpha, drag, two wall-history rows and the ID: 260 B read
    and 260 B written once), the list build (own position 32 B, the
    neighbour indices 4 B each, count, history mask and build position
    40 B) and the carry-over of the tangential history (slot history read,
    (partner ID, xi) rows written and read back, slot history written:
    per active contact 2 h + 2 x 28 B with h = 24 B, 12 B in mixed mode)."""
    h = 12 if mixed else 24
    return 40 + 12 + 520 + 72 + 4 * mean_nbr + mean_contacts * (2 * h + 56)


def particle_bench(args, name, precision, K, W, rebuilds=0, cpu_steps=0):
    """Time K bench steps (each args.substeps particle steps + one averaging)
    of one workload after W warm-up bench steps; then per-phase device times,
    the force-kernel roofline, forced rebuilds and the oracle CPU baseline."""
    import torch

    import paper_1601_03801_amd as sm
    import workloads

    t0 = time.time()
    w = workloads.workload(name)
    prm = dict(w["params"], drag_law=args.drag,
               avg_bandwidth_z=args.bandwidth_z * workloads.D50, c_lift=args.lift,
               avg_solid_velocity=1 if args.solid_velocity else 0,
               avg_scheme=1 if args.scheme == "bdf2" else 0)
    n = len(w["d"])
    print(f"bench: workload {name}: {n} spheres, mesh {w['meta']['mesh']}, "
          f"generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    dmax = float(w["d"].max())
    g = sm.Sedimi(prm, n, precision=precision, d_max=dmax, skin=0.1 * dmax,
                  max_neighbors=24)
    g.set_fluid(w["U"], w["gradp"], w["dudt"])
    g.set_particles(w["x"], w["v"], w["d"], w["rho"], omega=w["w"])
    g.average()
    g.compute_forces(update_history=False)
    S = args.substeps
    for _ in range(W):
        g.step(S, average_every=S)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(K):
        g.step(S, average_every=S)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    elapsed = t2 - t1
    value = n * S * K / elapsed
    print(f"bench: {name} timed {K} bench steps in {elapsed:.3f} s", file=sys.stderr,
          flush=True)

    # per-phase device times (HIP events on the library's stream)
    g.set_profiling(True)
    for _ in range(max(2, K // 4)):
        g.step(S, average_every=S)
    prof = g.profile()
    g.set_profiling(False)
    st = g.stats()
    f_ms, f_cnt = prof["forces"]
    f_avg = f_ms / max(f_cnt, 1)
    mixed = precision == "mixed"
    bpp = force_bytes_per_particle(st["mean_neighbors"], st["mean_contacts"], mixed)
    ncell = prm["nx"] * prm["ny"] * prm["nz"]
    bytes_launch = n * bpp + ncell * ((4 if args.lift > 0 else 3) * 32 + 8)
    achieved = bytes_launch / (f_avg * 1e-3) / 1e9
    traffic = None
    pmc = FORCE_PMC.get((name, precision))
    if (pmc is not None and args.drag == "difelice" and args.lift == 0
            and pmc["sources_sha256"] == force_sources_sha()):
        traffic = int(1024 * (pmc["fetch_kib"] * pmc["fetch_scale"]
                              + pmc["write_kib"] * pmc["write_scale"]))
    roofline = {"bound": "hbm", "kernel": "k_forces (step)", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "avg_launch_ms": round(f_avg, 5),
                "bytes_per_launch": int(bytes_launch),
                "bytes_per_particle": round(bpp, 1)}
    phases = {k: {"ms_per_launch": round(v[0] / max(v[1], 1), 5), "launches": v[1]}
              for k, v in prof.items()}
    avg_ms = (prof["deposit"][0] + prof["smooth"][0]) / max(prof["smooth"][1], 1)
    dep_r, sol_r = averaging_rooflines(
        n, ncell, prof["deposit"][0] / max(prof["deposit"][1], 1),
        prof["smooth"][0] / max(prof["smooth"][1], 1), st["solve_iters"] == 0,
        w["meta"]["mesh"], g.nch)
    # the particle step alone (drift, gated rebuild chain, forces), per step
    dem_ms = (prof["drift"][0] + prof["rebuild"][0] + prof["forces"][0]) / max(prof["forces"][1], 1)

    # forced neighbour-list rebuilds (binning, re-sort, pair search, history
    # carry-over) on the same bed: the timed run above rebuilds only when a
    # particle has moved half the skin
    rebuild = None
    if rebuilds > 0:
        g.rebuild()
        g.set_profiling(True)
        for _ in range(rebuilds):
            g.step(1, average_every=0)
            g.rebuild()
        prof_r = g.profile()
        g.set_profiling(False)
        st_r = g.stats()
        # phase 1 holds the forced rebuilds and the gated (idle) chains of the steps
        idle_ms = prof["rebuild"][0] / max(prof["rebuild"][1], 1)
        r_ms = (prof_r["rebuild"][0] - rebuilds * idle_ms) / rebuilds
        rb_bpp = rebuild_bytes_per_particle(st_r["mean_neighbors"], st_r["mean_contacts"], mixed)
        r_bytes = n * rb_bpp + 8 * n  # + bin counts and starts (about one bin per particle)
        rebuild = {"ms": round(r_ms, 5), "forced": rebuilds, "bytes": int(r_bytes),
                   "bytes_per_particle": round(rb_bpp, 1), "bound": "hbm",
                   "achieved_GBps": round(r_bytes / (r_ms * 1e-3) / 1e9, 1),
                   "frac": round(r_bytes / (r_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "gated_idle_ms_per_step": round(idle_ms, 5)}
        print(f"bench: {name} forced rebuild {r_ms:.3f} ms", file=sys.stderr, flush=True)

    cpu = None
    if cpu_steps > 0:
        cpu = cpu_baseline(w, prm, cpu_steps)
    stats = {"mean_neighbors": round(st["mean_neighbors"], 3),
             "mean_contacts": round(st["mean_contacts"], 3),
             "rebuilds": st["rebuilds"], "steps": st["steps"]}
    g.close()
    del g
    return {"value": value, "elapsed": elapsed, "n": n, "prm": prm, "steps": K,
            "mesh": w["meta"]["mesh"], "meta": w["meta"], "roofline": roofline,
            "phases": phases,
            "averaging": {"plain_ms": round(avg_ms, 4),
                          "solver": "direct" if st["solve_iters"] == 0 else "iterative",
                          "solve_iters": st["solve_iters"], "residual": st["solve_residual"],
                          "deposit": dep_r, "solve": sol_r},
            "particle_step_only": {"ms_per_step": round(dem_ms, 5),
                                   "particle_updates_per_s": round(n / (dem_ms * 1e-3), 1)},
            "rebuild": rebuild, "cpu": cpu, "stats": stats}


def host_cpu():
    """The host CPU's model name (from /proc/cpuinfo), its logical CPU count
    and the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline(w, prm, steps):
    """The FP64 oracle on the host: a few particle steps of the same bed, on
    one thread and on all the threads this process may use (its OpenMP loops
    keep every sum in order, so both runs give the same bits)."""
    import oracle
    n = len(w["d"])
    host = host_cpu()
    all_threads = int(os.environ.get("OMP_NUM_THREADS") or host["affinity"])
    runs = {}
    for threads in (1, all_threads):
        oracle.set_threads(threads)
        ost = oracle.State(prm, w["x"], w["v"], w["w"], w["d"], w["rho"], U=w["U"],
                           gradp=w["gradp"], dudt=w["dudt"])
        ost.average()
        ost.init_accel()
        c0 = time.perf_counter()
        ost.run(steps)
        c1 = time.perf_counter()
        runs[threads] = (c1 - c0, ost.x.copy())
        print(f"bench: oracle {steps} steps on {threads} threads in {c1 - c0:.1f} s",
              file=sys.stderr, flush=True)
    oracle.set_threads(1)
    el_all, x_all = runs[all_threads]
    el_one, x_one = runs[1]
    return {"value": round(n * steps / el_all, 1), "unit": "particle-updates/s",
            "cores": all_threads, "kind": "oracle",
            "sample": f"{steps} particle steps of the same {n}-sphere bed "
                      f"({el_all:.1f} s on {all_threads} threads), no averaging",
            "single_thread": {"value": round(n * steps / el_one, 1), "cores": 1,
                              "seconds": round(el_one, 2)},
            "bit_identical_across_threads": bool(np.array_equal(x_all, x_one)),
            **host}


def surrogate_section(args):
    """Learned stand-in for the averaging on the fine 256 x 128 x 128 mesh
    (cells of 3.125d x 3.125d x 0.5d): train on snapshots of 8 seeded
    2M-sphere beds (random periodic translations, targets from the plain
    solve on the GPU), measure the error against the plain solve on beds of 2
    held-out seeds, then run the 4M-sphere bed with averaging every step
    under each averaging mode and compare time, fallback rate and error
    against the plain solve (direct, and the iterative solver the paper's
    method runs)."""
    import numpy as np
    import torch

    import paper_1601_03801_amd as sm
    import workloads

    t0 = time.time()
    train_seeds, held_seeds = list(range(1000, 1008)), [1010, 1011]
    beds = {s: workloads.workload("fine2m", seed=s) for s in train_seeds + held_seeds}
    w4 = workloads.workload("fine4m")
    print(f"bench: surrogate beds generated in {time.time() - t0:.1f} s", file=sys.stderr,
          flush=True)
    prm = dict(w4["params"])
    dmax = float(max(max(b["d"].max() for b in beds.values()), w4["d"].max()))
    n4 = len(w4["d"])
    g = sm.Sedimi(prm, n4, precision="mixed", d_max=dmax, skin=0.1 * dmax, max_neighbors=24,
                  nn=True, nn_alpha=args.nn_alpha, nn_bound=1e-3, nn_sample=0.01)
    rng = np.random.default_rng(2024)
    Lx, Ly = prm["Lx"], prm["Ly"]

    def load(seed):
        b = beds[seed]
        g.set_fluid(b["U"], b["gradp"], b["dudt"])
        g.set_particles(b["x"], b["v"], b["d"], b["rho"])
        g.compute_forces()

    def snapshot():
        # the drag law reads the smoothed solid fraction of this snapshot, as
        # in a coupled step (not the one of the previous, translated snapshot)
        g.translate(rng.uniform(0, Lx), rng.uniform(0, Ly))
        g.average()
        g.compute_forces()
        g.deposit()

    # per-channel scale without a shift: the map raw -> smooth is linear and
    # homogeneous, so a cell with no particles stays exactly zero in and out
    raws = []
    for s in train_seeds[:4]:
        load(s)
        snapshot()
        raws.append(g.get_field(0))
    raws = np.stack(raws)
    rms = np.sqrt((raws ** 2).mean(axis=(0, 2))) + 1e-30
    g.nn_set_norm(np.zeros(4), rms)
    # one channel group per field: the averaging smooths each field alone, so
    # the solid fraction's output must not depend on the drag inputs (which
    # change once particles move)
    g.nn_set_groups(args.nn_groups)
    g.nn_init(11)
    T = args.nn_train_steps
    switch = max(1, T // 40)
    losses = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    train_ms = 0.0
    for it in range(T):
        if it % switch == 0:
            load(train_seeds[(it // switch) % len(train_seeds)])
        snapshot()
        g.smooth(4)
        lr = 1e-6 + 0.5 * (args.nn_lr - 1e-6) * (1 + math.cos(math.pi * it / max(T, 1)))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        losses.append(g.nn_train_step(lr))
        e1.record()
        e1.synchronize()
        train_ms += e0.elapsed_time(e1)
    train_s = time.perf_counter() - t1
    step_ms = train_ms / max(T, 1)
    # medians over one pass through all the training beds at each end
    print(f"bench: trained {T} steps on {len(train_seeds)} beds in {train_s:.1f} s, median loss "
          f"{np.median(losses[:8 * switch]):.3e} -> {np.median(losses[-8 * switch:]):.3e}",
          file=sys.stderr, flush=True)

    # held-out beds: network error against the plain solve, and the check's estimate
    errs, checks = [], []
    for s in held_seeds:
        load(s)
        for _ in range(2):
            snapshot()
            g.smooth(4)
            plain = g.get_field(1)
            g.nn_forward()
            nn = g.get_field(1)
            checks.append([float(v) for v in g.nn_check()])
            rel = np.linalg.norm(nn - plain, axis=1) / (np.linalg.norm(plain, axis=1) + 1e-300)
            raw = g.get_field(0)
            rel_raw = np.linalg.norm(raw - plain, axis=1) / (np.linalg.norm(plain, axis=1) + 1e-300)
            errs.append([float(np.abs(nn[0] - plain[0]).max())] + [float(r) for r in rel] +
                        [float(rel_raw[0])])
    errs = np.array(errs)
    checks = np.array(checks)
    print(f"bench: held-out eps_s rel-L2 {errs[:, 1].max():.3e}, check estimate "
          f"{checks[:, 0].max():.3e}", file=sys.stderr, flush=True)

    # network forward alone against the plain solves alone, HIP events per call
    def timed(fn, reps=5):
        tot = 0.0
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            tot += e0.elapsed_time(e1)
        return tot / reps
    g.nn_forward()
    fwd_ms = timed(g.nn_forward)
    solve_ms = timed(lambda: g.smooth(4))
    check_ms = timed(g.nn_check)
    ncell = prm["nx"] * prm["ny"] * prm["nz"]
    C = 32
    fwd_flop = 2 * 27 * ncell * (4 * C + 4 * C * C + C * 4)
    mfma = {"forward_ms": round(fwd_ms, 4), "plain_solve_ms": round(solve_ms, 4),
            "check_ms": round(check_ms, 4),
            "forward_tflops": round(fwd_flop / (fwd_ms * 1e-3) / 1e12, 2),
            "peak_tflops_bf16": 2500.0,
            "frac": round(fwd_flop / (fwd_ms * 1e-3) / 2.5e15, 4)}
    print(f"bench: network forward {fwd_ms:.3f} ms ({mfma['forward_tflops']} TFLOP/s), "
          f"plain solve {solve_ms:.3f} ms, check {check_ms:.3f} ms", file=sys.stderr, flush=True)

    # coupled 4M-sphere run, averaging every step, per averaging mode
    g.set_fluid(w4["U"], w4["gradp"], w4["dudt"])
    g.set_particles(w4["x"], w4["v"], w4["d"], w4["rho"])
    g.average()
    g.compute_forces()
    modes = {}
    K = args.nn_steps
    for name, mode in (("plain", sm.AVG_PLAIN), ("surrogate_checked", sm.AVG_SURROGATE_CHECKED),
                       ("surrogate", sm.AVG_SURROGATE)):
        g.set_avg_mode(mode)
        g.step(2, average_every=1)
        st0 = g.stats()
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        g.step(K, average_every=1)
        torch.cuda.synchronize()
        el = time.perf_counter() - c0
        g.set_profiling(True)
        g.step(3, average_every=1)
        pr = g.profile()
        g.set_profiling(False)
        st1 = g.stats()
        avg_ms = (pr["deposit"][0] + pr["smooth"][0]) / max(pr["smooth"][1], 1)
        calls = st1["nn_calls"] - st0["nn_calls"]
        modes[name] = {"particle_updates_per_s": round(n4 * K / el, 1),
                       "ms_per_step": round(1000 * el / K, 3),
                       "averaging_ms": round(avg_ms, 3),
                       "fallback_rate": (round((st1["nn_fallbacks"] - st0["nn_fallbacks"]) /
                                               calls, 3) if calls else None),
                       "last_check": st1["nn_last_check"] if calls else None}
        print(f"bench: 4M bed, {name}: {modes[name]}", file=sys.stderr, flush=True)
    g.set_avg_mode(sm.AVG_PLAIN)
    g.close()
    del g
    torch.cuda.empty_cache()
    # the plain method with the iterative solver (Chebyshev, the route of
    # meshes the direct solve does not diagonalise) on the same bed
    gi = sm.Sedimi(prm, n4, precision="fp64", d_max=dmax, skin=0.1 * dmax, max_neighbors=24,
                   solver="iterative")
    gi.set_fluid(w4["U"], w4["gradp"], w4["dudt"])
    gi.set_particles(w4["x"], w4["v"], w4["d"], w4["rho"])
    gi.compute_forces()
    gi.deposit()
    gi.smooth(4)
    iter_ms = timed(lambda: gi.smooth(4), reps=3)
    iters = gi.stats()["solve_iters"]
    gi.close()
    print(f"bench: iterative plain solve {iter_ms:.3f} ms ({iters} iterations)", file=sys.stderr,
          flush=True)
    return {
        "workload": "fine4m", "mesh": w4["meta"]["mesh"], "particles": n4,
        "leaky_relu_alpha": args.nn_alpha, "channel_groups": args.nn_groups,
        "train": {"snapshots": T, "lr": f"cosine {args.nn_lr:g} -> 1e-06", "beds": f"fine2m seeds {train_seeds[0]}-{train_seeds[-1]}, "
                                          "random periodic translations",
                  "seconds": round(train_s, 2), "ms_per_train_step": round(step_ms, 3),
                  "loss_median_first_pass": float(np.median(losses[:8 * switch])),
                  "loss_median_last_pass": float(np.median(losses[-8 * switch:]))},
        "error_vs_plain": {"held_out_seeds": held_seeds,
                           "eps_s_maxabs": float(errs[:, 0].max()),
                           "rel_l2_per_channel": [float(v) for v in errs[:, 1:5].max(axis=0)],
                           "eps_s_rel_l2_unsmoothed": float(errs[:, 5].min()),
                           "check_estimate_per_channel": [float(v) for v in checks.max(axis=0)],
                           "bound": 1e-3},
        "mfma": mfma,
        "plain_iterative": {"solve_ms": round(iter_ms, 3), "iterations": iters},
        "modes": modes,
    }

if __name__ == "__main__":
    main()

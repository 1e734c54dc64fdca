#!/usr/bin/env python3
"""Throughput benchmark of the short-range MD hot path on one MI355X.

Default workload: Kob-Andersen 80:20 binary Lennard-Jones mixture, N = 4096,
density 1.2, Nose-Hoover NVT at T = 0.45 (tau = 0.2), dt = 0.005, shifted-force
cutoff 2.5 sigma_ab, skin 0.3, float32 positions and forces with float64
reductions.  Seeded random non-overlapping start, relaxed by an untimed
2000-step NVT run at dt = 0.001 and untimed NVT steps at dt = 0.005 until the
temperature is within 3 % of T0; the layout autotuner (untimed) then picks
threads per particle, block size, list builder and launch form at skin 0.3,
and W untimed and K timed steps follow (one srmd_step call).  A step is one
pass of the whole hot path: displacement check, list rebuild when due (cell
binning, counting sort, reorder, cell-stencil list), pair forces, integrator
and thermostat.

Prints one JSON line with particle-steps/s (whole job), the roofline position of
the dominant kernel (per step: algorithmic bytes and FLOPs against HBM and FP32
peaks, from kernel durations taken in a separate untimed pass), the CPU oracle's
rate on the host cores and on one core, and the batched-replica comparison of
256 Kob-Andersen replicas against one system per launch.
"""
import argparse
import json
import os

import numpy as np
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec & timesteps/sec, LJ/KA N=1k-1M; batched replicas vs single"
LIST_MODES = {1: "wave per particle", 2: "thread per particle", 3: "wave per cell", 4: "all pairs",
              5: "row-staged threads"}
STEP_FORMS = {0: "list kernel, step kernel, end-of-step kernel", 1: "list kernel, step kernel ending the step",
              2: "one step kernel (list build, forces, integrator, end of step)"}
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name, n, skin):
    from workloads import generators as gen

    if name == "ka4096":
        state = gen.config1_state()
        sig, eps, rc = gen.ka_params()
        desc = dict(workload="Kob-Andersen 80:20 NVT", n=state.n, rho=1.2, T0=0.45, tau=0.2, dt=0.005,
                    cutoff="shifted-force 2.5 sigma_ab", skin=skin, seed=state.seed, start="random insertion dmin 0.75"
                    " sigma_ab + 2000 NVT steps dt 0.001")
        return state, (sig, eps, rc), "sf", ("nvt", 0.005, 0.45, 0.2), desc
    if name == "lj":
        state = gen.config2_state(n) if n != 864 else gen.config0_state()
        sig, eps, rc = gen.lj_params()
        desc = dict(workload="Lennard-Jones NVE (melting FCC)", n=state.n, rho=0.8442, T=0.722, dt=0.005,
                    cutoff="shifted-potential 2.5", skin=skin, seed=state.seed, start="FCC lattice")
        return state, (sig, eps, rc), "sp", ("nve", 0.005), desc
    if name == "salt":
        n = 2000 if n == 864 else n
        state = gen.molten_salt_state(n, n)
        sig, eps, rc, q, rcc = gen.salt_params()
        desc = dict(workload="molten salt NVT (charged LJ, shifted-force Coulomb)", n=state.n, rho=gen.SALT_RHO,
                    T0=gen.SALT_T, tau=0.2, dt=0.004, cutoff="shifted-force LJ 2.5 + shifted-force Coulomb 6.0",
                    charges="+1/-1", skin=skin, seed=state.seed, start="random insertion dmin 0.8 + 2000 NVT steps "
                    "dt 0.001")
        return state, (sig, eps, rc, q, rcc), "sf", ("nvt", 0.004, gen.SALT_T, 0.2), desc
    raise SystemExit(f"unknown workload {name}")


FP32_PEAK_TFLOPS = 157.3


def path_bytes_per_particle_step(list_len, steps_per_rebuild, whole_path):
    """Algorithmic bytes per particle-step: force kernel 4 per list entry + 40 (list
    length, own position, force and energy out, virial), integrator 96 (position,
    velocity, force and last-build position in; position and velocity out), and for
    the whole path (the persistent kernel, the one-launch chain) the rebuild's 170 +
    4 per list entry amortised over the steps between rebuilds.  The neighbours' positions count once:
    the spatially sorted position array serves every neighbour read."""
    b = 4.0 * list_len + 40.0 + 96.0
    if whole_path:
        b += (170.0 + 4.0 * list_len) / max(steps_per_rebuild, 1.0)
    return b


def flops_per_particle_step(list_len, in_range, method):
    """Algorithmic FP32 FLOPs per particle-step (FMA = 2, rcp / rsq = 1): 20 per list
    entry (difference, minimum image, r^2) and per in-range pair 21 (shifted
    potential) or 27 (shifted force)."""
    return 20.0 * list_len + (27.0 if method == "sf" else 21.0) * in_range


def in_range_pairs_per_particle(pos, types, box, rc):
    """Mean count of partners within r_c,ab (float64 distances of the final state)."""
    from scipy.spatial import cKDTree

    p = np.mod(pos.astype(np.float64) + box / 2, box)
    tree = cKDTree(p, boxsize=box)
    pr = tree.query_pairs(float(np.max(rc)), output_type="ndarray")
    d = p[pr[:, 0]] - p[pr[:, 1]]
    d -= box * np.rint(d / box)
    r = np.sqrt((d * d).sum(1))
    keep = r < rc[types[pr[:, 0]], types[pr[:, 1]]]
    return 2.0 * keep.sum() / len(pos)


def hbm_traffic_per_step(workload_name, n, mode, tp, ppb, skin, list_mode):
    """HBM bytes per step of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (profiles/traffic.json; per dispatch, divided by
    the steps of that dispatch), or None when they were taken with another kernel
    source (each entry records the hash of the kernel source it was taken with) or
    another workload / launch shape."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_1506_05094_amd", "csrc", "kernels.hip")
    try:
        with open(path) as f:
            table = json.load(f)
        with open(src, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    for e in table.get("entries", []):
        if e.get("kernels_hip_sha256") != digest:
            continue  # counters of another kernel source are never reported
        if (e["workload"], e["n"], e["mode"], e["tp"], e["ppb"], e["skin"], e["list_mode"]) == (
                workload_name, n, mode, tp, ppb, skin, list_mode):
            per_dispatch = 1024.0 * (e["fetch_kib"] * e["fetch_scale"] + e["write_kib"] * e["write_scale"])
            return per_dispatch / e["steps_per_launch"]
    return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(state, params, method, integ, budget_s=12.0):
    """The oracle (FP64, O(N^2), OpenMP over particles) on every host core, and on one."""
    import oracle

    sig, eps, rc = params[:3]
    kw = {}
    if len(params) == 5:
        kw = dict(charges=params[3], rc_coul=params[4])
    if integ[0] == "nvt":
        kw.update(thermostat=True, T0=integ[2], tau=integ[3])

    def rate(budget):
        t0 = time.perf_counter()
        oracle.integrate(state.pos, state.vel, state.types, state.mass, state.box, sig, eps, rc, method, integ[1], 1,
                         **kw)
        t1 = time.perf_counter() - t0
        steps = int(max(1, min(2000, budget / max(t1, 1e-6))))
        t0 = time.perf_counter()
        oracle.integrate(state.pos, state.vel, state.types, state.mass, state.box, sig, eps, rc, method, integ[1],
                         steps, **kw)
        dt = time.perf_counter() - t0
        return state.n * steps / dt, steps, dt

    cores = oracle.num_threads()
    v_all, steps, dt = rate(budget_s)
    oracle.set_num_threads(1)
    try:
        v_one, steps1, dt1 = rate(budget_s / 3)
    finally:
        oracle.set_num_threads(cores)
    return {"value": v_all, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "value_one_core": v_one,
            "sample": f"{steps} oracle steps of the same system (N={state.n}, O(N^2) FP64 forces) from the seeded "
                      f"start on {cores} threads, {dt:.1f} s wall; {steps1} steps on one thread, {dt1:.1f} s wall"}


def replica_comparison(args, steps=None, base_steps=None):
    """Config 3: 256 Kob-Andersen replicas (N ~ U[500, 8000], T ~ U[0.4, 1.0], NVT dt
    0.005) advanced by one persistent launch per 500 steps, against the same systems
    advanced one system per launch.  Every replica's full state is saved before the
    timed batched run, so the one-system-per-launch forms start from the same states:
    at the batch's own launch shape (launch chains) each replica then follows its
    batched trajectory bit for bit over the same steps, so the energy drift is equal
    (checked on the recorded H); at each system's default shape (launch chains, and the
    persistent kernel) the list is rebuilt for that shape and the drift is reported
    beside the rate.  Returns a dict."""
    import torch

    from paper_1506_05094_amd import srmd
    from workloads import generators as gen

    steps = steps or args.replica_steps
    base_steps = base_steps or args.baseline_steps
    t0 = time.perf_counter()
    states = gen.ka_replica_states(args.replicas, workers=min(16, os.cpu_count() or 1))
    log(f"generated {len(states)} replicas (N = {sum(s.n for s in states)}) in {time.perf_counter() - t0:.1f} s")
    sig, eps, rc = gen.ka_params()
    temps = [T for (_, T, _) in gen.config3_states(args.replicas)]
    stream = torch.cuda.current_stream().cuda_stream
    # start layout t_p = 1, 256 particles per block; the batch autotuner picks the
    # layout below unless --tp is given
    tp, ppb = args.tp or 1, args.ppb or max(1, 256 // (args.tp or 1))
    systems = []
    for st, T in zip(states, temps):
        s = srmd.system_from_state(st, sig, eps, rc, "sf", skin=0.3, stream=stream)
        s.set_launch(tp, ppb)
        s.set_integrator_nvt(0.001, T, 0.2)
        systems.append(s)
    shapes = [(tp, ppb)] * len(systems)
    ntot = sum(s.n for s in systems)
    nr = np.array([s.n for s in systems])
    every = max(1, steps // 50)

    def drift(trace, k):
        h = trace["h_conserved"] / nr[:, None]
        x = np.arange(h.shape[1]) * k
        d = np.array([np.polyfit(x, h[r], 1)[0] for r in range(h.shape[0])])
        return {"median_abs": float(np.median(np.abs(d))), "max_abs": float(np.max(np.abs(d)))}

    batch = srmd.Batch(systems)
    batch.step(2000)  # relax the random insertion (untimed)
    for s, T in zip(systems, temps):
        s.set_integrator_nvt(0.005, T, 0.2)
    batch.step(max(args.warmup, 200))
    tuned = None
    if not args.tp:
        # untimed: the batch autotuner (shared t_p, then a block size per replica size
        # bucket); every trial starts from the stored states, which it restores
        t0 = time.perf_counter()
        tp, ppb_r = batch.autotune(200)
        shapes = [(tp, int(b)) for b in ppb_r]
        tuned = {"tp": tp, "ppb_counts": {str(b): int(c) for b, c in zip(*np.unique(ppb_r, return_counts=True))},
                 "seconds": round(time.perf_counter() - t0, 1)}
        log(f"batch autotune: {tuned}")
    blobs = [s.save_state() for s in systems]  # the common start of every form
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    trace = batch.step(steps, thermo_every=every)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    value_b = ntot * steps / wall_b
    batch.close()
    log(f"batched: {steps} steps of {len(systems)} replicas in {wall_b:.3f} s -> {value_b:.4e} particle-steps/s")
    baselines = {}
    for name, same, mode, nst in (("chain_same_shape", True, 0, steps),
                                  ("chain_default_shape", False, 0, min(steps, base_steps)),
                                  ("persistent_default_shape", False, -1, min(steps, base_steps))):
        k = max(1, nst // 50)
        for s, blob, shape in zip(systems, blobs, shapes):
            s.set_launch(*(shape if same else (0, 0)))
            s.set_persistent(mode)
            s.step(nst)  # graphs of these lengths captured, first build at this shape (untimed)
            s.load_state(blob)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = [s.step(nst, thermo_every=k) for s in systems]
        torch.cuda.synchronize()
        wall_s = time.perf_counter() - t0
        tr = np.stack(tr)
        entry = {"value": ntot * nst / wall_s, "steps": nst, "wall_s": wall_s,
                 "h_drift_per_particle_per_step": drift(tr, k)}
        if name == "chain_same_shape":
            entry["trajectories_equal_to_batch"] = bool(np.array_equal(tr["h_conserved"], trace["h_conserved"]))
        baselines[name] = entry
        log(f"one system per launch ({name}): {nst} steps each in {wall_s:.3f} s -> "
            f"{entry['value']:.4e} particle-steps/s; batched / this = {value_b / entry['value']:.2f}")
    for s in systems:
        s.close()
    best = max(baselines.values(), key=lambda b: b["value"])
    return {
        "workload": f"{len(systems)} Kob-Andersen replicas, N ~ U[500, 8000], T ~ U[0.4, 1.0], NVT dt 0.005, "
                    "one persistent launch per 500 steps",
        "n_total": ntot, "tp": tp, "ppb": ppb if tuned is None else tuned["ppb_counts"],
        "layout": "srmd_batch_autotune" if tuned else "given", "autotune": tuned,
        "steps": steps, "value": value_b, "unit": "particle-steps/s",
        "wall_s": wall_b, "one_launch_per_system": baselines,
        "batched_over_single_same_shape": value_b / baselines["chain_same_shape"]["value"],
        "batched_over_single_best": value_b / best["value"],
        "note": "all forms start from the same saved states; same shape: the same steps with every replica's "
                "trajectory (and so its energy drift) equal to the batch's bit for bit; best: the fastest "
                "one-system-per-launch form at its own shape, drift reported beside it",
        "h_drift_per_particle_per_step": drift(trace, every),
    }


def run_replicas(args):
    """Batched Kob-Andersen replicas: one persistent launch vs one launch chain per system."""
    r = replica_comparison(args, steps=args.steps)
    out = {
        "metric": METRIC, "value": r["value"], "unit": "particle-steps/s", "n_gpus": 1, "steps": r["steps"],
        "warmup": args.warmup, "ms_per_step": r["wall_s"] / r["steps"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": r["workload"], "n_total": r["n_total"], "tp": r["tp"], "ppb": r["ppb"]},
        "one_launch_per_system": r["one_launch_per_system"],
        "batched_over_single_same_shape": r["batched_over_single_same_shape"],
        "batched_over_single_best": r["batched_over_single_best"], "note": r["note"],
        "h_drift_per_particle_per_step": r["h_drift_per_particle_per_step"],
    }
    print(json.dumps(out), flush=True)


def run_precision(args):
    """Precision study: LJ N = 32768 (melting FCC, config 0 parameters), NVE dt 0.005,
    float32 / compensated float32 / float64 positions.  Energy drift per particle per
    step from a linear fit of H/N over the run; force error against the FP64 oracle
    on a sample of particles at a few frames."""
    import torch

    import oracle
    from paper_1506_05094_amd import srmd
    from workloads import generators as gen

    state = gen.config4_state()
    sig, eps, rc = gen.lj_params()
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(4)
    sample = np.sort(rng.choice(state.n, size=256, replace=False)).astype(np.int32)
    frames = max(1, args.frames)
    every = max(1, args.steps // 100)
    out = {"metric": METRIC, "workload": "precision study", "n": state.n, "steps": args.steps, "dt": 0.005,
           "variants": {}}
    for prec in ("f32", "f32_kahan", "f64pos"):
        s = srmd.system_from_state(state, sig, eps, rc, "sp", skin=0.3, precision=prec, stream=stream)
        if args.tp:
            s.set_launch(args.tp, args.ppb or max(1, 256 // args.tp))
        s.set_integrator_nve(0.005)
        h, ferr = [], []
        chunk = args.steps // frames
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in range(frames):
            tr = s.step(chunk, thermo_every=every)
            h.append(tr["h_conserved"] / state.n)
            s.compute_forces()
            st = s.get_state()
            F = st["force"][sample].astype(np.float64)
            Fr, _, _, _, _ = oracle.forces_f32(st["pos"], state.types, state.box, sig, eps, rc, "sp", sel=sample)
            ferr.append(float(np.abs(F - Fr).max() / np.abs(Fr).max()))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        h = np.concatenate(h)
        x = np.arange(h.size) * every
        slope = float(np.polyfit(x, h, 1)[0])
        out["variants"][prec] = {"drift_per_particle_per_step": slope, "h0_per_particle": float(h[0]),
                                 "h_range_per_particle": float(np.ptp(h)), "force_error_max_norm": ferr,
                                 "steps_per_s_incl_checks": args.steps / wall}
        log(f"{prec}: drift {slope:.3e} per particle per step, H/N range {np.ptp(h):.3e}, force errors {ferr}")
        s.close()
    print(json.dumps(out), flush=True)


def run_sweep(args):
    """Size sweep of the LJ fluid (config 0 parameters): per N, the autotuner's layout,
    then 2000 timed NVE steps at dt 0.005."""
    import torch

    from paper_1506_05094_amd import srmd
    from workloads import generators as gen

    sig, eps, rc = gen.lj_params()
    stream = torch.cuda.current_stream().cuda_stream
    rows = []
    for n in [int(v) for v in args.sizes.split(",")]:
        state = gen.config2_state(n) if n != 864 else gen.config0_state()
        s = srmd.system_from_state(state, sig, eps, rc, "sp", skin=0.3, stream=stream)
        s.set_integrator_nve(0.005)
        s.step(100)
        tuned = {}
        if args.tune_full:
            tuned = s.autotune_full(args.tune_steps, args.tune_cache)
            tp, ppb = tuned["tp"], tuned["ppb"]
        else:
            tp, ppb = s.autotune(args.tune_steps)
        groups = s.stats()["persistent_groups"]
        s.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(args.steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = s.stats()
        row = {"n": state.n, "tp": tp, "ppb": ppb, "mode": "persistent" if groups else "chain", "groups": groups,
               "steps_per_s": args.steps / wall, "particle_steps_per_s": state.n * args.steps / wall,
               "rebuilds": st["n_rebuilds"], "list_mode": st["list_mode"],
               "step_form": None if groups else st["step_form"]}
        if tuned:
            row.update({"skin": tuned["skin"], "trials": tuned["trials"],
                        "from_cache": tuned["from_cache"],
                        "trial_steps_per_s_baseline": 1e3 / tuned["baseline_ms_per_step"]
                        if tuned["baseline_ms_per_step"] > 0 else None,
                        "trial_steps_per_s_tuned": 1e3 / tuned["tuned_ms_per_step"]
                        if tuned["tuned_ms_per_step"] > 0 else None})
        log(row)
        rows.append(row)
        s.close()
    print(json.dumps({"metric": METRIC, "workload": "LJ size sweep (autotuned)", "steps": args.steps, "rows": rows}),
          flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--workload", default="ka4096", choices=["ka4096", "lj", "salt", "ka-replicas", "precision", "sweep"])
    ap.add_argument("--frames", type=int, default=4, help="force checks in the precision study")
    ap.add_argument("--tune", action="store_true",
                    help="run the layout autotuner (the default unless --no-tune, --tp or --mode is given)")
    ap.add_argument("--skin", type=float, default=0.3,
                    help="neighbour-list skin of the ka4096, lj and salt workloads (default 0.3)")
    ap.add_argument("--tune-full", action="store_true",
                    help="as --tune (and for the size sweep) with the full autotuner: skin optimisation, every "
                         "list method within 20 %% of the fastest, and the tuned-parameter file of --tune-cache")
    ap.add_argument("--tune-cache", default=None, help="tuned-parameter file of --tune-full (default: none)")
    ap.add_argument("--sizes", default="1000,4000,16000,64000,256000,1024000", help="N values of the size sweep")
    ap.add_argument("--tune-steps", type=int, default=1000, help="steps per autotuner trial (size sweep, --tune)")
    ap.add_argument("--replicas", type=int, default=256)
    ap.add_argument("--baseline-steps", type=int, default=200,
                    help="steps per system of each one-system-per-launch form in the replica comparison")
    ap.add_argument("--replica-steps", type=int, default=1000,
                    help="batched steps of the replica comparison in the default line (0: leave it out)")
    ap.add_argument("--n", type=int, default=864, help="particles for --workload lj (salt: 2000 unless given)")
    ap.add_argument("--tp", type=int, default=0, help="threads per particle (0: default / tuned)")
    ap.add_argument("--ppb", type=int, default=0)
    ap.add_argument("--mode", default=None, choices=["persistent", "chain"],
                    help="persistent: 500 steps per launch of one kernel (systems up to 8192 particles here); "
                         "chain: graph-captured launch chains (default: the layout autotuner's choice)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the layout autotuner: the persistent kernel (or --mode) at the default layout "
                         "(or --tp / --ppb)")
    ap.add_argument("--groups", type=int, default=-1, help="workgroups of the persistent kernel (-1: automatic)")
    ap.add_argument("--list-mode", type=int, default=0,
                    help="list builder (0 automatic, 1 wave, 2 thread, 3 cell, 4 all pairs)")
    ap.add_argument("--sort-interval", type=int, default=0,
                    help="all-pairs lists: spatial re-sort before every k-th build (0: never)")
    ap.add_argument("--profile-steps", type=int, default=1000,
                    help="steps of the untimed pass that times the dominant kernel's launches")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB between two device buffers three times (a plain copy of known "
                         "size, the reference for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (one process, one MI355X).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1506_05094_amd import srmd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    srmd.load()
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {nbytes} bytes")
        del src, dst
    if args.workload == "ka-replicas":
        run_replicas(args)
        return
    if args.workload == "precision":
        run_precision(args)
        return
    if args.workload == "sweep":
        run_sweep(args)
        return
    state, params, method, integ, desc = workload(args.workload, args.n, args.skin)
    sig, eps, rc = params[:3]
    s = srmd.system_from_state(state, sig, eps, rc, method, skin=args.skin,
                               stream=torch.cuda.current_stream().cuda_stream)
    if len(params) == 5:
        s.set_coulomb_sf(params[3], params[4])
    if args.tp:
        s.set_launch(args.tp, args.ppb or max(1, 256 // args.tp))
    if args.list_mode:
        s.set_rebuild_path(0, args.list_mode)
    if args.sort_interval:
        s.set_sort_interval(args.sort_interval)
    # the layout autotuner (untimed, after the relaxation) picks t_p, block size, list
    # builder and launch form at the configured skin unless a layout or form is given
    layout_tune = args.tune or not (args.no_tune or args.tp or args.mode or args.tune_full)
    persistent = (args.mode or "persistent") == "persistent" and state.n <= 8192
    if not (layout_tune or args.tune_full):
        s.set_persistent(args.groups if persistent else 0)
    if integ[0] == "nvt":
        s.set_integrator_nvt(0.001, integ[2], integ[3])
        s.step(2000)  # relax the random insertion (untimed)
        s.set_integrator_nvt(integ[1], integ[2], integ[3])
        # untimed: bring the temperature to T0 whatever --warmup is
        for _ in range(40):
            tr = s.step(500, thermo_every=10)
            if abs(np.mean(tr["temperature"][-10:]) / integ[2] - 1.0) < 0.03:
                break
    else:
        s.set_integrator_nve(integ[1])
    tuned = None
    if args.tune_full:
        # untimed: the full autotuner picks layout, list builder, mode and skin
        tuned = s.autotune_full(args.tune_steps, args.tune_cache)
        log(f"autotune_full: {tuned}")
        desc["skin_tuned"] = tuned["skin"]
        persistent = s.stats()["persistent_groups"] > 0
    elif layout_tune:
        # untimed: the autotuner picks layout, list builder and mode from this state
        t0 = time.perf_counter()
        s.autotune(args.tune_steps)
        desc["tuned"] = (f"srmd_autotune: t_p, block size, list builder and launch form at skin {args.skin} "
                         f"({time.perf_counter() - t0:.1f} s, untimed)")
        persistent = s.stats()["persistent_groups"] > 0
    s.step(args.warmup)
    torch.cuda.synchronize()
    st0 = s.stats()
    # HIP events on the system's stream (the current stream) bracket the timed region
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    s.step(args.steps)  # the product call: every timed step in one srmd_step
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    region_ms = ev0.elapsed_time(ev1)
    st1 = s.stats()
    th = s.thermo()
    n = state.n
    value = n * args.steps / wall
    log(f"timed {args.steps} steps in {wall:.4f} s: {value:.4e} particle-steps/s, {args.steps / wall:.1f} steps/s, "
        f"rebuilds {st1['n_rebuilds'] - st0['n_rebuilds']}, tp {st1['tp']} ppb {st1['ppb']}, "
        f"groups {st1['persistent_groups']}, list mode {st1['list_mode']}, step form {st1['step_form']}, "
        f"T {th['temperature']:.4f}")
    # untimed: the dominant kernel's launches timed one by one with HIP events on the
    # system's stream (persistent: launches of 500 steps; chains: the step kernel)
    prof_steps = max(args.profile_steps, 1000 if persistent else 200)
    ev_ms, dev_ms, launches = s.profile_step_kernel(prof_steps)
    st2 = s.stats()
    steps_per_launch = prof_steps / launches if persistent else 1.0
    # list length of a list built at the final positions (the counter of the last
    # build reads 0 when the run ended on a step that scheduled a rebuild), and the
    # measured steps per rebuild over the timed and profiled steps
    fin = s.get_state()
    s.build_neighbor_list()
    list_len = s.stats()["list_entries"] / n
    rebuilds = st2["n_rebuilds"] - st0["n_rebuilds"]
    steps_per_rebuild = (args.steps + prof_steps) / max(rebuilds, 1)
    # the Coulomb term's cutoff widens the pairs whose force is evaluated (molten salt)
    rc_eval = np.maximum(rc, params[4]) if len(params) == 5 else rc
    in_range = in_range_pairs_per_particle(fin["pos"], state.types, state.box, rc_eval)
    # dominant kernel, per step: when it is the only kernel of a step (the one-launch
    # chain), the events over the timed region (HIP events around single launches add
    # the dispatch latency, a third of a step here); otherwise the per-launch events
    one_kernel = not persistent and st1["step_form"] == 2
    step_s = region_ms / 1e3 / args.steps if one_kernel else ev_ms / 1e3 / launches / steps_per_launch
    # the whole path runs in the dominant kernel in the persistent form and in the
    # one-launch chain (step form 2: list build, forces, integrator, end of step)
    whole = persistent or st1["step_form"] == 2
    bytes_step = n * path_bytes_per_particle_step(list_len, steps_per_rebuild, whole)
    flops_step = n * flops_per_particle_step(list_len, in_range, method)
    hbm_gbs = bytes_step / step_s / 1e9
    tflops = flops_step / step_s / 1e12
    hbm_frac, fp32_frac = hbm_gbs / HBM_PEAK_GBS, tflops / FP32_PEAK_TFLOPS
    kname = ("k_multi (persistent: list build, sort, pair force, integrator, reductions)" if persistent
             else "k_step (list build, pair force, integrator, end of step and sort)" if whole
             else "k_step (pair force, integrator, end of step)" if st1["step_form"] == 1
             else "k_step (pair force, integrator)")
    traffic = hbm_traffic_per_step(desc["workload"], n, "persistent" if persistent else "chain", st1["tp"],
                                   st1["ppb"], desc["skin"], st1["list_mode"])
    # the arithmetic intensity sits below the FP32 ridge (157.3 / 8 = 19.7 FLOP/B), so
    # the roofline bound is HBM; when both fractions are far below one the kernel is
    # held by latency and synchronisation instead (small systems, paper section 3)
    bound = "hbm" if max(hbm_frac, fp32_frac) >= 0.1 else "latency"
    log(f"dominant kernel: {launches} launches of {steps_per_launch:g} steps, {step_s * 1e6:.3f} us/step; "
        f"{bytes_step / 1e6:.3f} MB and {flops_step / 1e6:.2f} MFLOP algorithmic per step -> {hbm_gbs:.1f} GB/s "
        f"({hbm_frac:.4f} of HBM), {tflops:.3f} TFLOP/s ({fp32_frac:.4f} of FP32); list {list_len:.1f}, "
        f"in range {in_range:.1f}, steps per rebuild {steps_per_rebuild:.1f}")
    roofline = {"bound": bound, "achieved": round(hbm_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 5), "traffic": traffic,
                "traffic_note": "HBM bytes per step of the dominant kernel (rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE, "
                                "copy-calibrated), null when the counters belong to other kernel source or shape",
                "bytes_per_step": bytes_step, "units": "per step (algorithmic bytes and FLOPs / kernel time per step)",
                "fp32": {"achieved": round(tflops, 4), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(fp32_frac, 5), "flops_per_step": flops_step},
                "kernel": kname, "steps_per_launch": steps_per_launch, "us_per_step": round(step_s * 1e6, 3),
                "timing": ("HIP events over the timed region (the step kernel is the only kernel of a step)"
                           if one_kernel else "HIP events around each launch of the kernel (untimed pass)"),
                "us_per_step_events_per_launch": round(ev_ms * 1e3 / launches / steps_per_launch, 3),
                "profiled_steps": prof_steps, "list_entries_per_particle": round(list_len, 2),
                "in_range_per_particle": round(in_range, 2), "steps_per_rebuild": round(steps_per_rebuild, 2)}
    s.close()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(state, params, method, integ)
        log(f"cpu baseline: {cpu}")
    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": dict(desc, tp=st1["tp"], ppb=st1["ppb"], mode="persistent" if persistent else "chain",
                       groups=st1["persistent_groups"], list_mode=LIST_MODES.get(st1["list_mode"], st1["list_mode"]),
                       list_mode_chosen_by="autotuner" if layout_tune else ("caller" if args.list_mode else "default"),
                       step_form=None if persistent else STEP_FORMS.get(st1["step_form"]),
                       sort_interval=args.sort_interval),
        "timesteps_per_sec": args.steps / wall,
        "rebuilds_in_timed_region": st1["n_rebuilds"] - st0["n_rebuilds"],
        "final_temperature": th["temperature"],
        "roofline": roofline, "cpu_baseline": cpu,
    }
    if args.workload == "ka4096" and args.replica_steps > 0:
        out["batched_replicas"] = replica_comparison(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

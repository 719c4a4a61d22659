"""Benchmark: SLPIC particle pushes per second on one MI355X.

Workload: the 1D argon sheath at production shape -- 2048 cells over 1024
Debye lengths, 1000 macroparticles per cell per species (4,096,000
particles), Te = 1 eV, Ti = 0.05 eV, speed limit u = 2 v_ti, dt = 1/omega_pi,
FP32 particles (int32 fixed-point positions, float velocities) with FP64
grids.  A step is one pass of the whole hot path: push + beta-weighted
deposit, wall absorption, source injection, field solve, and the cell sort
at the autotuned period.  Steps replay as HIP graphs of blocks of steps.

Prints one JSON line.  `value` is live particle pushes per second over the
timed steps (whole-step time, host clock around the timed region with device
synchronisation on both sides).  `roofline` prices the dominant kernel
(push + deposit) by its algorithmic bytes (24 B per live particle: read x,
v_x, v_y, v_z; write x, v_x -- the build stores v_perp^2 and moves 20 B) over
its average launch time, measured with HIP events captured around each push
launch on the launch stream inside the timed region.  `cpu_baseline` is the
FP64 oracle on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-pushes/s per GPU; time-to-steady-sheath, batched+warm-start vs plain"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per 1D3V push, the measurement plan's accounting: read
# x, vx, vy, vz, write x, vx (FP32: 16 + 8 B).  The build stores v_perp^2 in
# place of vy and vz (invariant in 1D electrostatics) and moves 20 B (FP64: 40).
BYTES_PER_PUSH = {"f32": 24, "f64": 48}
MOVED_BYTES_PER_PUSH = {"f32": 20, "f64": 40}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "push_deposit_traffic.json")


def _oracle_leg(cfg: dict, budget_s: float) -> dict:
    """One single-threaded oracle run of the workload for about budget_s of
    steps after its cold load: particles pushed and seconds."""
    import oracle
    run = oracle.Run(dict(cfg, sort_every=16))
    n0 = sum(run.nlive(s) for s in range(2))
    steps, t0 = 0, time.perf_counter()
    while True:
        run.step(1)
        steps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    return {"particles": n0, "steps": steps, "seconds": time.perf_counter() - t0}


def host_cpu() -> dict:
    """The host's logical CPUs, the ones this process may run on, and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def cpu_baseline(cfg: dict, budget_s: float = 12.0, max_procs: int = 16) -> dict:
    """The FP64 oracle (single thread, as written) on a bounded sample of the
    same workload, timed on the host's cores: once alone, then as one
    independent run per usable core (child processes started fresh, at most
    max_procs, the host share this benchmark may use), each from its own cold
    load for about budget_s of steps; the all-core value is their summed
    pushes over the longest run's time."""
    import subprocess
    single = _oracle_leg(cfg, budget_s)
    cpu = host_cpu()
    procs = max(1, min(cpu["affinity"], max_procs))
    code = ("import json, sys; sys.path.insert(0, %r); import bench; "
            "print(json.dumps(bench._oracle_leg(json.loads(sys.argv[1]), float(sys.argv[2]))))" % ROOT)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    children = [subprocess.Popen([sys.executable, "-c", code, json.dumps(cfg), str(budget_s)], stdout=subprocess.PIPE,
                                 env=env, text=True) for _ in range(procs)]
    legs = []
    for c in children:
        out, _ = c.communicate()
        if c.returncode == 0:
            legs.append(json.loads(out.strip().splitlines()[-1]))
    one = single["particles"] * single["steps"] / single["seconds"]
    allc = (sum(l["particles"] * l["steps"] for l in legs) / max(l["seconds"] for l in legs)) if legs else None
    return {"value": allc if allc else one, "unit": "particle-pushes/s", "cores": len(legs) if legs else 1,
            "kind": "oracle", "single_thread_value": one, "host": cpu,
            "sample": f"the same sheath from its cold load ({single['particles']} particles): {single['steps']} "
                      f"steps on one thread, and {len(legs)} independent runs of about {budget_s:.0f} s of steps "
                      f"each, one per core, FP64 C oracle (single-threaded as written)"}


def _copy_calibration():
    """The calibration kernel of the traffic counters: a 1 GiB device copy
    (1 GiB read + 1 GiB written)."""
    import torch
    src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()


def traffic_probe(args) -> int:
    """The workload for the counter runs (rocprofv3 --pmc): the benchmark's
    warm-up steps, then the 1 GiB copy that calibrates the traffic counters,
    then --steps direct-launch steps, so that the push dispatches after the
    copy are those of the timed region's particle states (steps after the
    warm-up), each one counted."""
    import torch
    import workloads
    from paper_1511_08225_amd import slpic
    if args.only_2d:
        cfg = workloads.sheath2d()
        sim = slpic.Sim2D(cfg, cfg["ny"], precision=args.precision, sort_every=cfg["sort_every"], tile=cfg["tile"])
        sim.step(args.warmup)
        torch.cuda.synchronize()
        _copy_calibration()
        sim.step(args.steps)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "traffic", "workload": "sheath2d", "warmup": args.warmup, "steps": args.steps,
                          "pushed": sim.status()["pushed_total"]}), flush=True)
        sim.close()
        return 0
    cfg = workloads.production_sheath(u_over_vti=args.u, ppc=args.ppc)
    params = launch_params(cfg, args)
    sim = slpic.Sim(cfg, precision=args.precision, sort_every=params["sort_every"], sort_bucket=params["sort_bucket"],
                    chunk=params["chunk"], block=params["block"], graph_steps=0,
                    push_order=params.get("push_order", 0), sort_tile=params.get("sort_tile", 0))
    sim.step(args.warmup)
    torch.cuda.synchronize()
    _copy_calibration()
    sim.step(args.steps)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "traffic", "warmup": args.warmup, "steps": args.steps, "pushed": sim.pushed_total(),
                      "launch": params}), flush=True)
    sim.close()
    return 0


def after_copy(rows):
    """Counter rows of the dispatches that follow the calibration copy (the
    probe's steps after its warm-up), in dispatch order."""
    key = "Dispatch_Id" if rows and "Dispatch_Id" in rows[0] else None
    if key:
        rows = sorted(rows, key=lambda r: int(r[key]))
    grid = "Grid_Size" if rows and "Grid_Size" in rows[0] else "Grid_Size_X"  # counter / kernel-trace files
    copies = [(int(r[grid]), i) for i, r in enumerate(rows) if "copyBuffer" in r["Kernel_Name"]]
    if not copies:
        return rows
    big = max(g for g, _ in copies)  # the calibration copy: the largest grid (other copies move small tables)
    first = min(i for g, i in copies if g == big)
    return rows[first:]


# The push + deposit target, as a fraction of the HBM roofline, and what the
# counters show limits it (profiles/push_valu_counters.md).
PUSH_TARGET_FRAC = 0.60
PUSH_LIMIT_NOTE = ("the push is bound by VALU issue (the exact speed-limited velocity map and "
                   "the FP64 deposit weight), and at this size also by latency with under one occupancy round "
                   "of waves; its HBM traffic is the 20 B per push the build moves, not more")

# The sources of the push kernels: a counter record holds their fingerprint
# and is reported only while it matches (a changed kernel reports null).
PUSH_SOURCES = {
    False: ("kernels.inc", "slpic_device.h", "slpic_internal.h", "field.inc"),
    True: ("kernels2d.inc", "slpic_device.h", "slpic2d_internal.h"),
}


def push_sources_sha(two_d: bool) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in PUSH_SOURCES[two_d]:
        with open(os.path.join(ROOT, "paper_1511_08225_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from(fetch_csv: str, write_csv: str, ppc: int, chunk: int, two_d: bool = False) -> int:
    """Per-launch HBM bytes of the push from two rocprofv3 --pmc counter files
    (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), each scaled by what the same
    counter reads for the 1 GiB copy; written where the benchmark reads it."""
    import csv
    kernel = "k_push2d" if two_d else "k_push_deposit"

    def per_kernel(path, counter):
        rows = after_copy([r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter])
        copy = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        push = [float(r["Counter_Value"]) for r in rows if kernel in r["Kernel_Name"]
                and ", true," in r["Kernel_Name"]]
        return copy, push

    fc, fp = per_kernel(fetch_csv, "FETCH_SIZE")
    wc, wp = per_kernel(write_csv, "WRITE_SIZE")
    if not (fc and fp and wc and wp):
        print("counter files lack the copy or push dispatches", file=sys.stderr)
        return 1
    gib_kib = 1024.0 * 1024.0
    f_scale = gib_kib / max(fc)  # KiB actually read by the copy / KiB the counter reports
    w_scale = gib_kib / max(wc)
    fetch = sum(fp) / len(fp) * f_scale * 1024.0
    write = sum(wp) / len(wp) * w_scale * 1024.0
    out = {"workload": "sheath2d" if two_d else "production_sheath", "ppc": ppc, "chunk": chunk,
           "launches": len(fp),
           "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "bytes_per_launch": fetch + write, "fetch_scale": f_scale, "write_scale": w_scale,
           "copy_fetch_kib": max(fc), "copy_write_kib": max(wc), "sources_sha": push_sources_sha(two_d)}
    table = json.load(open(TRAFFIC_FILE)) if os.path.exists(TRAFFIC_FILE) else {}
    table["sheath2d" if two_d else str(ppc)] = out
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps(out))
    return 0


def traffic_for_2d(tile: int):
    """Counter-measured HBM bytes per 2D push launch, if recorded for this
    tile with the current kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = json.load(open(TRAFFIC_FILE)).get("sheath2d")
    if t and t.get("chunk") == tile and t.get("sources_sha") == push_sources_sha(True):
        return t.get("bytes_per_launch")
    return None


def traffic_for(ppc: int, chunk: int):
    """Counter-measured HBM bytes per push launch, if recorded for this shape
    with the current kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = json.load(open(TRAFFIC_FILE)).get(str(ppc))
    if (t and t.get("workload") == "production_sheath" and t.get("chunk") == chunk
            and t.get("sources_sha") == push_sources_sha(False)):
        return t.get("bytes_per_launch")
    return None


def sweep_bench(args) -> int:
    """The batched sweep: 256 independent sheaths (ragged cells and particle
    counts) advanced together, launch parameters from the autotuner; prints
    one JSON line with pushes/s over the whole step."""
    import torch
    import workloads
    from paper_1511_08225_amd import autotune, slpic
    cfgs = workloads.batched_sweep(nruns=args.runs, seed=1)
    t0 = time.perf_counter()
    params = autotune.tune(cfgs, args.precision, log=lambda m: print(m, file=sys.stderr, flush=True))
    tune_s = time.perf_counter() - t0
    g = max(16, params["sort_every"])
    sim = slpic.Sim(cfgs, precision=args.precision, sort_every=params["sort_every"],
                    sort_bucket=params["sort_bucket"], chunk=params["chunk"], block=params["block"], graph_steps=g,
              push_order=params.get("push_order", 0), sort_tile=params.get("sort_tile", 0))
    steps = max(g, (args.steps // g) * g)
    sim.step(g * max(1, args.warmup // g))
    torch.cuda.synchronize()
    sim.profile(True)
    p0 = sim.pushed_total()
    t1 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    pushes = sim.pushed_total() - p0
    prof = sim.profile_read()["push"]
    st = sim.status()
    sim.close()
    npart = sum(c["nx"] * 2 * c["species"][0]["ppc"] for c in cfgs)
    push_ms = prof["ms"] / max(prof["launches"], 1)
    achieved = BYTES_PER_PUSH[args.precision] * pushes / max(prof["launches"], 1) / (push_ms * 1e-3) / 1e9
    print(json.dumps({
        "metric": "particle-pushes/s (batched sweep)", "value": pushes / el, "unit": "particle-pushes/s",
        "n_gpus": 1, "steps": steps, "ms_per_step": el * 1e3 / steps, "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"{args.runs} independent 1D3V sheaths: cells U[128, 2048], ppc U[200, 1000], "
                               f"Te/Ti log-U[5, 100], ion mass {{4, 20, 40, 84}} amu, u U[2, 10] v_ti",
                   "runs": args.runs, "particles_at_load": npart, "tuned": params, "tune_seconds": tune_s},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "kernel": "k_push_deposit", "avg_launch_ms": push_ms},
        "error_flags": sum(1 for s in st if s["error_flags"]),
    }), flush=True)
    return 0


def _to_steady(sim, nruns, max_steps, block, prune=False):
    """Step until every run is steady (or max_steps); returns per-run steady
    steps (-1 if not reached), per-run wall seconds when first seen steady
    (block granularity), total wall seconds and steps taken.  prune: take
    the retired runs out of the push and sort work at every status poll."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seen = [None] * nruns
    steps = 0
    st = sim.status()
    while steps < max_steps:
        sim.step(block)
        steps += block
        if prune:
            sim.prune_retired()
        st = sim.status()  # synchronises
        now = time.perf_counter() - t0
        for r in range(nruns):
            if seen[r] is None and st[r]["steady_step"] >= 0:
                seen[r] = now
        if all(s is not None for s in seen):
            break
    total = time.perf_counter() - t0
    return [s["steady_step"] for s in st], seen, total, steps, [s["error_flags"] for s in st]


def _plain_launch(cfg: dict, precision: str):
    """A lone run's own tuned launch (the autotuner's entry for its
    signature) and its graph block: the plain side of the time-to-steady
    comparison runs each sheath as it would run alone, not with the
    batch's launch."""
    from paper_1511_08225_amd import autotune
    p = autotune.tune([cfg], precision)
    g = max(16, p["sort_every"])
    kw = dict(precision=precision, sort_every=p["sort_every"], sort_bucket=p["sort_bucket"], chunk=p["chunk"],
              block=p["block"], graph_steps=g, push_order=p.get("push_order", 0), sort_tile=p.get("sort_tile", 0))
    return kw, g * max(1, 256 // g), p


def steady_bench(args) -> int:
    """Wall time to the steady sheath (wall-potential detector) from cold
    loads: all runs batched in one context, each run retired (frozen) by the
    library from the step after its detector flags it, and the same runs one
    at a time (a subset, the first --plain-runs), each stopped when flagged."""
    import workloads
    from paper_1511_08225_amd import autotune, slpic
    cfgs = workloads.batched_sweep(nruns=args.runs, seed=1)
    params = autotune.tune(cfgs, args.precision)
    g = max(16, params["sort_every"])
    block = g * max(1, 256 // g)
    kw = dict(precision=args.precision, sort_every=params["sort_every"], sort_bucket=params["sort_bucket"],
              chunk=params["chunk"], block=params["block"], graph_steps=g,
              push_order=params.get("push_order", 0), sort_tile=params.get("sort_tile", 0))
    import torch
    plain = []
    # both sides on a side stream, where blocks of g steps replay as HIP graphs
    with torch.cuda.stream(torch.cuda.Stream()):
        sim = slpic.Sim(cfgs, retire_steady=True, **kw)
        b_steady, b_seen, b_total, b_steps, b_err = _to_steady(sim, len(cfgs), args.max_steps, block, prune=True)
        sim.close()
        for r in range(min(args.plain_runs, len(cfgs))):
            kw1, block1, p1 = _plain_launch(cfgs[r], args.precision)
            one = slpic.Sim([cfgs[r]], **kw1)  # same run id: the same realisation as in the batch
            s1, seen1, tot1, steps1, err1 = _to_steady(one, 1, args.max_steps, block1)
            one.close()
            plain.append({"run": r, "steady_step": s1[0], "seconds": seen1[0] if seen1[0] is not None else tot1,
                          "reached": seen1[0] is not None, "error_flags": err1[0], "launch": p1})
    n_b = sum(1 for s in b_seen if s is not None)
    plain_mean = sum(p["seconds"] for p in plain) / max(len(plain), 1)
    print(json.dumps({
        "metric": "time-to-steady-sheath, batched vs plain (cold start)", "unit": "s",
        "runs": len(cfgs), "max_steps": args.max_steps, "block_steps": block, "tuned": params,
        "batched_mode": "one context, steady runs retired (slpic_tuning.retire_steady) and pruned "
                        "from the push and sort work at each status poll (slpic_prune_retired)",
        "batched": {"seconds_all": b_total, "steps": b_steps, "reached": n_b,
                    "seconds_median_run": sorted(s for s in b_seen if s is not None)[n_b // 2] if n_b else None,
                    "steady_steps": b_steady, "error_runs": [r for r, e in enumerate(b_err) if e]},
        "plain": {"runs_measured": len(plain), "seconds_mean_per_run": plain_mean,
                  "seconds_estimate_all": plain_mean * len(cfgs), "runs": plain},
        "speedup_estimate": (plain_mean * len(cfgs)) / b_total if b_total > 0 else None,
    }), flush=True)
    return 0


def time_to_steady(args, runs: int = 256, plain_runs: int = 16, max_steps: int = 16384, warm: bool = True,
                   train_runs: int = 256, train_steps: int = 4096) -> dict:
    """A bounded time-to-steady measurement for the default line (about 45 s
    on one MI355X): `runs` sheaths of the batched sweep distribution (seed 1)
    from cold loads, all in one context with steady runs retired and pruned,
    against the first `plain_runs` of them one at a time (the same kernels,
    graph replay), each stopped at its device steady flag or at max_steps; a
    run that never flags counts with its time at the cap (censored).  With
    warm: the network is trained in this run on `train_runs` other sweep runs
    (seed 2, profiles over the last quarter of `train_steps` steps), the
    `runs` sheaths are loaded warm from its prediction and batched the same
    way; the line gives their time to the flag, the preparation time apart,
    and how many settle within 2 % of the cold run's window mean (the
    reference)."""
    import torch
    import workloads
    from paper_1511_08225_amd import autotune, slpic
    cfgs = workloads.batched_sweep(nruns=runs, seed=1)
    params = autotune.tune(cfgs, args.precision)
    g = max(16, params["sort_every"])
    block = g * max(1, 256 // g)
    kw = dict(precision=args.precision, sort_every=params["sort_every"], sort_bucket=params["sort_bucket"],
              chunk=params["chunk"], block=params["block"], graph_steps=g, push_order=params.get("push_order", 0),
              sort_tile=params.get("sort_tile", 0))
    plain = []
    with torch.cuda.stream(torch.cuda.Stream()):
        sim = slpic.Sim(cfgs, retire_steady=True, **kw)
        b_steady, b_seen, b_total, b_steps, b_err = _to_steady(sim, len(cfgs), max_steps, block, prune=True)
        cold_means = [st["window_mean"][0] for st in sim.status()]
        sim.close()
        for r in range(min(plain_runs, len(cfgs))):
            kw1, block1, _ = _plain_launch(cfgs[r], args.precision)
            one = slpic.Sim([cfgs[r]], **kw1)
            s1, seen1, tot1, _, err1 = _to_steady(one, 1, max_steps, block1)
            one.close()
            plain.append({"run": r, "steady_step": s1[0], "seconds": seen1[0] if seen1[0] is not None else tot1,
                          "censored": seen1[0] is None, "error_flags": err1[0]})
        warm_out = None
        if warm:
            import numpy as np
            from paper_1511_08225_amd import warmstart
            t_prep = time.perf_counter()
            train_cfgs = workloads.batched_sweep(nruns=train_runs, seed=2)
            prof, _ = warmstart.collect_profiles(train_cfgs, steps=train_steps, sample_last=train_steps // 4,
                                                 tuning=params)
            X = np.stack([warmstart.features(c) for c in train_cfgs])
            net, std, losses = warmstart.train(X, prof.reshape(len(prof), -1), epochs=200)
            pred = warmstart.quasi_neutral(warmstart.predict(net, std, cfgs))
            t_prep = time.perf_counter() - t_prep
            simw = slpic.Sim(cfgs, retire_steady=True, warm=list(pred), **kw)
            w_steady, w_seen, w_total, _, w_err = _to_steady(simw, len(cfgs), max_steps, block, prune=True)
            warm_means = [st["window_mean"][0] for st in simw.status()]
            simw.close()
            both = [r for r in range(len(cfgs)) if b_steady[r] >= 0 and w_steady[r] >= 0]
            within = sum(1 for r in both if abs(warm_means[r] - cold_means[r]) <= 0.02 * abs(cold_means[r]))
            n_w = sum(1 for x in w_seen if x is not None)
            warm_out = {"batched_seconds": w_total, "batched_steady": n_w, "batched_censored": len(cfgs) - n_w,
                        "prepare_seconds": t_prep, "train_runs": train_runs, "train_steps": train_steps,
                        "train_loss_first_last": [losses[0], losses[-1]],
                        "steady_in_both": len(both), "within_2pct_of_cold": within,
                        "error_runs": [r for r, e in enumerate(w_err) if e]}
    n_b = sum(1 for x in b_seen if x is not None)
    plain_mean = sum(p["seconds"] for p in plain) / max(len(plain), 1)
    cens_b = len(cfgs) - n_b
    cens_p = sum(1 for p in plain if p["censored"])
    if warm_out is not None:
        w = warm_out["batched_seconds"]
        warm_out["speedup_vs_plain"] = (plain_mean * len(cfgs)) / w if w > 0 else None
        warm_out["note"] = ("the warm runs' flag is their own detector's; a warm load settles in a different "
                            "quasi-steady state than the cold run (within_2pct_of_cold counts the runs that "
                            "agree with the cold reference), so this ratio is not the warm start's gain")
    return {
        "metric": "time to the steady sheath, batched (cold start) vs plain one at a time", "unit": "s",
        "runs": len(cfgs), "plain_runs_timed": len(plain), "max_steps": max_steps, "launch": params,
        "plain_launch": "each plain run with its own tuned launch (the autotuner's entry for its signature)",
        "criterion": "device detector: three window means of Phi_w (nx/4 steps each) within 2 % of their average",
        "batched_seconds": b_total, "batched_steady": n_b, "batched_censored": cens_b,
        "plain_seconds_mean_per_run": plain_mean, "plain_censored": cens_p,
        "plain_seconds_estimate_all": plain_mean * len(cfgs),
        "speedup": (plain_mean * len(cfgs)) / b_total if b_total > 0 else None,
        "censored": bool(cens_b or cens_p),
        "note": "runs that never flag steady count at the step cap on both sides, so with censoring the ratio "
                "is a bound, not a measured speed-up",
        "error_runs": [r for r, e in enumerate(b_err) if e],
        "batched_warm": warm_out,
    }


def _histories(sim, nruns, steps):
    """Step `steps` steps, reading each run's full Phi_w series; returns the
    series (runs x steps) and the wall seconds of the stepping."""
    import numpy as np
    import torch
    out = np.zeros((nruns, steps))
    done, el = 0, 0.0
    while done < steps:
        n = min(4096, steps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(n)
        torch.cuda.synchronize()
        el += time.perf_counter() - t0
        for r in range(nruns):
            out[r, done:done + n] = sim.wall_history(r)[-n:]
        done += n
    return out, el


def warm_bench(args) -> int:
    """Learned warm start end to end at the C5 scale: steady profiles
    (phi, n, Gamma, T per species) of --train-runs batched cold runs (seed 2)
    over --horizon steps, the network trained on them in the library's
    kernels, then --eval-runs held-out runs (seed 3).  Reports (1) the
    prediction of the late wall potential against the held-out cold runs
    (the reference: their mean over the last quarter of the horizon) beside the
    naive prediction (the training mean) and beside the cold runs' own
    running estimate, with the cold steps each prediction is worth; (2) the
    held-out runs loaded warm from the prediction, and from their own late
    profiles (a perfect prediction), against the cold reference, and the
    batched warm vs plain cold wall time to the steady criterion."""
    import numpy as np
    import torch
    import workloads
    from paper_1511_08225_amd import autotune, slpic, warmstart
    H = args.horizon
    g = 64
    t_all = time.perf_counter()
    train_cfgs = workloads.batched_sweep(nruns=args.train_runs, seed=2)
    params = autotune.tune(train_cfgs[:256], args.precision)
    profs, t_col = [], time.perf_counter()
    for k in range(0, len(train_cfgs), 256):
        p, _ = warmstart.collect_profiles(train_cfgs[k:k + 256], steps=H, sample_last=H // 4, tuning=params)
        profs.append(p)
        print(f"collected {k + len(p)} / {len(train_cfgs)} training profiles", file=sys.stderr, flush=True)
    Y = np.concatenate(profs)
    X = np.stack([warmstart.features(c) for c in train_cfgs])
    t_col = time.perf_counter() - t_col
    t_tr = time.perf_counter()
    net, std, losses = warmstart.train(X, Y.reshape(len(Y), -1), epochs=args.epochs,
                                       log=lambda m: print(m, file=sys.stderr, flush=True))
    t_tr = time.perf_counter() - t_tr
    eval_cfgs = workloads.batched_sweep(nruns=args.eval_runs, seed=3)
    t_pred = time.perf_counter()
    pred = warmstart.predict(net, std, eval_cfgs)
    t_pred = time.perf_counter() - t_pred
    kw = dict(precision=args.precision, sort_every=params["sort_every"], sort_bucket=params["sort_bucket"],
              chunk=params["chunk"], block=params["block"], graph_steps=g,
              push_order=params.get("push_order", 0), sort_tile=params.get("sort_tile", 0))
    n = len(eval_cfgs)
    W = [max(1, c["nx"] // 4) for c in eval_cfgs]
    cold = slpic.Sim(eval_cfgs, **kw)
    hc, el_c = _histories(cold, n, H)
    cold.close()
    ref = hc[:, -H // 4:].mean(axis=1)
    # (1) the prediction of the late wall potential
    pw = pred[:, 0, 0] - pred[:, 0, -1]
    naive = float((Y[:, 0, 0] - Y[:, 0, -1]).mean())
    e_net = np.abs(pw - ref) / np.abs(ref)
    e_naive = np.abs(naive - ref) / np.abs(ref)

    def cold_estimate_err(t):
        return np.array([abs(hc[r, t - W[r]:t].mean() - ref[r]) / abs(ref[r]) for r in range(n)])

    def steps_worth(r, err):  # cold steps until its window estimate stays (3 windows) within err
        nw = H // W[r]
        means = hc[r, :nw * W[r]].reshape(nw, W[r]).mean(axis=1)
        ok = np.abs(means - ref[r]) <= err * abs(ref[r])
        for k in range(nw - 2):
            if ok[k] and ok[k + 1] and ok[k + 2]:
                return (k + 1) * W[r]
        return H

    worth_net = [steps_worth(r, e_net[r]) for r in range(n)]
    worth_naive = [steps_worth(r, e_naive[r]) for r in range(n)]
    prediction = {
        "reference": "held-out cold run: mean Phi_w over the last quarter of the horizon",
        "median_rel_err_network": float(np.median(e_net)), "median_rel_err_naive_mean": float(np.median(e_naive)),
        "network_better_than_naive": int((e_net < e_naive).sum()),
        "median_rel_err_cold_estimate": {f"H/{d}": float(np.median(cold_estimate_err(H // d))) for d in (8, 4, 2)},
        "cold_steps_worth_median": {"network": float(np.median(worth_net)), "naive_mean": float(np.median(worth_naive))},
        "note": "cold steps worth: the steps a cold run needs until its window estimate of Phi_w stays within "
                "the prediction's error of the reference (the horizon if never)",
        "predict_seconds": t_pred,
    }
    # (2) warm loads: from the prediction, and from the held-out runs' own late profiles
    warm = slpic.Sim(eval_cfgs, warm=list(warmstart.quasi_neutral(pred)), **kw)
    hw, el_w = _histories(warm, n, H)
    warm.close()
    own, _ = warmstart.collect_profiles(eval_cfgs, steps=H, sample_last=H // 4, tuning=params)
    perfect = slpic.Sim(eval_cfgs, warm=list(warmstart.quasi_neutral(own)), **kw)
    hp, _ = _histories(perfect, n, H)
    perfect.close()
    tc = [warmstart.steady_index(hc[r], W[r], ref[r]) for r in range(n)]
    tw = [warmstart.steady_index(hw[r], W[r], ref[r]) for r in range(n)]
    reach = {}
    for tol in (0.02, 0.05, 0.1):
        reach[str(tol)] = {name: int(sum(warmstart.steady_index(h[r], W[r], ref[r], tol) >= 0 for r in range(n)))
                           for name, h in (("cold", hc), ("warm_predicted", hw), ("warm_own_late_profiles", hp))}
    late = lambda h: h[:, -H // 4:].mean(axis=1)  # noqa: E731
    # plain: each run alone, step time measured per run
    tau1 = []
    for c in eval_cfgs[:min(64, n)]:
        one = slpic.Sim([dict(c, run=0)], **kw)
        one.step(g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one.step(4 * g)
        torch.cuda.synchronize()
        tau1.append((time.perf_counter() - t0) / (4 * g))
        one.close()
    tau1 = float(np.mean(tau1))
    steps_c = [t if t >= 0 else H for t in tc]
    steps_w = [t if t >= 0 else H for t in tw]
    plain_s = float(sum(steps_c)) * tau1
    batched_warm_s = max(steps_w) * el_w / H
    censored_c, censored_w = any(t < 0 for t in tc), any(t < 0 for t in tw)
    print(json.dumps({
        "metric": "learned warm start: prediction of the late sheath, and time to the steady sheath, "
                  "batched+warm-start vs plain", "unit": "s",
        "horizon_steps": H, "train_runs": len(train_cfgs), "eval_runs": n, "tuned": params,
        "prediction": prediction,
        "criterion": "window mean of Phi_w (nx/4 steps) within 2% of the cold run's mean over its last 25%, "
                     "for three windows",
        "reached_by_tol": reach,
        "late_phi_w_ratio_median": {"warm_predicted": float(np.median(late(hw) / ref)),
                                    "warm_own_late_profiles": float(np.median(late(hp) / ref))},
        "plain_seconds_estimate": plain_s, "plain_censored": censored_c,
        "batched_warm_seconds": batched_warm_s, "batched_warm_censored": censored_w,
        "speedup_batched_warm_vs_plain": (plain_s / batched_warm_s
                                          if batched_warm_s > 0 and not (censored_c or censored_w) else None),
        "batched_step_ms": el_c / H * 1e3, "plain_step_ms_mean": tau1 * 1e3,
        "train_loss_first_last": [losses[0], losses[-1]], "collect_seconds": t_col, "train_seconds": t_tr,
        "total_seconds": time.perf_counter() - t_all,
    }), flush=True)
    return 0


BYTES_PER_PUSH_2D = {"f32": 36, "f64": 72}


def cpu_baseline_2d(cfg: dict, budget_s: float = 12.0) -> dict:
    """The 2D FP64 oracle on a bounded sample: the full 512 x 512 grid with
    4 particles per cell per species (2,097,152 particles), as many steps as
    fit the budget (its load and the first deposit and solve untimed)."""
    import oracle
    small = dict(cfg)
    small["species"] = [dict(sp, ppc=4) for sp in cfg["species"]]
    run = oracle.Run2D(small, cfg["ny"], tile=cfg["tile"])
    n0 = sum(run.nslots(s) for s in range(2))
    steps, t0 = 0, time.perf_counter()
    while True:
        run.step(1)
        steps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": n0 * steps / dt, "unit": "particle-pushes/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the 512 x 512 sheath at 4 particles per cell per species ({n0} "
                      f"particles; the field solve is a plain O(nx ny^2) DFT), FP64 C oracle, one thread"}


def run_2d(args, steps: int = 256, warmup: int = 64) -> dict:
    """The 2D3V sheath (512 x 512 cells, 64 per cell per species, 33,554,432
    particles, FP32 particles with FP64 grids, tile sort every 8 steps):
    pushes/s over the timed steps and the push kernel's roofline."""
    import torch
    import workloads
    from paper_1511_08225_amd import slpic
    cfg = workloads.sheath2d()
    se = cfg["sort_every"]
    g = 2 * se  # steps per replayed HIP graph
    steps = max(g, steps // g * g)
    warmup = max(g, warmup // g * g)
    # the timed steps replay graphs on a side stream (the library captures
    # only on a non-default stream); a second context from the same seed
    # repeats them with HIP events around every push launch (direct
    # launches), which gives the push kernel's average duration
    with torch.cuda.stream(torch.cuda.Stream()):
        sim = slpic.Sim2D(cfg, cfg["ny"], precision=args.precision, sort_every=se, tile=cfg["tile"], graph_steps=g)
        sim.step(warmup)
        torch.cuda.synchronize()
        p0 = sim.status()["pushed_total"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = sim.status()
        pushes = st["pushed_total"] - p0
        sim.close()
        prof = slpic.Sim2D(cfg, cfg["ny"], precision=args.precision, sort_every=se, tile=cfg["tile"])
        prof.step(warmup)
        prof.profile(1)
        q0 = prof.status()["pushed_total"]
        prof.step(steps)
        ms, launches = prof.profile_read()["push"]
        prof_pushes = prof.status()["pushed_total"] - q0
        prof.close()
    bpp = BYTES_PER_PUSH_2D[args.precision]
    push_ms = ms / max(launches, 1)
    achieved = bpp * prof_pushes / max(launches, 1) / (push_ms * 1e-3) / 1e9
    out = {
        "metric": "particle-pushes/s per GPU (2D3V)", "value": pushes / (t1 - t0), "unit": "particle-pushes/s",
        "steps": steps, "warmup": warmup, "ms_per_step": (t1 - t0) * 1e3 / steps, "dtype": args.precision,
        "config": {"workload": (f"2D3V argon sheath, {cfg['nx']} x {cfg['ny']} cells (y periodic), 64 particles/"
                                f"cell/species ({2 * cfg['nx'] * cfg['ny'] * 64} particles at load), Te/Ti=20, "
                                f"u=3 v_ti, dt={cfg['dt']:.4g}/omega_pe, tile sort ({cfg['tile']}x{cfg['tile']} "
                                f"cells) every {se} steps, blocks of {g} steps replayed as HIP graphs")},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for_2d(cfg["tile"]), "kernel": "k_push2d",
                     "bytes_per_push": bpp, "avg_launch_ms": push_ms, "launches": launches},
        "wall_potential": st["wall_potential"], "error_flags": st["error_flags"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_2d(cfg)
    return out


def run_wave(args, n: int = 4_194_304, steps: int = 4000, per_launch: int = 500) -> dict:
    """Test electrons in the prescribed traveling wave (the paper's
    wave-particle test) at v0 = 2 v_phi, FP32: pushes/s of slpic_wave_push
    (each launch carries every particle through `per_launch` steps in
    registers), timed with events on the launch stream, and the oracle on a
    bounded sample."""
    import torch
    import numpy as np
    import workloads
    from paper_1511_08225_amd import slpic
    w, x0, v0 = workloads.wave_test(2.0, n=n, seed=0)
    x = torch.tensor(x0.astype(np.float32), device="cuda")
    v = torch.tensor(v0.astype(np.float32), device="cuda")
    slpic.wave_push(w, x, v, 0, per_launch)  # warm-up launch
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    done = per_launch
    while done < per_launch + steps:
        slpic.wave_push(w, x, v, done, per_launch)
        done += per_launch
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    out = {"metric": "test-particle pushes/s (prescribed traveling wave)", "value": n * steps / (ms * 1e-3),
           "unit": "particle-pushes/s", "steps": steps, "particles": n, "ms_per_step": ms / steps, "dtype": "f32",
           "config": {"workload": f"1D1V electrons, v_phi = v_te, e phi_max/T_e = 0.1, v0 = 2 v_phi, dt = dx/v0, "
                                  f"{per_launch} steps per launch"}}
    if not args.no_cpu_baseline:
        import oracle
        m = 20000
        t0 = time.perf_counter()
        oracle.wave_push(w, x0[:m], v0[:m], 0, 100)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": m * 100 / dt, "unit": "particle-pushes/s", "cores": 1, "kind": "oracle",
                               "sample": f"{m} particles x 100 steps of the same workload, FP64 C oracle, one thread"}
    return out


def _plates_leg(v0, ppc, runs, t_us, avg_us, graph_steps=16, samples=200):
    """One side of the plates experiment: `runs` seeds of the plates workload
    at speed limit v0 (inf = PIC) in one FP32 context on a side stream (so
    that blocks of graph_steps steps replay as HIP graphs), stepped from the
    empty box to t_us microseconds, with the moments sampled over the last
    avg_us at a stride of whole graph blocks.  Returns the wall time (host
    clock around the synchronised run), the steps, the final status of run 0
    and the run-averaged window means (phi, n_e, n_i)."""
    import torch
    import numpy as np
    import workloads
    from paper_1511_08225_amd import slpic
    cfg = workloads.plates_sheath(v0, ppc=ppc, sort_every=16, capacity_factor=0.5)
    cfg["steady_window"] = max(1, workloads.plates_steps(cfg, 1.0))  # windows of 1 us of simulated time
    total = workloads.plates_steps(cfg, t_us)
    avg = workloads.plates_steps(cfg, avg_us)
    stride = max(1, avg // samples)
    if stride >= graph_steps:
        stride = stride // graph_steps * graph_steps
    in_step = graph_steps % stride == 0  # sampled inside the captured step blocks
    nsamp = avg // stride
    configs = [dict(cfg, seed=1000 + r, run=r) for r in range(runs)]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        # 256-slot push chunks and 2048-slot sort tiles: a few 1e5 particles
        # spread over more wavefronts and sort workgroups than the defaults give
        sim = slpic.Sim(configs, precision="f32", sort_every=16, graph_steps=graph_steps, chunk=256,
                        sort_tile=2048)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        first = total - nsamp * stride
        sim.step(first)
        if in_step:
            sim.set_sampling(stride)
            sim.step(nsamp * stride)
        else:
            for _ in range(nsamp):
                sim.step(stride)
                sim.moments_sample(-1)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = sim.status()
        win = np.mean([sim.moments_window(r).cpu().numpy() for r in range(runs)], axis=0)
        pushed = sim.pushed_total()
        sim.close()
    flags = [s["error_flags"] for s in st]
    if any(flags):
        raise RuntimeError(f"plates run raised error flags {flags}")
    steady = [s["steady_step"] for s in st]
    return {"v0_over_vte": v0, "dt": cfg["dt"], "steps": total, "wall_s": wall, "ms_per_step": wall * 1e3 / total,
            "pushes_per_s": pushed / wall, "samples": nsamp, "sample_stride": stride,
            "final_particles": [st[0]["nslots"][0], st[0]["nslots"][1]],
            "steady_us": [None if k < 0 else k * cfg["dt"] / workloads.PAPER_OMEGA_PE_US for k in steady],
            "profiles": {"phi": win[0], "n_e": win[1], "n_i": win[4]}}


def run_plates(args, ppc: int = 9000, runs: int = 1) -> dict:
    """The paper's sheath experiment (Sec. IV): PIC (dt = dx/(5 v_te)) and
    SLPIC (v0 = 0.0158 v_te, dt = dx/v0) from the empty box to 24 us, the
    time-averaged phi, n_e, n_i over the last 8 us (one ion crossing) of
    each, their agreement (relative L2 over the interior nodes), and the
    wall-time ratio; the oracle's SLPIC run beside it on a bounded sample."""
    import numpy as np
    import workloads
    P = workloads.PLATES_PAPER
    sl = _plates_leg(0.0158, ppc, runs, P["t_steady_us"], P["t_cross_us"])
    if getattr(args, "plates_leg", "both") == "slpic":  # the SLPIC side alone (for kernel profiles)
        del sl["profiles"]
        return {"metric": "SLPIC run of the two-plate sheath to 24 us", "slpic": sl}
    pic = _plates_leg(math.inf, ppc, runs, P["t_steady_us"], P["t_cross_us"])
    agree = {}
    for k in ("phi", "n_e", "n_i"):
        a, b = sl["profiles"][k][1:-1], pic["profiles"][k][1:-1]
        agree[k + "_rel_l2"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    prof = {k: {"slpic": [round(float(v), 4) for v in sl["profiles"][k][::10]],
                "pic": [round(float(v), 4) for v in pic["profiles"][k][::10]]} for k in ("phi", "n_e", "n_i")}
    for leg in (sl, pic):
        del leg["profiles"]
    out = {"metric": "wall-time speed-up of SLPIC over PIC to the steady two-plate sheath",
           "value": pic["wall_s"] / sl["wall_s"], "unit": "x", "higher_is_better": True, "dtype": "f32",
           "config": {"workload": (f"two-plate argon sheath of Sec. IV: 100 cells over 25.65 Debye lengths, bias "
                                   f"5.68 T_e/e, both species injected through x = L, {ppc} g-particles per cell "
                                   f"at n0, {runs} run(s) per context, 24 us simulated, profiles averaged over "
                                   f"the last 8 us")},
           "slpic": sl, "pic": pic, "step_ratio": pic["steps"] / sl["steps"], "agreement": agree,
           "profiles_every_10_nodes": prof,
           "paper": {"speedup": P["speedup"], "pic_steps": P["pic_steps"], "slpic_steps": P["slpic_steps"],
                     "ions": P["ions"], "electrons": P["electrons"]}}
    if not args.no_cpu_baseline:
        import oracle
        cfg = workloads.plates_sheath(0.0158, ppc=ppc // 10, sort_every=16, capacity_factor=0.5)
        run = oracle.Run(cfg)
        n = workloads.plates_steps(cfg, P["t_steady_us"])
        t0 = time.perf_counter()
        run.step(n)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": dt * 10, "unit": "s to 24 us (SLPIC)", "cores": 1, "kind": "oracle",
                               "sample": f"the SLPIC run at {ppc // 10} g-particles per cell (a tenth of the "
                                         f"particles), all {n} steps, FP64 C oracle, one thread; its time x 10"}
    return out


def run_langmuir(args, nx: int = 128, ppc: int = 4000, seeds: int = 8, steps: int = 700) -> dict:
    """The speed-limited plasma frequency (plasma-oscillation section): a
    periodic box per (u, seed), u/v_te in {0.1, 0.25, 0.5, 1, 2, inf}, all in
    one FP32 context (48 runs, 49M particles), electrons displaced by a 0.3 %
    sine; the seed-averaged amplitude of E's fundamental mode from the device
    history, fitted frequency against the root of the speed-limited
    dispersion relation and its long-wavelength limit
    omega_p <(beta v_x)^2>^(1/2)/v_t (the oracle's quadratures)."""
    import torch
    import numpy as np
    import oracle
    import workloads
    from paper_1511_08225_amd import slpic
    us = [0.1, 0.25, 0.5, 1.0, 2.0, math.inf]
    cfgs = []
    for r, u in enumerate(us):
        for sd in range(seeds):
            cfgs.append(dict(workloads.langmuir_box(u, nx=nx, ppc=ppc, seed=40 + 100 * sd + r, sort_every=16),
                             run=len(cfgs)))
    with torch.cuda.stream(torch.cuda.Stream()):
        sim = slpic.Sim(cfgs, precision="f32", sort_every=16, graph_steps=16)
        for r in range(len(cfgs)):
            xe, vxe, vpe = sim.export_particles(r, 0)
            sim.import_particles(r, 0, workloads.langmuir_displacement(xe, nx, 0.003), vxe, vpe)
        sim.refresh_fields()
        torch.cuda.synchronize()
        p0 = sim.pushed_total()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        pushes = sim.pushed_total() - p0
        hist = np.array([sim.wall_history(r)[-steps:] for r in range(len(cfgs))])
        flags = [s["error_flags"] for s in sim.status()]
        sim.close()
    k = 2 * math.pi / (nx * 0.5)
    rows = []
    for r, u in enumerate(us):
        dt = cfgs[r * seeds]["dt"]
        t = dt * np.arange(1, steps + 1)
        root = oracle.slpic_dispersion("step", 8.0 if math.isinf(u) else u, k)
        w = workloads.fit_frequency(t, hist[r * seeds:(r + 1) * seeds].mean(axis=0), root)
        rows.append({"u_over_vte": None if math.isinf(u) else u, "dt": dt, "omega_measured": w,
                     "omega_dispersion_root": root,
                     "omega_long_wavelength": math.sqrt(oracle.slpic_plasma_freq2("step", u)),
                     "rel_err": w / root - 1.0, "omega_dt": w * dt})
    return {"metric": "speed-limited plasma frequency omega_s/omega_p (periodic box, fundamental mode)",
            "rows": rows, "k_lambda_D": k, "runs": len(cfgs), "particles": 2 * nx * ppc * len(cfgs), "steps": steps,
            "wall_s": wall, "pushes_per_s": pushes / wall, "error_flags": flags, "dtype": "f32",
            "config": {"workload": f"periodic box, {nx} cells of 0.5 Debye lengths, {ppc} g-particles per cell per "
                                   f"species, argon, Te/Ti = 20, {seeds} seeds per u, 0.3 % density perturbation"}}


def launch_params(cfg, args) -> dict:
    """Push chunk, workgroup size, sort period and bucket: from the autotuner
    (cached per workload signature) unless given on the command line."""
    from paper_1511_08225_amd import autotune
    if args.no_tune:
        return {"chunk": args.chunk, "block": 128, "sort_every": args.sort_every, "sort_bucket": 1, "push_order": 0}
    return autotune.tune([cfg], args.precision, log=lambda m: print(m, file=sys.stderr, flush=True))


def run_timed(cfg, args, steps, warmup, params):
    import torch
    from paper_1511_08225_amd import slpic
    g = max(16, params["sort_every"])
    steps = max(g, (steps // g) * g)
    warmup = max(g, (warmup // g) * g)
    # a side stream: the library captures blocks of g steps as HIP graphs
    # only on a non-default stream.  The timed region replays graphs; a second
    # context from the same seed then repeats the same steps with HIP events
    # around every push launch (direct launches), which gives the push
    # kernel's average duration over the same particle states.
    def make():
        return slpic.Sim(cfg, precision=args.precision, sort_every=params["sort_every"],
                         sort_bucket=params["sort_bucket"], chunk=params["chunk"], block=params["block"],
                         graph_steps=g, push_order=params.get("push_order", 0),
                         sort_tile=params.get("sort_tile", 0))
    with torch.cuda.stream(torch.cuda.Stream()):
        sim = make()
        sim.step(warmup)
        torch.cuda.synchronize()
        p0 = sim.pushed_total()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pushes = sim.pushed_total() - p0
        st = sim.status(0)
        sim.close()
        sim = make()
        sim.step(warmup)
        sim.profile(True)  # events around each push launch, on the launch stream
        q0 = sim.pushed_total()
        sim.step(steps)
        prof = sim.profile_read()["push"]
        prof["pushes"] = sim.pushed_total() - q0
        sim.close()
    return pushes, t1 - t0, prof, st, steps, warmup


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1024)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--u", type=float, default=2.0, help="speed limit in ion thermal speeds (inf = PIC)")
    ap.add_argument("--ppc", type=int, default=1000)
    ap.add_argument("--sort-every", type=int, default=16)
    ap.add_argument("--chunk", type=int, default=512, help="slots per push wavefront (with --no-tune)")
    ap.add_argument("--no-tune", action="store_true", help="use --chunk/--sort-every instead of the autotuner")
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hbm-variant", action="store_true")
    ap.add_argument("--no-u-sweep", action="store_true", help="leave out the u = 5, 10, inf v_ti lines and the "
                                                               "developed-state timing")
    ap.add_argument("--no-steady", action="store_true", help="leave out the bounded time-to-steady measurement")
    ap.add_argument("--sweep", action="store_true", help="batched-sweep throughput (autotuned) and exit")
    ap.add_argument("--runs", type=int, default=256, help="runs in the batched sweep")
    ap.add_argument("--steady", action="store_true", help="time to the steady sheath, batched vs plain, and exit")
    ap.add_argument("--plain-runs", type=int, default=32, help="runs timed one at a time in --steady")
    ap.add_argument("--max-steps", type=int, default=16384, help="step cap in --steady")
    ap.add_argument("--warm", action="store_true", help="learned warm start end to end, and exit")
    ap.add_argument("--train-runs", type=int, default=4096)
    ap.add_argument("--eval-runs", type=int, default=512)
    ap.add_argument("--horizon", type=int, default=8192, help="steps per run in --warm")
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--only-2d", action="store_true", help="the 2D3V sheath line alone, and exit")
    ap.add_argument("--no-2d", action="store_true", help="leave out the 2D3V sheath measurement")
    ap.add_argument("--only-wave", action="store_true", help="the wave-particle test-particle line alone, and exit")
    ap.add_argument("--no-wave", action="store_true", help="leave out the wave-particle measurement")
    ap.add_argument("--only-plates", action="store_true", help="the two-plate PIC vs SLPIC experiment alone, and exit")
    ap.add_argument("--only-langmuir", action="store_true", help="the speed-limited plasma frequency alone, and exit")
    ap.add_argument("--no-langmuir", action="store_true", help="leave out the speed-limited plasma frequency")
    ap.add_argument("--no-plates", action="store_true", help="leave out the two-plate PIC vs SLPIC experiment")
    ap.add_argument("--plates-ppc", type=int, default=9000, help="g-particles per cell at n0 in the plates experiment")
    ap.add_argument("--plates-runs", type=int, default=1, help="seeds per context in the plates experiment")
    ap.add_argument("--plates-leg", choices=("both", "slpic"), default="both",
                    help="slpic: run only the SLPIC side of the plates experiment (for kernel profiles)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run the counter workload (copy calibration + direct-launch steps) and exit")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 counter files into the per-launch traffic record and exit")
    args = ap.parse_args()
    if args.traffic_from:
        import workloads
        if args.only_2d:  # the record keeps the sort tile in its "chunk" field
            c2 = workloads.sheath2d()
            return traffic_from(args.traffic_from[0], args.traffic_from[1], c2["species"][0]["ppc"], c2["tile"],
                                two_d=True)
        chunk = launch_params(workloads.production_sheath(u_over_vti=args.u, ppc=args.ppc), args)["chunk"]
        return traffic_from(args.traffic_from[0], args.traffic_from[1], args.ppc, chunk)
    if args.traffic_probe:
        return traffic_probe(args)
    if args.sweep:
        return sweep_bench(args)
    if args.steady:
        return steady_bench(args)
    if args.warm:
        return warm_bench(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        return 2
    if args.only_2d:
        print(json.dumps(run_2d(args, args.steps, args.warmup)), flush=True)
        return 0
    if args.only_wave:
        print(json.dumps(run_wave(args)), flush=True)
        return 0
    if args.only_plates:
        print(json.dumps(run_plates(args, args.plates_ppc, args.plates_runs)), flush=True)
        return 0
    if args.only_langmuir:
        print(json.dumps(run_langmuir(args)), flush=True)
        return 0

    import workloads
    cfg = workloads.production_sheath(u_over_vti=args.u, ppc=args.ppc)
    params = launch_params(cfg, args)
    pushes, elapsed, prof, st, steps, warmup = run_timed(cfg, args, args.steps, args.warmup, params)
    bpp = BYTES_PER_PUSH[args.precision]
    launches = max(prof["launches"], 1)
    push_ms = prof["ms"] / launches
    bytes_per_launch = bpp * prof["pushes"] / launches
    achieved = bytes_per_launch / (push_ms * 1e-3) / 1e9
    traffic = traffic_for(args.ppc, params["chunk"])
    line = {
        "metric": METRIC,
        "value": pushes / elapsed,
        "unit": "particle-pushes/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": elapsed * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": (f"1D3V argon sheath, 2048 cells over 1024 Debye lengths, {args.ppc} particles/cell/"
                         f"species ({2 * 2048 * args.ppc} particles at load), Te/Ti=20, u={args.u} v_ti, "
                         f"dt={cfg['dt']:.4g}/omega_pe, cell sort every {params['sort_every']} steps"),
            "particles": 2 * 2048 * args.ppc,
            "u_over_vti": args.u,
            "dt": cfg["dt"],
            "launch": params,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "k_push_deposit",
            "bytes_per_push": bpp,
            "moved_bytes_per_push": MOVED_BYTES_PER_PUSH[args.precision],
            "avg_launch_ms": push_ms,
            "launches": prof["launches"],
            "target_frac": PUSH_TARGET_FRAC,
            "meets_target": achieved / HBM_PEAK_GBS >= PUSH_TARGET_FRAC,
            "limit": None if achieved / HBM_PEAK_GBS >= PUSH_TARGET_FRAC else PUSH_LIMIT_NOTE,
        },
        "wall_potential": st["wall_potential"],
        "error_flags": st["error_flags"],
    }
    line["steps_requested"] = args.steps
    line["warmup_requested"] = args.warmup
    line["steps_note"] = (f"steps and warm-up are rounded up to whole blocks of {max(16, params['sort_every'])} "
                          f"steps, each replayed as one HIP graph")
    if not args.no_u_sweep and args.ppc == 1000:
        # the other speed limits of the production sweep (inf: the PIC step dx/(5 v_te))
        rows = []
        for u in (5.0, 10.0, math.inf):
            cfg_u = workloads.production_sheath(u_over_vti=u, ppc=args.ppc)
            pu = launch_params(cfg_u, args)
            nu, eu, prof_u, st_u, su, _ = run_timed(cfg_u, args, 256, 64, pu)
            lu = max(prof_u["launches"], 1)
            ms_u = prof_u["ms"] / lu
            au = bpp * prof_u["pushes"] / lu / (ms_u * 1e-3) / 1e9
            rows.append({"u_over_vti": None if math.isinf(u) else u, "dt": cfg_u["dt"], "value": nu / eu,
                         "steps": su, "ms_per_step": eu * 1e3 / su, "push_avg_launch_ms": ms_u,
                         "achieved_GBs": au, "frac": au / HBM_PEAK_GBS, "launch": pu,
                         "error_flags": st_u["error_flags"]})
        line["u_sweep"] = rows
        # a developed state: the same sheath timed after two ion transits (L / c_s ~ 1025 steps at u = 2 v_ti)
        nd, ed, prof_d, st_d, sd, wd = run_timed(cfg, args, 512, 2048, params)
        ld = max(prof_d["launches"], 1)
        ms_d = prof_d["ms"] / ld
        ad = bpp * prof_d["pushes"] / ld / (ms_d * 1e-3) / 1e9
        line["developed_state"] = {"warmup": wd, "steps": sd, "value": nd / ed, "ms_per_step": ed * 1e3 / sd,
                                   "push_avg_launch_ms": ms_d, "achieved_GBs": ad, "frac": ad / HBM_PEAK_GBS,
                                   "wall_potential": st_d["wall_potential"], "error_flags": st_d["error_flags"]}
    if not args.no_steady:
        line["time_to_steady"] = time_to_steady(args)
    if not args.no_hbm_variant and args.ppc == 1000:
        # the same sheath with 10x the particles per cell (41M particles,
        # 655 MB of particle state: larger than the 256 MB Infinity Cache)
        cfg10 = workloads.production_sheath(u_over_vti=args.u, ppc=10 * args.ppc)
        params10 = launch_params(cfg10, args)
        p10, e10, prof10, _, s10, _ = run_timed(cfg10, args, 256, 64, params10)
        l10 = max(prof10["launches"], 1)
        ms10 = prof10["ms"] / l10
        a10 = bpp * prof10["pushes"] / l10 / (ms10 * 1e-3) / 1e9
        line["hbm_variant"] = {"particles": 2 * 2048 * 10 * args.ppc, "value": p10 / e10, "steps": s10,
                               "launch": params10, "push_avg_launch_ms": ms10, "achieved_GBs": a10,
                               "frac": a10 / HBM_PEAK_GBS, "bound": "hbm", "peak": HBM_PEAK_GBS,
                               "bytes_per_push": bpp, "moved_bytes_per_push": MOVED_BYTES_PER_PUSH[args.precision],
                               "target_frac": PUSH_TARGET_FRAC, "meets_target": a10 / HBM_PEAK_GBS >= PUSH_TARGET_FRAC,
                               "traffic": traffic_for(10 * args.ppc, params10["chunk"])}
    if not args.no_2d:
        line["sheath_2d"] = run_2d(args)
    if not args.no_wave:
        line["wave_test"] = run_wave(args)
    if not args.no_plates:
        line["plates_sheath"] = run_plates(args, args.plates_ppc, args.plates_runs)
    if not args.no_langmuir:
        line["plasma_frequency"] = run_langmuir(args)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

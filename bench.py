"""Benchmark: SLPIC particle pushes per second on one MI355X.

Workload: the 1D argon sheath at production shape -- 2048 cells over 1024
Debye lengths, 1000 macroparticles per cell per species (4,096,000
particles), Te = 1 eV, Ti = 0.05 eV, speed limit u = 2 v_ti, FP32 particles
(int32 fixed-point positions, float velocities) with FP64 grids.  A step is
one pass of the whole hot path: push + beta-weighted deposit, wall
absorption, source injection, field solve and the periodic cell sort.

Prints one JSON line.  `value` is live particle pushes per second over the
timed steps (whole step time); `roofline` prices the dominant kernel
(push + deposit) by its algorithmic bytes over its average launch time,
measured with HIP events on the launch stream inside the timed region.
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
BYTES_PER_PUSH_F32 = 20  # read x, vx, vperp^2 (12 B); write x, vx (8 B)
BYTES_PER_PUSH_F64 = 40


def cpu_baseline(cfg: dict, budget_s: float = 12.0) -> dict:
    """The FP64 oracle (single thread, as written) on a bounded sample of the
    same workload: the full particle count, as many steps as fit the budget."""
    import oracle
    run = oracle.Run(dict(cfg, sort_every=16))
    n0 = sum(run.nlive(s) for s in range(2))
    steps, t0 = 0, time.perf_counter()
    while True:
        run.step(1)
        steps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": n0 * steps / dt, "unit": "particle-pushes/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the same sheath ({n0} particles), FP64 C oracle, 1 thread"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--u", type=float, default=2.0, help="speed limit in ion thermal speeds (inf = PIC)")
    ap.add_argument("--ppc", type=int, default=1000)
    ap.add_argument("--sort-every", type=int, default=16)
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", default="", help="JSON with measured HBM bytes per push launch")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        return 2

    import torch
    import workloads
    from paper_1511_08225_amd import slpic

    cfg = workloads.production_sheath(u_over_vti=args.u, ppc=args.ppc, sort_every=args.sort_every)
    sim = slpic.Sim(cfg, precision=args.precision, sort_every=args.sort_every)
    torch.cuda.synchronize()
    sim.step(args.warmup)
    torch.cuda.synchronize()

    sim.profile(True)
    p0 = sim.pushed_total()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pushes = sim.pushed_total() - p0
    prof = sim.profile_read()
    sim.profile(False)
    st = sim.status(0)

    elapsed = t1 - t0
    value = pushes / elapsed
    bpp = BYTES_PER_PUSH_F32 if args.precision == "f32" else BYTES_PER_PUSH_F64
    push_ms = prof["push"]["ms"] / max(prof["push"]["launches"], 1)
    bytes_per_launch = bpp * pushes / max(prof["push"]["launches"], 1)
    achieved = bytes_per_launch / (push_ms * 1e-3) / 1e9
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        traffic = json.load(open(args.traffic)).get("bytes_per_launch")
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": (f"1D3V argon sheath, 2048 cells over 1024 Debye lengths, {args.ppc} particles/cell/"
                         f"species ({2 * 2048 * args.ppc} particles), Te/Ti=20, u={args.u} v_ti, "
                         f"dt={cfg['dt']:.4g}/omega_pe, sort every {args.sort_every} steps"),
            "particles": 2 * 2048 * args.ppc,
            "u_over_vti": args.u,
            "dt": cfg["dt"],
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
            "avg_launch_ms": push_ms,
        },
        "kernel_ms_per_step": {k: v["ms"] / max(v["launches"], 1) for k, v in prof.items()},
        "wall_potential": st["wall_potential"],
        "error_flags": st["error_flags"],
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

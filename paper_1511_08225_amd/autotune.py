"""Launch-parameter tuner for a set of runs.

Chooses the push chunk (particles per wavefront), the push workgroup size,
the sort period, the sort key bucket, the push order of the species' chunks
and the sort tile (slots per sort workgroup) for a given run set by timing short
trials of the real step on the GPU (coordinate descent over the candidate
lists), and caches the choice per workload signature in a JSON file so that
later contexts over similar run sets start tuned.  The sort schedule changes
only the slot order (the physics is the same up to FP64 summation order), so
every candidate is a valid setting.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import slpic

CANDIDATES = {
    "chunk": (128, 256, 512, 1024),
    "block": (64, 128, 256),
    "sort_every": (8, 16, 32, 64),
    "sort_bucket": (1, 2, 4),
    "push_order": (0, 1),
    "sort_tile": (2048, 4096, 8192, 16384, 32768),
}
DEFAULT = {"chunk": 512, "block": 128, "sort_every": 16, "sort_bucket": 1, "push_order": 0, "sort_tile": 16384}
GROUPS = (("chunk", "block"), ("sort_every",), ("sort_bucket",), ("push_order",), ("sort_tile",))
SWITCH_MARGIN = 0.01  # relative gain a trial needs to replace the incumbent
CACHE_PATH = os.environ.get("SLPIC_TUNING_CACHE",
                            os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json"))


def signature(configs: list[dict], precision: str) -> str:
    """Workload key: precision, run count, total particles and mean cells
    (each rounded to a power of two), mean speed limit in ion thermal speeds
    (rounded to an integer)."""
    n = len(configs)
    parts = sum(c["nx"] * sum(s["ppc"] for s in c["species"]) for c in configs)
    cells = sum(c["nx"] for c in configs) / n
    k = sum(c.get("u_over_vti", 0.0) if math.isfinite(c.get("u_over_vti", math.inf)) else 0.0
            for c in configs) / n
    return (f"{precision}|runs={1 << max(0, round(math.log2(n)))}|particles=2^{round(math.log2(max(parts, 1)))}"
            f"|cells={1 << round(math.log2(max(cells, 1)))}|u={round(k)}")


def _load_cache(path: str) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


MIN_TRIAL_SECONDS = 0.025  # a trial's timed steps span at least this (small run sets: more steps)
MAX_TRIAL_STEPS = 4096


def measure(configs: list[dict], precision: str, params: dict, steps: int = 64, warmup: int = 32) -> float:
    """Seconds per particle-step of the whole step (push, source, field,
    amortised sort) with these parameters, over graph-replayed steps after
    `warmup` steps from the cold load: `steps`, or as many more whole graph
    blocks (at most MAX_TRIAL_STEPS) as the warm-up's pace says span
    MIN_TRIAL_SECONDS, so that host timing noise stays small for small run
    sets; infinite if any run raised an error flag (a sort period too long
    for its slot headroom overflows)."""
    se = params["sort_every"]
    g = max(16, se)
    steps = max(g, (steps // g) * g)
    warmup = max(2 * g, (warmup // g) * g)  # the first block captures the graph; the last one is timed
    sim = slpic.Sim(configs, precision=precision, sort_every=se, sort_bucket=params["sort_bucket"],
                    chunk=params["chunk"], block=params["block"], graph_steps=g,
                    push_order=params.get("push_order", 0), sort_tile=params.get("sort_tile", 0))
    try:
        sim.step(warmup - g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(g)  # the last warm-up block, timed for the pace
        torch.cuda.synchronize()
        per_step = (time.perf_counter() - t0) / g
        want = math.ceil(MIN_TRIAL_SECONDS / max(per_step, 1e-9) / g) * g
        steps = min(max(steps, want), max(steps, MAX_TRIAL_STEPS // g * g))
        p0 = sim.pushed_total()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        pushes = sim.pushed_total() - p0
        flagged = any(s["error_flags"] for s in sim.status())
    finally:
        sim.close()
    return math.inf if flagged else dt / max(pushes, 1)


def cached(configs: list[dict], precision: str = "f32", cache_path: str = CACHE_PATH) -> dict | None:
    """The cached parameters of this run set's signature (complete entries
    only), without measuring anything; None if there are none."""
    entry = _load_cache(cache_path).get(signature(configs, precision))
    if entry and all(k in entry["params"] for k in DEFAULT):
        return dict(entry["params"])
    return None


def tune(configs: list[dict], precision: str = "f32", cache_path: str = CACHE_PATH, force: bool = False,
         steps: int = 64, warmup: int = 32, log=None, measure_fn=None) -> dict:
    """Best parameters for this run set (cached by signature).  measure_fn
    (configs, precision, params, steps, warmup) -> seconds per particle-step
    defaults to timing the real step on the GPU."""
    measure_fn = measure_fn or measure
    key = signature(configs, precision)
    cache = _load_cache(cache_path)
    groups, best, earlier = GROUPS, dict(DEFAULT), []
    if not force and key in cache:
        cached = cache[key]["params"]
        if all(k in cached for k in DEFAULT):
            return dict(cached)
        # an entry from before a parameter existed: continue from its best
        # over the groups it lacks (its own trials are kept apart: they were
        # timed in another session)
        best = dict(DEFAULT, **cached)
        groups = tuple(g for g in GROUPS if any(n not in cached for n in g))
        earlier = cache[key].get("earlier_trials", []) + cache[key].get("trials", [])
    best_t = measure_fn(configs, precision, best, steps, warmup)
    trials = [(dict(best), best_t)]
    for group in groups:
        options = [{}]
        for name in group:
            options = [dict(o, **{name: v}) for o in options for v in CANDIDATES[name]]
        for opt in options:
            p = dict(best, **opt)
            if any(p == q for q, _ in trials):  # measured already
                continue
            t = measure_fn(configs, precision, p, steps, warmup)
            trials.append((dict(p), t))
            if log:
                log(f"trial {p}: {t * 1e12:.2f} ps/push")
            if t < best_t * (1.0 - SWITCH_MARGIN):  # a change must beat the incumbent beyond noise
                best, best_t = p, t
    cache[key] = {"params": best, "ps_per_push": best_t * 1e12,
                  "trials": [{"params": p, "ps_per_push": t * 1e12} for p, t in trials]}
    if earlier:
        cache[key]["earlier_trials"] = earlier
    os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
    with open(cache_path, "w") as f:
        json.dump(cache, f, indent=1)
    return dict(best)

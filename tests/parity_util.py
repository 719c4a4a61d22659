"""Helpers shared by the GPU parity tests: move an oracle state into the HIP
library (through the C ABI) and compare the two sides.  Every input comes
from the oracle or from the seeded workload definitions."""
import math

import numpy as np

import oracle


def print_case(msg: str):
    print(f"[case] {msg}", flush=True)


def oracle_state(run: "oracle.Run", s: int):
    x, vx, vy, vz = run.particles(s)
    return x, vx, vy * vy + vz * vz


def quantize_for_f32(x, vx, vp2, fixed_bits):
    """The representation an F32 context stores: int32 fixed-point positions
    (round to nearest even), float32 velocities."""
    scale = math.ldexp(1.0, fixed_bits)
    xq = np.where(x < 0, -1.0, np.rint(x * scale) / scale)
    return xq, vx.astype(np.float32).astype(np.float64), vp2.astype(np.float32).astype(np.float64)


def set_oracle_particles(run: "oracle.Run", s: int, x, vx, vp2):
    """Give the oracle a state whose |v_perp|^2 is vp2 (v_perp along y)."""
    run.set_particles(s, x, vx, np.sqrt(vp2), np.zeros_like(vp2))


def bench_launch(cfg: dict, precision: str = "f32") -> dict:
    """The launch parameters the benchmark runs this workload with: the
    autotuner's committed cache entry for its signature (no measuring)."""
    from paper_1511_08225_amd import autotune
    p = autotune.cached([cfg], precision)
    assert p is not None, "no tuned launch cached for " + autotune.signature([cfg], precision)
    return p


def push_oracle_to_gpu(sim, r: int, run: "oracle.Run", quantize: bool):
    st = sim.status(r)
    for s in range(2):
        x, vx, vp2 = oracle_state(run, s)
        if quantize:
            x, vx, vp2 = quantize_for_f32(x, vx, vp2, st["fixed_bits"])
            set_oracle_particles(run, s, x, vx, vp2)
        sim.import_particles(r, s, x, vx, vp2)
    sim.set_counters(r, run.step_index, run.acc_e)
    if run.cfg.get("geometry") == "plates":
        sim.set_flux_counters(r, run.acc_flux())
    run.refresh_fields()
    sim.refresh_fields()


def rel_inf(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def cells_agree(xg, xo, tol):
    """Cell indices equal wherever the oracle position is farther than tol
    from a cell edge (dead slots must agree exactly)."""
    dead_g, dead_o = xg < 0, xo < 0
    assert np.array_equal(dead_g, dead_o)
    live = ~dead_o
    cg = np.floor(xg[live]).astype(np.int64)
    co = np.floor(xo[live]).astype(np.int64)
    frac = xo[live] - co
    clear = (frac > tol) & (frac < 1 - tol)
    return bool(np.array_equal(cg[clear], co[clear])), int((~clear).sum())

"""A change of the speed limit mid-run on the HIP path (slpic_set_speed_limit)
against the oracle, raised or lowered: FP64 resampling bit-exact (the same
copies in the same slots), the new weights, the recomputed fields, and
lockstep steps at the new limit and time step; FP32 counts; a batched
context where one run changes; and the paper's use, raising the limit to
verify the result: the two-plate sheath run as SLPIC to 16 us and then as
PIC reaches the PIC steady state."""
import math

import numpy as np
import pytest

import oracle
import workloads
from parity_util import oracle_state, print_case, push_oracle_to_gpu, rel_inf

pytestmark = pytest.mark.gpu


def _exact(sim, run, r=0):
    for s in range(2):
        xg, vxg, vpg = sim.export_particles(r, s)
        xo, vxo, vpo = oracle_state(run, s)
        assert len(xg) == len(xo), (s, len(xg), len(xo))
        assert np.array_equal(xg, xo) and np.array_equal(vxg, vxo) and np.array_equal(vpg, vpo), s


@pytest.mark.parametrize("case", ["sheath_x3", "sheath_pic", "periodic_pic", "plates_x4", "sheath_lower",
                                  "periodic_lower"])
def test_resampling_bit_exact_f64(gpu_lib, case):
    if case.startswith("sheath"):
        cfg = workloads.small_sheath(sort_every=1, seed=61)
        warm = 30
    elif case.startswith("periodic"):
        cfg = workloads.langmuir_box(0.3 if case == "periodic_pic" else 1.0, nx=64, ppc=100, seed=62,
                                     sort_every=1)
        cfg["capacity_factor"] = 1.5  # a lowering may add copies
        warm = 10
    else:
        cfg = workloads.plates_sheath(0.0158, ppc=40, sort_every=1, seed=63)
        warm = 200
    u_new = {"sheath_x3": 3 * cfg["u"], "sheath_pic": math.inf, "periodic_pic": math.inf,
             "plates_x4": 4 * cfg["u"], "sheath_lower": cfg["u"] / 3, "periodic_lower": 0.2}[case]
    dt_new = cfg["dx"] / 5.0 if math.isinf(u_new) else cfg["dx"] / u_new
    if case.startswith("sheath"):
        dt_new = min(cfg["dt"], dt_new) if not math.isinf(u_new) else 0.1
    run = oracle.Run(cfg)
    run.step(warm)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=1)
    push_oracle_to_gpu(sim, 0, run, quantize=False)
    print_case(f"speed limit {case}: resample")
    sim.set_speed_limit(0, u_new, dt_new)
    run.set_speed_limit(u_new, dt_new)
    _exact(sim, run)
    st = sim.status(0)
    for s in range(2):
        assert st["weight"][s] == pytest.approx(run.weight(s), rel=1e-12)
    g, o = sim.grid(0), run.grid()
    for s in range(2):
        assert rel_inf(g["Q"][s], o["Q"][s]) <= 1e-12
    assert rel_inf(g["E"], o["E"]) <= 1e-10
    for k in range(5):  # the new limit and step in the push and the source
        push_oracle_to_gpu(sim, 0, run, quantize=False)
        sim.step(1)
        run.step(1)
        g, o = sim.grid(0), run.grid()
        for s in range(2):
            assert rel_inf(g["Q"][s], o["Q"][s]) <= 1e-12, (k, s)


def test_resampling_f32_counts(gpu_lib):
    cfg = workloads.langmuir_box(0.3, nx=128, ppc=400, seed=64, sort_every=16)
    run = oracle.Run(cfg)
    sim = gpu_lib.Sim(cfg, precision="f32", sort_every=16)
    push_oracle_to_gpu(sim, 0, run, quantize=True)
    sim.set_speed_limit(0, 1.0, 0.5)
    run.set_speed_limit(1.0, 0.5)
    st = sim.status(0)
    for s in range(2):
        # float velocities move beta, and so p, by ~1e-7: a handful of draws flip
        assert abs(st["nslots"][s] - run.nslots(s)) <= 5, s
        assert st["weight"][s] == pytest.approx(run.weight(s), rel=1e-12)
    g, o = sim.grid(0), run.grid()
    for s in range(2):
        assert rel_inf(g["Q"][s], o["Q"][s]) <= 5e-3, s


def test_batched_only_one_run_changes(gpu_lib):
    """Run 1 of two changes its limit; run 0 keeps its live particles (the
    shared resampling pass only compacts it) and steps on as before."""
    a = workloads.small_sheath(sort_every=0, seed=65)
    b = dict(workloads.small_sheath(sort_every=0, seed=66), run=1)
    ra, rb = oracle.Run(a), oracle.Run(b)
    ra.step(20)
    rb.step(20)
    sim = gpu_lib.Sim([a, b], precision="f64", sort_every=0)
    push_oracle_to_gpu(sim, 0, ra, quantize=False)
    push_oracle_to_gpu(sim, 1, rb, quantize=False)
    live0 = [oracle_state(ra, s) for s in range(2)]
    sim.set_speed_limit(1, 3 * b["u"], b["dt"] / 3)
    rb.set_speed_limit(3 * b["u"], b["dt"] / 3)
    _exact(sim, rb, r=1)
    for s in range(2):
        xg, vxg, vpg = sim.export_particles(0, s)
        keep = live0[s][0] >= 0
        assert np.array_equal(xg, live0[s][0][keep]) and np.array_equal(vxg, live0[s][1][keep])
    st = sim.status()
    assert st[0]["weight"] == pytest.approx([ra.weight(0), ra.weight(1)], rel=1e-12)
    for bad in ((0.0, a["dt"]), (0.5 * a["u"], 0.0)):
        with pytest.raises(gpu_lib.SlpicError):
            sim.set_speed_limit(0, *bad)


def test_raise_to_pic_reaches_the_pic_steady_state(gpu_lib):
    """The paper's use of a time-varying limit, to verify the approximation:
    the two-plate sheath (2000 g-particles per cell at n0, two seeds) run as
    SLPIC (v0 = 0.0158 v_te) to 16 us, then raised to u = inf with the PIC
    step for 8 us, against pure PIC runs: the time averages over the last
    4 us agree within noise (phi 2 %, n_e and n_i 5 %)."""
    import torch
    ppc, seeds = 2000, 2
    sl = workloads.plates_sheath(0.0158, ppc=ppc, sort_every=16, capacity_factor=0.5)
    pic = workloads.plates_sheath(math.inf, ppc=ppc, sort_every=16, capacity_factor=0.5)
    out = {}
    with torch.cuda.stream(torch.cuda.Stream()):
        for name in ("switched", "pic"):
            cfg = sl if name == "switched" else pic
            sim = gpu_lib.Sim([dict(cfg, seed=700 + r, run=r) for r in range(seeds)], precision="f32",
                              sort_every=16, graph_steps=16, chunk=256, sort_tile=2048)
            if name == "switched":
                sim.step(workloads.plates_steps(sl, 16.0))
                for r in range(seeds):
                    sim.set_speed_limit(r, math.inf, pic["dt"])
                left = workloads.plates_steps(pic, 8.0)
            else:
                left = workloads.plates_steps(pic, 24.0)
            sample = workloads.plates_steps(pic, 4.0)
            sim.step(left - sample)
            for _ in range(sample // 320):
                sim.step(320)
                sim.moments_sample(-1)
            out[name] = np.mean([sim.moments_window(r).cpu().numpy() for r in range(seeds)], axis=0)
            st = sim.status()
            assert all(x["error_flags"] == 0 for x in st), st
            print_case(f"{name}: particles {st[0]['nslots']}")
            sim.close()
    for row, name, tol in ((0, "phi", 0.02), (1, "n_e", 0.05), (4, "n_i", 0.05)):
        a, b = out["switched"][row][1:-1], out["pic"][row][1:-1]
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        print_case(f"raised-to-PIC vs PIC: {name} rel L2 {err:.4f}")
        assert err <= tol, (name, err)

"""The two-plate sheath of Sec. IV on the HIP path against the oracle,
through the C ABI: the empty box's vacuum field, the flux injection through
the plate at x = L (counts exact, particles element by element), absorption
at both plates, the Dirichlet field solve, the monitored mid-plane
potential, the steady detector fed by it, and a plates run batched with a
sheath run.  Tolerances as in the sheath parity tests: FP64 charge per
species within 1e-12 of its infinity norm, FP32 within 1e-5."""
import math

import numpy as np
import pytest

import oracle
import workloads
from parity_util import cells_agree, oracle_state, print_case, push_oracle_to_gpu, rel_inf

pytestmark = pytest.mark.gpu

V_ABS_TOL = 1e-11


def _plates(v0=0.0158, ppc=40, **kw):
    return workloads.plates_sheath(v0, ppc=ppc, **kw)


def _compare_particles(sim, run, r=0, tol_x=1e-11, tol_v=1e-11, v_abs=V_ABS_TOL):
    for s in range(2):
        xg, vxg, vpg = sim.export_particles(r, s)
        xo, vxo, vpo = oracle_state(run, s)
        assert len(xg) == len(xo), (s, len(xg), len(xo))
        np.testing.assert_allclose(xg, xo, rtol=0, atol=tol_x)
        np.testing.assert_allclose(vxg, vxo, rtol=tol_v, atol=v_abs)
        np.testing.assert_allclose(vpg, vpo, rtol=1e-13, atol=0)
        ok, _ = cells_agree(xg, xo, max(tol_x, 1e-12))
        assert ok, s


def _compare_grid(sim, run, r=0, tol_q=1e-12, tol_phi=1e-11):
    g, o = sim.grid(r), run.grid()
    for s in range(2):
        if np.abs(o["Q"][s]).max() > 0:
            assert rel_inf(g["Q"][s], o["Q"][s]) <= tol_q, s
        else:
            assert np.abs(g["Q"][s]).max() == 0.0
    assert rel_inf(g["phi"], o["phi"]) <= tol_phi
    assert rel_inf(g["E"], o["E"]) <= 10 * tol_phi
    return g, o


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_empty_box_vacuum_field(gpu_lib, prec):
    cfg = _plates(sort_every=1)
    print_case(f"plates empty box {prec}")
    sim = gpu_lib.Sim(cfg, precision=prec, sort_every=1)
    st = sim.status(0)
    assert st["nslots"] == [0, 0]
    for s in range(2):
        assert st["weight"][s] == pytest.approx(oracle.weight(cfg, s), rel=1e-12)
    g = sim.grid(0)
    L = cfg["nx"] * cfg["dx"]
    x = np.arange(cfg["nx"] + 1) * cfg["dx"]
    assert np.abs(g["Q"]).max() == 0.0
    assert np.abs(g["phi"] - cfg["bias"] * x / L).max() <= 1e-13 * cfg["bias"]
    assert np.abs(g["E"] + cfg["bias"] / L).max() <= 1e-12 * cfg["bias"] / L
    assert g["phi"][0] == 0.0 and g["phi"][-1] == cfg["bias"]
    assert st["wall_potential"] == pytest.approx(cfg["bias"] / 2, rel=1e-13)
    sim.close()


@pytest.mark.parametrize("kind", ["step", "smooth"])
def test_lockstep_from_empty_f64(gpu_lib, kind):
    """150 steps from the empty box: the oracle's state at step k goes into
    the library and both take step k+1 (the library injects with its own
    generator and carries its own flux fractions)."""
    cfg = _plates(sort_every=1, beta_kind=kind, seed=21)
    run = oracle.Run(cfg)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=1)
    for k in range(150):
        if k % 50 == 0:
            print_case(f"plates lockstep {kind} step {k}")
        push_oracle_to_gpu(sim, 0, run, quantize=False)
        sim.step(1)
        run.step(1)
        _compare_grid(sim, run)
        st = sim.status(0)
        for s in range(2):
            assert st["injected_total"][s] == run.injected_total(s), (k, s)
            assert st["acc_flux"][s] == pytest.approx(run.acc_flux()[s], abs=1e-12)
        if k % 25 == 24:
            _compare_particles(sim, run)
            assert st["wall_potential"] == pytest.approx(run.grid()["phi"][cfg["nx"] // 2], rel=1e-12)
    assert sum(run.absorbed_total(s) for s in range(2)) > 0  # particles reached a plate


def test_free_run_from_empty_f64(gpu_lib):
    """60 steps without state transfer: counts, absorbed totals, the steady
    detector's windows and every particle as in the oracle's own run."""
    cfg = _plates(sort_every=4, seed=22)
    cfg["steady_window"] = 10
    run = oracle.Run(cfg)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=4)
    print_case("plates free run f64")
    sim.step(60)
    run.step(60)
    st = sim.status(0)
    for s in range(2):
        assert st["injected_total"][s] == run.injected_total(s)
        assert st["absorbed_total"][s] == run.absorbed_total(s)
    _compare_grid(sim, run, tol_q=1e-10, tol_phi=1e-10)
    _compare_particles(sim, run, tol_x=1e-9, tol_v=1e-9, v_abs=1e-9)
    od = run.steady()
    assert st["windows"] == od["windows"] == 6
    for a, b in zip(st["window_mean"], od["window_mean"]):
        assert a == pytest.approx(b, rel=1e-10)
    hist = sim.wall_history(0)
    assert hist[-1] == pytest.approx(st["wall_potential"], rel=0, abs=0)


def test_developed_state_f64_and_f32(gpu_lib):
    """After 400 oracle steps (the box filled, both plates absorbing): five
    FP64 lockstep steps, then one FP32 step within 1e-5."""
    cfg = _plates(sort_every=1, seed=23)
    run = oracle.Run(cfg)
    run.step(400)
    n = [run.nslots(s) for s in range(2)]
    assert min(n) > 200, n
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=1)
    for k in range(5):
        print_case(f"plates developed f64 step {k}")
        push_oracle_to_gpu(sim, 0, run, quantize=False)
        sim.step(1)
        run.step(1)
        _compare_grid(sim, run)
        _compare_particles(sim, run)
    sim.close()
    sim32 = gpu_lib.Sim(cfg, precision="f32", sort_every=1)
    print_case("plates developed f32 one step")
    push_oracle_to_gpu(sim32, 0, run, quantize=True)
    before = [run.injected_total(s) for s in range(2)]
    sim32.step(1)
    run.step(1)
    g, o = sim32.grid(0), run.grid()
    for s in range(2):
        assert rel_inf(g["Q"][s], o["Q"][s]) <= 1e-5, s
    assert rel_inf(g["phi"], o["phi"]) <= 1e-5
    st = sim32.status(0)  # a fresh context: its totals count this one step
    for s in range(2):
        assert st["injected_total"][s] == run.injected_total(s) - before[s]


def test_unlimited_speed_plates_is_pic_f64(gpu_lib):
    """u = inf (beta = 1) with dt = dx/(5 v_te): 40 lockstep steps."""
    cfg = _plates(math.inf, ppc=20, sort_every=1, seed=24)
    run = oracle.Run(cfg)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=1)
    print_case("plates pic lockstep")
    for k in range(40):
        push_oracle_to_gpu(sim, 0, run, quantize=False)
        sim.step(1)
        run.step(1)
        _compare_grid(sim, run)
    _compare_particles(sim, run)


def test_plates_batched_with_sheath(gpu_lib):
    """A plates run and a sheath run in one context, each against its own
    oracle after 30 free steps."""
    pl = _plates(sort_every=2, seed=25)
    sh = dict(workloads.small_sheath(sort_every=2, seed=26), run=1)
    sim = gpu_lib.Sim([pl, sh], precision="f64", sort_every=2)
    runs = [oracle.Run(pl), oracle.Run(sh)]
    print_case("plates + sheath batched")
    sim.step(30)
    for r, orun in enumerate(runs):
        orun.step(30)
        st = sim.status(r)
        for s in range(2):
            assert st["injected_total"][s] == orun.injected_total(s), (r, s)
        _compare_grid(sim, orun, r=r, tol_q=1e-10, tol_phi=1e-10)
        _compare_particles(sim, orun, r=r, tol_x=1e-9, tol_v=1e-9, v_abs=1e-9)
    assert sim.status(0)["wall_potential"] == pytest.approx(runs[0].grid()["phi"][pl["nx"] // 2], rel=1e-10)
    assert sim.status(1)["wall_potential"] == pytest.approx(runs[1].wall_potential(), rel=1e-10)


def test_flux_counters_argument_checks(gpu_lib):
    sim = gpu_lib.Sim(workloads.small_sheath(sort_every=0), precision="f64", sort_every=0)
    with pytest.raises(gpu_lib.SlpicError):
        sim.set_flux_counters(0, [0.5, 0.5])  # not a plates run
    sim.close()
    sim = gpu_lib.Sim(_plates(sort_every=0), precision="f64", sort_every=0)
    with pytest.raises(gpu_lib.SlpicError):
        sim.set_flux_counters(0, [1.0, 0.0])
    sim.set_flux_counters(0, [0.25, 0.75])
    assert sim.status(0)["acc_flux"] == [0.25, 0.75]
    sim.close()


def _to_24us(gpu_lib, v0, ppc, runs):
    """Runs of the plates workload from the empty box to 24 us, FP32, with
    the moments averaged over the last 8 us; returns the run-mean profiles
    (phi, n_e, n_i), the step count and the final status of run 0."""
    import torch
    cfg = workloads.plates_sheath(v0, ppc=ppc, sort_every=16, capacity_factor=0.5)
    total = workloads.plates_steps(cfg, 24.0)
    avg = workloads.plates_steps(cfg, 8.0)
    stride = 1 if avg < 400 else avg // 200 // 16 * 16
    nsamp = avg // stride
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim = gpu_lib.Sim([dict(cfg, seed=500 + r, run=r) for r in range(runs)], precision="f32", sort_every=16,
                          graph_steps=16, chunk=256, sort_tile=2048)
        sim.step(total - nsamp * stride)
        if stride == 1:
            sim.set_sampling(1)
            sim.step(nsamp)
        else:
            for _ in range(nsamp):
                sim.step(stride)
                sim.moments_sample(-1)
        win = np.mean([sim.moments_window(r).cpu().numpy() for r in range(runs)], axis=0)
        st = sim.status()
        sim.close()
    assert all(s["error_flags"] == 0 for s in st)
    assert all(s["moment_samples"] == nsamp for s in st)
    return win[[0, 1, 4]], total, st[0]


def test_slpic_reaches_the_pic_steady_state(gpu_lib):
    """The paper's sheath experiment at reduced particle count (2000
    g-particles per cell at n0, two seeds per side): after 24 us from the
    empty box, SLPIC at v0 = 0.0158 v_te (590 steps) and PIC (186625 steps)
    give the same time-averaged potential and densities within noise, and
    the particle counts of both sides settle near each other."""
    sl, n_sl, st_sl = _to_24us(gpu_lib, 0.0158, 2000, 2)
    print_case("plates physics: PIC leg")
    pic, n_pic, st_pic = _to_24us(gpu_lib, math.inf, 2000, 2)
    assert n_sl == 590 and n_pic == 186625
    names = ("phi", "n_e", "n_i")
    tol = (0.02, 0.04, 0.04)
    for k in range(3):
        a, b = sl[k][1:-1], pic[k][1:-1]
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        print_case(f"plates physics: {names[k]} rel L2 {err:.4f}")
        assert err <= tol[k], (names[k], err)
    # the sheath: phi rises from the grounded plate to the bias (every 5 nodes)
    phi = pic[0]
    assert np.all(np.diff(phi[::5]) > 0)
    # ions reach the grounded plate: their density there is a sizeable
    # fraction of the mid-gap density, electrons are repelled from it
    mid = len(phi) // 2
    assert pic[2][1] > 0.5 * pic[2][mid] and pic[1][1] < 0.1 * pic[1][mid]
    for s in range(2):
        assert abs(st_sl["nslots"][s] - st_pic["nslots"][s]) <= 0.5 * st_pic["nslots"][s]

"""A speed limit varying with position, v0(x), on the HIP path against the
oracle: the cold load cell by cell (counts and positions exact, velocities
to 1e-12), FP64 lockstep steps in the sheath, periodic and plates
geometries (charge per species within 1e-12 of its infinity norm), FP32
steps within 1e-5 (also at the production size in the benchmark's launch
configuration), a context mixing profile runs with uniform and unlimited
ones, and the calls that must refuse a profile."""
import math

import numpy as np
import pytest

import oracle
import workloads
from parity_util import (bench_launch, cells_agree, oracle_state, print_case, push_oracle_to_gpu, quantize_for_f32,
                         rel_inf)

pytestmark = pytest.mark.gpu


def _profile(nx, u0, depth=0.6, phase=0.0):
    return u0 * (1.0 + depth * np.cos(2.0 * np.pi * np.arange(nx + 1) / nx + phase))


def _rough(nx, u0, seed):
    return u0 * np.random.default_rng(seed).uniform(0.3, 1.7, nx + 1)


def _compare(sim, run, r=0, tol_q=1e-12, tol_x=1e-11, tol_v=1e-11):
    g, o = sim.grid(r), run.grid()
    for s in range(2):
        err = rel_inf(g["Q"][s], o["Q"][s])
        assert err <= tol_q, (s, err)
    for s in range(2):
        xg, vxg, _ = sim.export_particles(r, s)
        xo, vxo, _ = oracle_state(run, s)
        assert len(xg) == len(xo), (s, len(xg), len(xo))
        np.testing.assert_allclose(xg, xo, rtol=0, atol=tol_x)
        np.testing.assert_allclose(vxg, vxo, rtol=tol_v, atol=1e-11)
        ok, _ = cells_agree(xg, xo, max(tol_x, 1e-12))
        assert ok, s


@pytest.mark.parametrize("kind", ["step", "smooth"])
def test_cold_load_matches_oracle(gpu_lib, kind):
    for prec in ("f64", "f32"):
        cfg = workloads.sheath(nx=64, ppc=100, u_over_vti=3.0, dt=5.0, beta_kind=kind, sort_every=0, seed=21)
        cfg["limit_profile"] = _profile(cfg["nx"], cfg["u"])
        print_case(f"limit profile cold load {prec} {kind}")
        sim = gpu_lib.Sim(cfg, precision=prec, sort_every=0)
        run = oracle.Run(cfg)
        st = sim.status(0)
        for s in range(2):
            xg, vxg, vpg = sim.export_particles(0, s)
            xo, vxo, vpo = oracle_state(run, s)
            if prec == "f32":
                xo, vxo, vpo = quantize_for_f32(xo, vxo, vpo, st["fixed_bits"])
            assert len(xg) == len(xo), (s, len(xg), len(xo))
            assert np.array_equal(xg, xo)
            bad = ~(np.isclose(vxg, vxo, rtol=1e-12, atol=0) & np.isclose(vpg, vpo, rtol=1e-12, atol=0))
            assert bad.sum() <= 3, (s, bad.sum())
        if prec == "f64":
            g, o = sim.grid(0), run.grid()
            for s in range(2):
                assert rel_inf(g["Q"][s], o["Q"][s]) <= 1e-9
        sim.close()


@pytest.mark.parametrize("kind", ["step", "smooth"])
def test_lockstep_sheath_f64(gpu_lib, kind):
    """30 steps of a developed 64-cell sheath under a rough random profile
    (nodes 0.3 to 1.7 times u): each step starts both sides from the
    oracle's state."""
    cfg = dict(workloads.small_sheath(sort_every=1, seed=22), beta_kind=kind)
    cfg["limit_profile"] = _rough(cfg["nx"], cfg["u"], 5)
    run = oracle.Run(cfg)
    run.step(40)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=1)
    for k in range(30):
        if k % 10 == 0:
            print_case(f"limit profile lockstep {kind} step {k}")
        push_oracle_to_gpu(sim, 0, run, quantize=False)
        sim.step(1)
        run.step(1)
        _compare(sim, run)


@pytest.mark.parametrize("geometry", ["periodic", "plates"])
def test_lockstep_other_geometries_f64(gpu_lib, geometry):
    if geometry == "periodic":
        cfg = workloads.langmuir_box(0.5, nx=64, ppc=100, seed=23, sort_every=1)
        cfg["limit_profile"] = _profile(64, 0.5, phase=0.7)
        cfg["dt"] = cfg["dx"] / cfg["limit_profile"].max()
        warm = 20
    else:
        cfg = workloads.plates_sheath(0.0158, ppc=40, sort_every=1, seed=24)
        cfg["limit_profile"] = _rough(cfg["nx"], cfg["u"], 6)
        warm = 150
    run = oracle.Run(cfg)
    run.step(warm)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=1)
    for k in range(10):
        print_case(f"limit profile {geometry} step {k}")
        push_oracle_to_gpu(sim, 0, run, quantize=False)
        sim.step(1)
        run.step(1)
        _compare(sim, run)


def test_one_step_f32_developed_sheath(gpu_lib):
    cfg = workloads.sheath(nx=256, ppc=200, u_over_vti=3.0, sort_every=1, seed=25)
    cfg["limit_profile"] = _rough(256, cfg["u"], 7)
    run = oracle.Run(cfg)
    run.step(60)
    sim = gpu_lib.Sim(cfg, precision="f32", sort_every=1)
    push_oracle_to_gpu(sim, 0, run, quantize=True)
    sim.step(1)
    run.step(1)
    g, o = sim.grid(0), run.grid()
    for s in range(2):
        err = rel_inf(g["Q"][s], o["Q"][s])
        assert err <= 1e-5, (s, err)
    for s in range(2):
        xg, vxg, _ = sim.export_particles(0, s)
        xo, vxo, _ = oracle_state(run, s)
        n = min(len(xg), len(xo))
        live = (xg[:n] >= 0) & (xo[:n] >= 0)
        assert np.abs(xg[:n][live] - xo[:n][live]).max() <= 1e-5
        assert np.abs(vxg[:n][live] - vxo[:n][live]).max() <= 1e-5 * np.abs(vxo[:n][live]).max()
        assert abs(len(xg) - len(xo)) <= 2


def test_one_step_f32_production_size(gpu_lib):
    """2048 cells, 1000 per cell per species, u = 2 v_ti with a profile from
    0.4 to 1.6 times it, in the push launch the benchmark tunes for the
    uniform limit (the autotuner's cached chunk, workgroup and order)."""
    cfg = workloads.production_sheath(u_over_vti=2.0, sort_every=16)
    cfg["limit_profile"] = _profile(cfg["nx"], cfg["u"], phase=1.3)
    print_case("limit profile f32 production size: oracle load")
    run = oracle.Run(dict(cfg, sort_every=1))
    p = bench_launch(workloads.production_sheath(u_over_vti=2.0))
    sim = gpu_lib.Sim(cfg, precision="f32", sort_every=16, chunk=p["chunk"], block=p["block"],
                      push_order=p["push_order"])
    push_oracle_to_gpu(sim, 0, run, quantize=True)
    for k in range(2):
        print_case(f"limit profile f32 production size step {k}")
        sim.step(1)
        run.step(1)
        g, o = sim.grid(0), run.grid()
        for s in range(2):
            err = rel_inf(g["Q"][s], o["Q"][s])
            assert err <= 1e-5, (k, s, err)
        if k == 0:
            push_oracle_to_gpu(sim, 0, run, quantize=True)


def test_mixed_context_f64(gpu_lib):
    """A profile run, a uniform run and an unlimited run in one context
    (the kernels that read the profiles take the uniform path for the other
    two): each matches its own oracle step by step."""
    a = workloads.small_sheath(sort_every=1, seed=26)
    a["limit_profile"] = _rough(a["nx"], a["u"], 8)
    b = dict(workloads.small_sheath(sort_every=1, seed=27), run=1)
    c = dict(workloads.sheath(nx=64, ppc=50, u_over_vti=math.inf, sort_every=1, seed=28), run=2)
    runs = [oracle.Run(cfg) for cfg in (a, b, c)]
    for r in runs:
        r.step(20)
    sim = gpu_lib.Sim([a, b, c], precision="f64", sort_every=1)
    for k in range(5):
        print_case(f"mixed context step {k}")
        for i, r in enumerate(runs):
            push_oracle_to_gpu(sim, i, r, quantize=False)
        sim.step(1)
        for i, r in enumerate(runs):
            r.step(1)
            _compare(sim, r, r=i)


def test_profile_refusals(gpu_lib):
    cfg = workloads.small_sheath(sort_every=1, seed=29)
    nx = cfg["nx"]
    for bad in (np.zeros(nx + 1), np.full(nx + 1, np.inf)):
        with pytest.raises(gpu_lib.SlpicError):
            gpu_lib.Sim(dict(cfg, limit_profile=bad), precision="f64")
    with pytest.raises(gpu_lib.SlpicError):
        gpu_lib.Sim(dict(cfg, u=math.inf, limit_profile=np.ones(nx + 1)), precision="f64")
    with pytest.raises(gpu_lib.SlpicError):
        gpu_lib.Sim2D(dict(cfg, limit_profile=np.ones(nx + 1)), ny=8, precision="f64")
    sim = gpu_lib.Sim(dict(cfg, limit_profile=_profile(nx, cfg["u"])), precision="f64")
    with pytest.raises(gpu_lib.SlpicError):
        sim.set_speed_limit(0, 2 * cfg["u"], cfg["dt"])
    sim.close()

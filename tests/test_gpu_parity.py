"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Inputs always come from the oracle (its own load and steps from the seeded
workloads); the HIP library receives them through slpic_import_particles
and both sides advance one step.  Tolerances: FP64 particles, grid charge per
species within 1e-12 of its infinity norm; FP32 particles (int32 fixed-point
positions, float velocities), within 1e-5; cell indices and sort
permutations bit-exact where the oracle position is not within rounding of a
cell edge (FP64) or on identical stored positions (sort).
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
import workloads
from parity_util import (bench_launch, cells_agree, oracle_state, print_case, push_oracle_to_gpu, quantize_for_f32,
                         rel_inf, set_oracle_particles)

pytestmark = pytest.mark.gpu


# The exact-integral velocity map inverts G_c(p) = (p s + c^2 asinh(p/c))/2;
# in FP64 both sides carry an absolute velocity error of order
# eps * (p0^2 + c^2) / max(s1, c), up to ~1e-12 v_te for particles slowed
# through zero with a small perpendicular speed.  Velocities are compared
# with that absolute floor (positions inherit it times beta dt/dx).
V_ABS_TOL = 1e-11


def _compare_step(sim, run, r=0, tol_q=1e-12, tol_x=1e-11, tol_v=1e-11, exact_counts=True):
    g = sim.grid(r)
    o = run.grid()
    for s in range(2):
        err = rel_inf(g["Q"][s], o["Q"][s])
        assert err <= tol_q, (s, err)
    st = sim.status(r)
    for s in range(2):
        xg, vxg, vpg = sim.export_particles(r, s)
        xo, vxo, vpo = oracle_state(run, s)
        if exact_counts:
            assert len(xg) == len(xo), (s, len(xg), len(xo))
        n = min(len(xg), len(xo))
        np.testing.assert_allclose(xg[:n], xo[:n], rtol=0, atol=tol_x)
        np.testing.assert_allclose(vxg[:n], vxo[:n], rtol=tol_v, atol=V_ABS_TOL)
        ok, _ = cells_agree(xg[:n], xo[:n], max(tol_x, 1e-12))
        assert ok, s
    return st


def test_cold_load_matches_oracle(gpu_lib):
    for prec in ("f64", "f32"):
        for kind, k in (("step", 3.0), ("smooth", 3.0), ("step", math.inf)):
            cfg = workloads.sheath(nx=64, ppc=100, u_over_vti=k, dt=5.0 if k < 1e9 else 0.1,
                                   beta_kind=kind, sort_every=0, seed=11)
            print_case(f"load {prec} {kind} u/vti={k}")
            sim = gpu_lib.Sim(cfg, precision=prec, sort_every=0)
            run = oracle.Run(cfg)
            st = sim.status(0)
            for s in range(2):
                assert st["weight"][s] == pytest.approx(oracle.weight(cfg, s), rel=1e-12)
                xg, vxg, vpg = sim.export_particles(0, s)
                xo, vxo, vpo = oracle_state(run, s)
                if prec == "f32":
                    xo, vxo, vpo = quantize_for_f32(xo, vxo, vpo, st["fixed_bits"])
                assert len(xg) == len(xo)
                assert np.array_equal(xg, xo)
                # rejection sampling may take another branch when a libm result
                # differs in its last bit: allow a handful of such particles
                bad = ~(np.isclose(vxg, vxo, rtol=1e-12, atol=0) & np.isclose(vpg, vpo, rtol=1e-12, atol=0))
                assert bad.sum() <= 3, bad.sum()
            sim.close()


def _warm_profile(nx_phys_scale=1.0, hot=False):
    """phi, n_e, n_i, Gamma_e, Gamma_i, and (hot) temperature rows T_e from 1
    to 3 T_e, T_i from 1 to 1.5 times the source's (zero rows: the source
    temperatures)."""
    xi = np.arange(256) / 255.0
    p = np.zeros((7, 256))
    p[0] = 5.0 * (1 - xi ** 2)
    p[1] = 1.0 + 0.5 * np.cos(math.pi * xi)
    p[2] = p[1] * (1.0 + 0.05 * xi)
    p[3] = p[1] * 0.2 * xi
    p[4] = p[2] * 0.004 * xi * nx_phys_scale
    if hot:
        p[5] = 1.0 + 2.0 * xi
        p[6] = 0.05 * (1.0 + 0.5 * xi)
    return p


@pytest.mark.parametrize("hot", [False, True])
def test_warm_load_matches_oracle(gpu_lib, hot):
    """Warm load from a smooth profile (density, drifts, and with hot = True
    a temperature per cell): per-cell counts and positions as in the oracle,
    velocities to 1e-12 but for a few rejection flips from last-bit libm
    differences; a cold run beside it in the same context is unaffected."""
    prof = _warm_profile(hot=hot)
    for prec in ("f64", "f32"):
        for kind, k in (("step", 3.0), ("smooth", 3.0), ("step", math.inf)):
            cfg = workloads.sheath(nx=64, ppc=100, u_over_vti=k, dt=5.0 if k < 1e9 else 0.1,
                                   beta_kind=kind, sort_every=0, seed=12)
            cold = dict(cfg, run=1, seed=13)
            print_case(f"warm load {prec} {kind} u/vti={k} hot={hot}")
            sim = gpu_lib.Sim([cfg, cold], precision=prec, sort_every=0, warm=[prof, None])
            run = oracle.Run(cfg, warm=prof)
            run_cold = oracle.Run(cold)
            st = sim.status()
            for r, orun in ((0, run), (1, run_cold)):
                for s in range(2):
                    xg, vxg, vpg = sim.export_particles(r, s)
                    xo, vxo, vpo = oracle_state(orun, s)
                    if prec == "f32":
                        xo, vxo, vpo = quantize_for_f32(xo, vxo, vpo, st[r]["fixed_bits"])
                    assert len(xg) == len(xo), (r, s, len(xg), len(xo))
                    assert np.array_equal(xg, xo)
                    bad = ~(np.isclose(vxg, vxo, rtol=1e-12, atol=0) & np.isclose(vpg, vpo, rtol=1e-12, atol=0))
                    assert bad.sum() <= 3, (r, s, bad.sum())
            if prec == "f64":
                g, o = sim.grid(0), run.grid()
                for s in range(2):
                    assert rel_inf(g["Q"][s], o["Q"][s]) <= 1e-9
            sim.close()


def test_deposit_and_field_match_oracle_f64(gpu_lib):
    cfg = workloads.small_sheath(sort_every=0)
    run = oracle.Run(cfg)
    run.step(20)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=0)
    push_oracle_to_gpu(sim, 0, run, quantize=False)
    g, o = sim.grid(0), run.grid()
    for s in range(2):
        assert rel_inf(g["Q"][s], o["Q"][s]) <= 1e-12
    assert rel_inf(g["phi"], o["phi"]) <= 1e-11
    assert rel_inf(g["E"], o["E"]) <= 1e-10
    assert sim.status(0)["wall_potential"] == pytest.approx(o["phi"][0], rel=1e-11)


def test_lockstep_every_step_small_sheath_f64(gpu_lib):
    """Every step of the 64-cell sheath (1000 steps at dt = 5/omega_pe): the
    oracle's state at step k goes into the library, both take step k+1."""
    cfg = workloads.small_sheath(sort_every=1)
    run = oracle.Run(cfg)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=1)
    nsteps = workloads.SMALL_SHEATH_STEPS
    worst = 0.0
    for k in range(nsteps):
        if k % 100 == 0:
            print_case(f"lockstep f64 step {k}")
        push_oracle_to_gpu(sim, 0, run, quantize=False)
        sim.step(1)
        run.step(1)
        g, o = sim.grid(0), run.grid()
        for s in range(2):
            err = rel_inf(g["Q"][s], o["Q"][s])
            worst = max(worst, err)
            assert err <= 1e-12, (k, s, err)
        if k % 50 == 0 or k == nsteps - 1:
            _compare_step(sim, run)
            st = sim.status(0)
            assert st["absorbed_total"] is not None
    print_case(f"lockstep worst rel charge error {worst:.3e}")
    # the wall-potential windows and the steady step, fed by every step
    st, od = sim.status(0), run.steady()
    print_case(f"steady detector: gpu {st['steady_step']} oracle {od['steady_step']} windows {od['windows']}")
    assert st["windows"] == od["windows"] == nsteps // (cfg["nx"] // 4)
    for g, o in zip(st["window_mean"], od["window_mean"]):
        assert g == pytest.approx(o, rel=1e-10, abs=1e-12)
    assert st["steady_step"] == od["steady_step"]


def test_unlimited_speed_reduces_to_pic_f64(gpu_lib):
    cfg = workloads.sheath(nx=64, ppc=50, u_over_vti=math.inf, sort_every=1, seed=3)
    assert math.isinf(cfg["u"])
    run = oracle.Run(cfg)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=1)
    for k in range(40):
        push_oracle_to_gpu(sim, 0, run, quantize=False)
        sim.step(1)
        run.step(1)
        _compare_step(sim, run)


def test_smooth_beta_lockstep_f64(gpu_lib):
    cfg = workloads.small_sheath(sort_every=1, beta_kind="smooth", seed=4)
    run = oracle.Run(cfg)
    run.step(30)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=1)
    for k in range(10):
        push_oracle_to_gpu(sim, 0, run, quantize=False)
        sim.step(1)
        run.step(1)
        _compare_step(sim, run)


@pytest.mark.parametrize("u_over_vti,chunk", [(2.0, 0), (10.0, 0), (math.inf, 0), (2.0, 64), (2.0, 128),
                                              (2.0, 256), (2.0, 1024)])
def test_one_step_f32_developed_sheath(gpu_lib, u_over_vti, chunk):
    """FP32 particles: charge per species within 1e-5 after one step from a
    developed oracle state (256 cells, 200 per cell per species), with the
    default push chunk (512 particles per wavefront) and at u = 2 v_ti with
    every other chunk the autotuner may pick (1 to 16 particles per lane)."""
    cfg = workloads.sheath(nx=256, ppc=200, u_over_vti=u_over_vti, te_over_ti=20.0, sort_every=1,
                           seed=5)
    run = oracle.Run(cfg)
    run.step(60 if math.isfinite(u_over_vti) else 200)
    sim = gpu_lib.Sim(cfg, precision="f32", sort_every=1, chunk=chunk)
    print_case(f"f32 one step u/vti={u_over_vti} chunk={chunk}")
    push_oracle_to_gpu(sim, 0, run, quantize=True)
    g0, o0 = sim.grid(0), run.grid()
    for s in range(2):
        assert rel_inf(g0["Q"][s], o0["Q"][s]) <= 1e-6
    sim.step(1)
    run.step(1)
    g, o = sim.grid(0), run.grid()
    for s in range(2):
        err = rel_inf(g["Q"][s], o["Q"][s])
        assert err <= 1e-5, (s, err)
    fb = sim.status(0)["fixed_bits"]
    for s in range(2):
        xg, vxg, _ = sim.export_particles(0, s)
        xo, vxo, _ = oracle_state(run, s)
        n = min(len(xg), len(xo))
        live = (xg[:n] >= 0) & (xo[:n] >= 0)
        # positions within the fixed-point step plus float rounding of the displacement
        assert np.abs(xg[:n][live] - xo[:n][live]).max() <= 1e-5
        assert np.abs(vxg[:n][live] - vxo[:n][live]).max() <= 1e-5 * np.abs(vxo[:n][live]).max()
        assert abs(len(xg) - len(xo)) <= 2
        assert fb >= 19


@pytest.mark.parametrize("u_over_vti,other_order", [(2.0, False), (2.0, True), (5.0, False), (10.0, False),
                                                   (math.inf, False)])
def test_one_step_f32_production_size(gpu_lib, u_over_vti, other_order):
    """2048 cells, 1000 per cell per species (4,096,000 particles), every
    speed limit of the production sweep u in {2, 5, 10, inf} v_ti (inf: the
    PIC step dx/(5 v_te)), in the benchmark's launch configuration for that
    limit (the autotuner's cached push chunk and workgroup; at u = 2 v_ti
    also with the other push order)."""
    cfg = workloads.production_sheath(u_over_vti=u_over_vti, sort_every=16)
    p = bench_launch(cfg)
    order = 1 - p["push_order"] if other_order else p["push_order"]
    print_case(f"f32 production size, u/vti={u_over_vti}, launch {p}, push order {order}: oracle load")
    run = oracle.Run(dict(cfg, sort_every=1))
    sim = gpu_lib.Sim(cfg, precision="f32", sort_every=16, chunk=p["chunk"], block=p["block"], push_order=order)
    push_oracle_to_gpu(sim, 0, run, quantize=True)
    for k in range(2):
        print_case(f"f32 production size step {k}")
        sim.step(1)
        run.step(1)
        g, o = sim.grid(0), run.grid()
        for s in range(2):
            err = rel_inf(g["Q"][s], o["Q"][s])
            assert err <= 1e-5, (k, s, err)
        if k == 0:
            push_oracle_to_gpu(sim, 0, run, quantize=True)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("bucket", [1, 4, 5, 0])
@pytest.mark.parametrize("sort_tile", [0, 512, 2048])
def test_sort_permutation_bit_exact(gpu_lib, prec, bucket, sort_tile):
    """Stable cell sort with compaction, bit-exact against the oracle's.  The
    9600 slots per species are one sort tile by default (16384 slots) and 19
    or 5 tiles at 512 or 2048 slots, so the scan of per-tile key counts across
    tiles is exercised.  Buckets 1, 4, 5 and none give 64, 16, 13 and 1 keys
    (an odd count leaves the upper half of the scatter's last packed word
    unused)."""
    cfg = workloads.small_sheath(sort_every=0, sort_bucket=bucket if bucket else 0, seed=6)
    run = oracle.Run(cfg)
    run.step(40)  # dead slots and appended injections in place
    print_case(f"sort {prec} bucket={bucket} sort_tile={sort_tile}")
    sim = gpu_lib.Sim(cfg, precision=prec, sort_every=0, sort_bucket=bucket, sort_tile=sort_tile, record_perm=True)
    push_oracle_to_gpu(sim, 0, run, quantize=(prec == "f32"))
    before = [oracle_state(run, s) for s in range(2)]
    assert any((b[0] < 0).any() for b in before)
    sim.sort_now()
    perms = run.sort()
    for s in range(2):
        pg = sim.perm(0, s)
        assert np.array_equal(pg, perms[s]), s
        xg, vxg, vpg = sim.export_particles(0, s)
        xo, vxo, vpo = oracle_state(run, s)
        assert np.array_equal(xg, xo)
        assert np.array_equal(vxg, vxo)


def test_ten_times_ppc_sampled_step(gpu_lib):
    """The 10x-ppc production sheath (10,000 per cell per species, 40,960,000
    particles) in the benchmark's launch configuration for it (the
    autotuner's cached launch: 16 particles per lane): after 40 steps, one
    step recomputed for 300 sampled particles per species by the oracle's
    exact velocity map from the GPU's own node field (Eq. A2a-b), and the
    charge identity Q = q w sum beta over the live particles (Eq. A2c)."""
    cfg = workloads.production_sheath(u_over_vti=2.0, ppc=10000)
    p = bench_launch(cfg)
    print_case(f"10x production size: load and 40 steps, launch {p}")
    sim = gpu_lib.Sim(cfg, precision="f32", sort_every=p["sort_every"], sort_bucket=p["sort_bucket"],
                      chunk=p["chunk"], block=p["block"], push_order=p["push_order"], sort_tile=p["sort_tile"])
    sim.step(40)  # no sort falls in step 41 (sorts end every 64th step): slots keep their particles
    assert sim.status(0)["nslots"][0] > 20_000_000
    g0 = sim.grid(0)
    before = [sim.export_particles(0, s) for s in range(2)]
    print_case("10x production size: one step")
    sim.step(1)
    g1 = sim.grid(0)
    nx, u, dt, dtdx = cfg["nx"], cfg["u"], cfg["dt"], cfg["dt"] / cfg["dx"]
    rng = np.random.default_rng(5)
    for s in range(2):
        X0, VX0, VP0 = before[s]
        X, VX, VP = sim.export_particles(0, s)
        qm = cfg["species"][s]["charge"] / cfg["species"][s]["mass"]
        vs = np.abs(VX0).max()
        checked = 0
        for d in rng.integers(0, len(X0), 300):
            if X0[d] < 0:
                continue
            c = int(X0[d])
            f = X0[d] - c
            e = g0["E"][c] * (1 - f) + g0["E"][c + 1] * f
            v1 = oracle.kick_exact("step", u, dt, [VX0[d], math.sqrt(VP0[d]), 0.0], [qm * e, 0.0, 0.0])
            sp = math.sqrt(v1 @ v1)
            b = 1.0 if sp <= u else u / sp
            xn = X0[d] + b * v1[0] * dtdx
            if xn < 0:  # symmetry plane: specular
                xn, v1[0] = -xn, -v1[0]
            if abs(xn - nx) < 1e-4:  # within rounding of the wall: either side is right
                continue
            if xn >= nx:
                assert X[d] < 0, (s, d)
                continue
            assert abs(X[d] - xn) <= 1e-5, (s, d, X[d], xn)
            assert abs(VX[d] - v1[0]) <= 1e-5 * vs, (s, d, VX[d], v1[0])
            assert VP[d] == VP0[d]  # v_perp^2 is invariant in 1D
            checked += 1
        assert checked >= 250, checked
        live = X >= 0
        s2 = VX[live] ** 2 + VP[live]
        beta = np.where(s2 <= u * u, 1.0, u / np.sqrt(np.maximum(s2, 1e-300)))
        want = cfg["species"][s]["charge"] * sim.status(0)["weight"][s] * beta.sum()
        assert g1["Q"][s].sum() == pytest.approx(want, rel=1e-9), s
    assert sim.status(0)["error_flags"] == 0
    sim.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_sort_without_permutation_record(gpu_lib, prec):
    """By default a sort stores no permutation.  From the same imported state
    (live slots over five 2048-slot sort tiles) the sorted particles are bit
    for bit the oracle's stable sort, as in a context that records the
    permutation; exporting it is refused."""
    cfg = workloads.small_sheath(sort_every=0, sort_bucket=1, seed=6)
    run = oracle.Run(cfg)
    run.step(40)  # dead slots and appended injections in place
    print_case(f"sort without permutation record, {prec}")
    sims = [gpu_lib.Sim(cfg, precision=prec, sort_every=0, sort_bucket=1, sort_tile=2048, record_perm=r)
            for r in (False, True)]
    for sim in sims:
        push_oracle_to_gpu(sim, 0, run, quantize=(prec == "f32"))
        sim.sort_now()
    run.sort()
    for s in range(2):
        xo, vxo, _ = oracle_state(run, s)
        assert len(xo) > 2048
        g0, g1 = sims[0].export_particles(0, s), sims[1].export_particles(0, s)
        assert np.array_equal(g0[0], xo) and np.array_equal(g0[1], vxo), s
        for u, v in zip(g0, g1):
            assert np.array_equal(u, v), s
    with pytest.raises(gpu_lib.SlpicError):
        sims[0].perm(0, 0)
    n = ctypes.c_int64(1 << 16)
    buf = np.zeros(1 << 16, dtype=np.int32)
    rc = gpu_lib.lib().slpic_export_perm(sims[0]._ctx, 0, 0, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                         ctypes.byref(n))
    assert rc == -1
    assert len(sims[1].perm(0, 0)) == sims[1].status(0)["nslots"][0]
    for sim in sims:
        sim.close()


@pytest.mark.parametrize("bucket,sort_tile", [(None, None), (4, 16384), (1, 16384)])
def test_sort_permutation_production_size(gpu_lib, bucket, sort_tile):
    """The production sheath (4,096,000 particles, 3,072,000 slots per species)
    sorted after 24 unsorted steps, in the benchmark's launch configuration
    (the autotuner's cached bucket and sort tile: 1500 tiles of 2048 slots
    per species), and with 188 tiles of 16384 slots at buckets 4 and 1:
    permutation and sorted particles bit-exact against the oracle's stable
    sort of the GPU's own positions."""
    p = bench_launch(workloads.production_sheath(u_over_vti=2.0))
    bucket = p["sort_bucket"] if bucket is None else bucket
    sort_tile = p["sort_tile"] if sort_tile is None else sort_tile
    cfg = workloads.production_sheath(u_over_vti=2.0, sort_every=0, sort_bucket=bucket)
    print_case(f"production-size sort, bucket {bucket}, sort tile {sort_tile}: 24 steps")
    sim = gpu_lib.Sim(cfg, precision="f32", sort_every=0, sort_bucket=bucket, chunk=p["chunk"], block=p["block"],
                      push_order=p["push_order"], sort_tile=sort_tile, record_perm=True)
    sim.step(24)
    run = oracle.Run(cfg, load=False)
    before = []
    for s in range(2):
        x, vx, vp2 = sim.export_particles(0, s)
        assert (x < 0).any()  # absorbed slots to drop
        set_oracle_particles(run, s, x, vx, vp2)
        before.append((x, vx, vp2))
    print_case(f"production-size sort, bucket {bucket}, sort tile {sort_tile}: sort")
    sim.sort_now()
    perms = run.sort()
    for s in range(2):
        pg = sim.perm(0, s)
        assert len(pg) > 2 * sort_tile
        assert np.array_equal(pg, perms[s]), s
        xg, vxg, vpg = sim.export_particles(0, s)
        x, vx, vp2 = before[s]
        assert np.array_equal(xg, x[perms[s]])
        assert np.array_equal(vxg, vx[perms[s]])
        assert np.array_equal(vpg, vp2[perms[s]])
    sim.close()


def test_moments_match_oracle_f64(gpu_lib):
    cfg = workloads.small_sheath(sort_every=0, seed=7)
    run = oracle.Run(cfg)
    run.step(50)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=0)
    push_oracle_to_gpu(sim, 0, run, quantize=False)
    mg = sim.moments(0).cpu().numpy()
    mo = run.moments()
    for row in range(7):
        assert rel_inf(mg[row], mo[row]) <= 1e-11, row


def test_moment_window_matches_oracle_mean_f64(gpu_lib):
    """Five moment samples at oracle states three steps apart: the device
    window mean equals the mean of the oracle's moments; reset empties it."""
    cfg = workloads.small_sheath(sort_every=0, seed=11)
    run = oracle.Run(cfg)
    run.step(30)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=0)
    acc = None
    for _ in range(5):
        push_oracle_to_gpu(sim, 0, run, quantize=False)
        sim.moments_sample(0)
        mo = run.moments()
        acc = mo if acc is None else acc + mo
        run.step(3)
    assert sim.status(0)["moment_samples"] == 5
    mg = sim.moments_window(0, reset=True).cpu().numpy()
    for row in range(7):
        assert rel_inf(mg[row], acc[row] / 5) <= 1e-11, row
    assert sim.status(0)["moment_samples"] == 0
    assert not sim.moments_window(0).abs().max().item()


@pytest.mark.parametrize("push_order", [0, 1])
def test_batched_runs_match_their_oracles(gpu_lib, push_order):
    """Ragged runs in one context (different cells, ppc, ion mass, speed
    limit) each match their own oracle after one step (either push order)."""
    cfgs = workloads.batched_sweep(nruns=3, seed=9, cells_range=(64, 200), ppc_range=(20, 60),
                                   sort_every=1)
    runs = []
    for c in cfgs:
        r = oracle.Run(c)
        r.step(10)
        runs.append(r)
    sim = gpu_lib.Sim(cfgs, precision="f64", sort_every=1, chunk=64, push_order=push_order)
    for r, run in enumerate(runs):
        push_oracle_to_gpu(sim, r, run, quantize=False)
    sim.step(1)
    for r, run in enumerate(runs):
        run.step(1)
        _compare_step(sim, run, r=r)
    # one moment sample of every run at once
    sim.moments_sample(-1)
    for r, run in enumerate(runs):
        mg = sim.moments_window(r).cpu().numpy()
        mo = run.moments()
        for row in range(7):
            assert rel_inf(mg[row], mo[row]) <= 1e-11, (r, row)


@pytest.mark.parametrize("cfg_name", ["sheath", "plates"])
def test_graph_replay_matches_direct_launches(gpu_lib, cfg_name):
    """Blocks of 8 steps captured once and replayed as a HIP graph (on a side
    stream: the library captures only on a non-default stream) against the
    same steps launched directly, checked after every replay with host
    reads and synchronisations between the replays."""
    import torch
    cfg = (workloads.small_sheath(seed=8) if cfg_name == "sheath"
           else workloads.plates_sheath(0.0158, ppc=200, seed=8))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        a = gpu_lib.Sim(cfg, precision="f64", sort_every=4, graph_steps=8)
        b = gpu_lib.Sim(cfg, precision="f64", sort_every=4, graph_steps=0)
        for k in range(4):
            print_case(f"graph replay {cfg_name} block {k}")
            a.step(8)
            b.step(8)
            ga, gb = a.grid(0), b.grid(0)
            for s in range(2):
                if np.abs(gb["Q"][s]).max() > 0:
                    assert rel_inf(ga["Q"][s], gb["Q"][s]) <= 1e-9, (k, s)
            sa, sb = a.status(0), b.status(0)
            assert sa["nslots"] == sb["nslots"] and sa["injected_total"] == sb["injected_total"], k
        assert a.status(0)["step"] == b.status(0)["step"] == 32
        a.close()
        b.close()


def test_in_step_sampling_matches_host_sampling(gpu_lib):
    """Moments sampled inside the step sequence (graph blocks of 8 steps
    replayed on a side stream, a sample every 2nd step) against the same
    samples taken from the host after direct-launched steps."""
    import torch
    cfg = workloads.plates_sheath(0.0158, ppc=200, seed=9)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        a = gpu_lib.Sim(cfg, precision="f64", sort_every=4, graph_steps=8)
        b = gpu_lib.Sim(cfg, precision="f64", sort_every=4, graph_steps=0)
        with pytest.raises(gpu_lib.SlpicError):
            a.set_sampling(3)  # must divide the graph block
        a.step(5)  # the graph blocks start once the step count is aligned again
        b.step(5)
        a.set_sampling(2)
        a.step(35)
        for k in range(6, 41):
            b.step(1)
            if k % 2 == 0:
                b.moments_sample(-1)
        print_case("in-step sampling window")
        wa, wb = a.moments_window(0).cpu().numpy(), b.moments_window(0).cpu().numpy()
        assert a.status(0)["moment_samples"] == b.status(0)["moment_samples"] == 18
        assert np.abs(wa - wb).max() <= 1e-9 * np.abs(wb).max()
        a.set_sampling(0)
        a.step(8)
        assert a.status(0)["moment_samples"] == 18
        a.close()
        b.close()


def test_profile_counts_every_launch(gpu_lib):
    """Kernel timing: one event pair per push and per source + field launch
    of every profiled step (graph replay is off while profiling), sorts every
    sort_every steps; reading clears nothing until the next enable."""
    import torch
    cfg = workloads.small_sheath(seed=12)
    with torch.cuda.stream(torch.cuda.Stream()):
        sim = gpu_lib.Sim(cfg, precision="f32", sort_every=4, graph_steps=8)
        sim.step(8)
        sim.profile(1 | 4)
        sim.step(16)
        p = sim.profile_read()
        assert p["push"]["launches"] == 16 and p["field"]["launches"] == 16
        assert p["sort"]["launches"] == 0  # bit 3 not enabled
        assert p["push"]["ms"] > 0 and p["field"]["ms"] > 0
        sim.profile(1 | 4 | 8)
        sim.step(8)
        p = sim.profile_read()
        assert p["push"]["launches"] == 8 and p["sort"]["launches"] == 2
        sim.profile(0)
        sim.step(8)
        assert sim.profile_read()["push"]["launches"] == 0
        assert sim.status(0)["step"] == 40
        sim.close()


def test_capacity_overflow_sets_sticky_flag(gpu_lib):
    cfg = workloads.small_sheath(capacity_factor=1.0, seed=10)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=0)
    sim.step(3000)
    st = sim.status(0)
    assert st["error_flags"] & gpu_lib.FLAG_CAPACITY
    assert st["nslots"][1] == st["capacity"][1]
    assert np.isfinite(st["wall_potential"])


def _live_sorted(parts):
    x, vx, vp = parts
    live = x >= 0
    m = np.stack([x[live], vx[live], vp[live]], axis=1)
    return m[np.lexsort((m[:, 2], m[:, 1], m[:, 0]))]


def test_retired_runs_freeze_at_their_steady_step(gpu_lib):
    """retire_steady: a run stops advancing once its detector has flagged it
    (its grid, particles and step count stay as at the flagged step) while the
    other runs of the context go on exactly as in a context that never
    retires."""
    cfgs = [workloads.sheath(nx=32, ppc=40, u_over_vti=3.0, dt=5.0, seed=s, run=r, steady_window=8,
                             steady_tol=0.5, sort_every=16) for r, s in enumerate((1, 2, 3))]
    sim = gpu_lib.Sim(cfgs, precision="f64", sort_every=16, retire_steady=True)
    ref = gpu_lib.Sim(cfgs, precision="f64", sort_every=16)
    flagged, snap = {}, {}
    for k in range(400):
        sim.step(1)
        ref.step(1)
        st = sim.status()
        for r in range(3):
            if r not in flagged and st[r]["steady_step"] >= 0:
                flagged[r] = st[r]["steady_step"]
                snap[r] = ref.grid(r)
        if len(flagged) == 3:
            break
    print_case(f"retire: steady steps {flagged}")
    assert len(flagged) == 3 and len(set(flagged.values())) > 1
    frozen = {r: (sim.grid(r), [sim.export_particles(r, s) for s in range(2)]) for r in range(3)}
    sim.step(40)  # crosses sorts
    st = sim.status()
    for r in range(3):
        assert st[r]["step"] == flagged[r] == st[r]["steady_step"]
        g = sim.grid(r)
        for key in ("Q", "phi", "E"):
            assert np.array_equal(g[key], frozen[r][0][key]), (r, key)
        for s in range(2):  # the same live particles (a sort may compact and reorder them)
            a = _live_sorted(sim.export_particles(r, s))
            b = _live_sorted(frozen[r][1][s])
            assert np.array_equal(a, b), (r, s)
        # the run's frozen state is the never-retired context's state at that step
        for s in range(2):
            assert rel_inf(g["Q"][s], snap[r]["Q"][s]) <= 1e-12, (r, s)
    sim.close()
    ref.close()


def test_pruned_runs_cost_nothing_and_change_nothing(gpu_lib):
    """slpic_prune_retired: retired runs are taken out of the push and sort
    work (graph replay on a side stream); the pruned runs keep their frozen
    state across sorts and buffer swaps, and the runs still active evolve
    exactly as in a context that never prunes (FP64, same launches for them)."""
    import torch
    cfgs = [workloads.sheath(nx=32, ppc=40, u_over_vti=3.0, dt=5.0, seed=s, run=r, steady_window=8,
                             steady_tol=tol, sort_every=8)
            for r, (s, tol) in enumerate(((1, 0.5), (2, 1e-9), (3, 0.5), (4, 1e-9)))]
    with torch.cuda.stream(torch.cuda.Stream()):
        sim = gpu_lib.Sim(cfgs, precision="f64", sort_every=8, graph_steps=8, retire_steady=True)
        ref = gpu_lib.Sim(cfgs, precision="f64", sort_every=8, graph_steps=8, retire_steady=True)
        pruned = 0
        for k in range(60):
            sim.step(8)
            ref.step(8)
            pruned = sim.prune_retired()
            if pruned == 2:
                break
        print_case(f"prune: {pruned} runs pruned after {8 * (k + 1)} steps")
        assert pruned == 2
        st0 = sim.status()
        frozen = {r: (sim.grid(r), [_live_sorted(sim.export_particles(r, s)) for s in range(2)])
                  for r in (0, 2)}
        sim.step(40)  # sorts and buffer swaps with the pruned runs out of the work
        ref.step(40)
        st, sr = sim.status(), ref.status()
        for r in (0, 2):
            assert st[r]["step"] == st0[r]["step"] == st[r]["steady_step"]
            g = sim.grid(r)
            for key in ("Q", "phi", "E"):
                assert np.array_equal(g[key], frozen[r][0][key]), (r, key)
            for s in range(2):
                assert np.array_equal(_live_sorted(sim.export_particles(r, s)), frozen[r][1][s]), (r, s)
        for r in (1, 3):  # still active: as in the context that never prunes
            assert st[r]["step"] == sr[r]["step"] and st[r]["nslots"] == sr[r]["nslots"]
            g, h = sim.grid(r), ref.grid(r)
            for s in range(2):
                assert rel_inf(g["Q"][s], h["Q"][s]) <= 1e-12, (r, s)
                a = _live_sorted(sim.export_particles(r, s))
                b = _live_sorted(ref.export_particles(r, s))
                assert np.allclose(a, b, rtol=1e-12, atol=1e-12), (r, s)
        sim.close()
        ref.close()


@pytest.mark.parametrize("geometry", ["sheath", "plates", "periodic"])
def test_field_solve_at_the_largest_grid(gpu_lib, geometry):
    """The deposit and the one-workgroup field solve at the largest run,
    2729 cells (3 nodes per thread; the moments workgroup's three FP64 node
    rows bound the run length), for each geometry on 40 000 random particles
    against the oracle (FP64)."""
    nx = 2729
    if geometry == "plates":
        cfg = dict(workloads.plates_sheath(0.0158, ppc=10, sort_every=0), nx=nx)
    elif geometry == "periodic":
        cfg = workloads.langmuir_box(0.25, nx=nx, ppc=10, sort_every=0)
    else:
        cfg = workloads.sheath(nx=nx, ppc=10, u_over_vti=3.0, dt=5.0, sort_every=0)
    rng = np.random.default_rng(91)
    run = oracle.Run(cfg, load=False)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=0)
    for s in range(2):
        n = 20000
        x = rng.uniform(0, nx, size=n)
        x[rng.random(n) < 0.05] = -1.0  # dead slots
        vx = rng.normal(size=n) * (1.0 if s == 0 else 0.01)
        vy = rng.normal(size=n) * (1.0 if s == 0 else 0.01)
        run.set_particles(s, x, vx, vy, np.zeros(n))
        sim.import_particles(0, s, x, vx, vy * vy)
    run.refresh_fields()
    sim.refresh_fields()
    g, o = sim.grid(0), run.grid()
    print_case(f"field solve at {nx} cells, {geometry}")
    for s in range(2):
        assert rel_inf(g["Q"][s], o["Q"][s]) <= 1e-12, s
    assert rel_inf(g["phi"], o["phi"]) <= 1e-9
    assert rel_inf(g["E"], o["E"]) <= 1e-9

"""2D3V HIP path vs the FP64 oracle through the C ABI (include/slpic2d.h).

Small runs are compared element by element on the oracle's own states
(loaded and stepped by the oracle, imported into the library): grid charge
per species within 1e-12 of its infinity norm in FP64 and 1e-5 in FP32,
particles within the rounding of each representation, sort permutations and
absorbed/injected counts exactly.  The full-size run (512 x 512 cells, 64
per cell per species, FP32, the benchmark's launch configuration) is checked
on sampled particles the oracle computes one by one and on properties that
hold at any size (charge identity, the five-point residual of phi, E from
phi, sort order and stability).
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from parity_util import print_case, rel_inf

pytestmark = pytest.mark.gpu

V_ABS_TOL = 1e-11  # FP64 velocity floor of the exact-integral inversion


def _cfg(nx=16, ny=16, ppc=12, u_over_vti=3.0, kind="step", seed=21, sort_every=1, dt=None):
    c = workloads.sheath(nx=nx, ppc=ppc, u_over_vti=u_over_vti, beta_kind=kind, seed=seed, sort_every=sort_every,
                         dt=dt)
    return c, ny


def _quantize(x, y, vx, vy, vz2, nx, ny, fb):
    sc = math.ldexp(1.0, fb)
    xq = np.where(x < 0, -1.0, np.minimum(np.rint(x * sc), nx * sc - 1) / sc)
    yq = np.where(x < 0, 0.0, np.minimum(np.rint(y * sc), ny * sc - 1) / sc)
    f = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    return xq, yq, f(vx), f(vy), f(vz2)


def _state(run, s):
    x, y, vx, vy, vz = run.particles(s)
    return x, y, vx, vy, vz * vz


def _push_to_gpu(sim, run, quantize):
    """The oracle's state into the library (F32: the oracle takes the
    quantized state first, so both sides start from the same numbers)."""
    fb = sim.status()["fixed_bits"]
    for s in range(2):
        x, y, vx, vy, vz2 = _state(run, s)
        if quantize:
            x, y, vx, vy, vz2 = _quantize(x, y, vx, vy, vz2, run.nx, run.ny, fb)
            run.set_particles(s, x, y, vx, vy, np.sqrt(vz2))
        sim.import_particles(s, x, y, vx, vy, vz2)
    sim.set_counters(run.step_index, run.acc_e)
    run.refresh_fields()


def _compare(sim, run, tol_q, tol_x, tol_v, exact_counts=True):
    g, o = sim.grid(), run.grid()
    for s in range(2):
        err = rel_inf(g["Q"][s], o["Q"][s])
        assert err <= tol_q, ("Q", s, err)
    for s in range(2):
        xg, yg, vxg, vyg, _ = sim.export_particles(s)
        xo, yo, vxo, vyo, _ = _state(run, s)
        if exact_counts:
            assert len(xg) == len(xo), (s, len(xg), len(xo))
        n = min(len(xg), len(xo))
        live = (xg[:n] >= 0) & (xo[:n] >= 0)
        if exact_counts:
            assert np.array_equal(xg[:n] < 0, xo[:n] < 0), s
        dy = np.abs(yg[:n][live] - yo[:n][live])
        dy = np.minimum(dy, run.ny - dy)  # periodic
        assert np.abs(xg[:n][live] - xo[:n][live]).max() <= tol_x, s
        assert dy.max() <= tol_x, s
        vs = max(np.abs(vxo[:n][live]).max(), np.abs(vyo[:n][live]).max())
        assert np.abs(vxg[:n][live] - vxo[:n][live]).max() <= tol_v * vs + V_ABS_TOL, s
        assert np.abs(vyg[:n][live] - vyo[:n][live]).max() <= tol_v * vs + V_ABS_TOL, s


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,k", [("step", 3.0), ("smooth", 3.0), ("step", math.inf)])
def test_cold_load2d_matches_oracle(gpu_lib, prec, kind, k):
    cfg, ny = _cfg(nx=16, ny=8, ppc=30, u_over_vti=k, kind=kind, sort_every=0, dt=None if k < 1e9 else 0.1)
    print_case(f"2d load {prec} {kind} u/vti={k}")
    sim = gpu_lib.Sim2D(cfg, ny, precision=prec, sort_every=0, tile=4)
    run = oracle.Run2D(cfg, ny, tile=4)
    st = sim.status()
    for s in range(2):
        assert st["weight"][s] == pytest.approx(run.weight(s), rel=1e-12)
        g = sim.export_particles(s)
        o = _state(run, s)
        if prec == "f32":
            o = _quantize(*o, run.nx, ny, st["fixed_bits"])
        assert len(g[0]) == len(o[0]) == cfg["nx"] * ny * 30
        assert np.array_equal(g[0], o[0]) and np.array_equal(g[1], o[1])
        # rejection sampling may branch differently on a last-bit libm difference
        bad = np.zeros(len(g[0]), dtype=bool)
        for a, b in zip(g[2:], o[2:]):
            bad |= ~np.isclose(a, b, rtol=1e-12, atol=0)
        assert bad.sum() <= 3, bad.sum()
    sim.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("tile", [1, 4, 5, 7])  # 320, 20, 16 and 9 keys on 20 x 16 cells
def test_sort2d_permutation_bit_exact(gpu_lib, prec, tile):
    cfg, ny = _cfg(nx=20, ny=16, ppc=10, sort_every=0)
    print_case(f"2d sort {prec} tile={tile}")
    sim = gpu_lib.Sim2D(cfg, ny, precision=prec, sort_every=0, tile=tile, record_perm=True)
    run = oracle.Run2D(cfg, ny, tile=tile)
    run.step(3)  # some absorbed (dead) slots and appended source particles
    _push_to_gpu(sim, run, quantize=(prec == "f32"))
    sim.sort_now()
    perms = run.sort()
    for s in range(2):
        pg = sim.perm(s)
        assert np.array_equal(pg, perms[s]), s
        g = sim.export_particles(s)
        o = _state(run, s)
        assert np.array_equal(g[0], o[0]) and np.array_equal(g[1], o[1])
    st = sim.status()
    assert st["nsorted"] == st["nslots"] == [run.nslots(0), run.nslots(1)]
    sim.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_sort2d_without_permutation_record(gpu_lib, prec):
    """By default a 2D sort stores no permutation (and its workspace holds
    none).  From the same imported state (live slots over three 1024-slot
    sort tiles) the sorted particles are bit for bit the oracle's stable
    sort, as in a context that records the permutation; exporting it is
    refused."""
    cfg, ny = _cfg(nx=24, ny=16, ppc=8, sort_every=0)
    run = oracle.Run2D(cfg, ny, tile=4)
    run.step(3)  # some absorbed (dead) slots and appended source particles
    print_case(f"2d sort without permutation record, {prec}")
    sims = [gpu_lib.Sim2D(cfg, ny, precision=prec, sort_every=0, tile=4, sort_tile=1024, record_perm=r)
            for r in (False, True)]
    assert sims[0].workspace.numel() < sims[1].workspace.numel()
    for sim in sims:
        _push_to_gpu(sim, run, quantize=(prec == "f32"))
        sim.sort_now()
    run.sort()
    for s in range(2):
        o = _state(run, s)
        assert len(o[0]) > 2 * 1024
        g0, g1 = sims[0].export_particles(s), sims[1].export_particles(s)
        assert np.array_equal(g0[0], o[0]) and np.array_equal(g0[1], o[1]), s
        for u, v in zip(g0, g1):
            assert np.array_equal(u, v), s
    with pytest.raises(gpu_lib.SlpicError):
        sims[0].perm(0)
    assert len(sims[1].perm(0)) == sims[1].status()["nslots"][0]
    for sim in sims:
        sim.close()


def test_sort2d_tile_size_invariance_at_full_size(gpu_lib):
    """The 512 x 512 sheath (33.5 M particles) sorted once from its cold load
    with 32768-slot tiles (1536 tiles) and with 2048-slot tiles (24576): the
    stable order by key does not depend on how the slots are split, so the
    two permutations of every slot agree bit for bit."""
    cfg = workloads.sheath2d()
    perms = []
    for st in (32768, 2048):
        print_case(f"2d full-size sort, sort_tile={st}")
        sim = gpu_lib.Sim2D(cfg, cfg["ny"], precision="f32", sort_every=0, tile=cfg["tile"], sort_tile=st,
                            record_perm=True)
        sim.sort_now()
        perms.append([sim.perm(s) for s in range(2)])
        sim.close()
    for s in range(2):
        assert len(perms[0][s]) == len(perms[1][s]) > 0
        assert np.array_equal(perms[0][s], perms[1][s]), s


@pytest.mark.parametrize("nx,ny", [(16, 8), (33, 64), (100, 128)])
def test_poisson2d_matches_oracle(gpu_lib, nx, ny):
    cfg, _ = _cfg(nx=nx, ny=ny, ppc=1)
    sim = gpu_lib.Sim2D(cfg, ny, precision="f64", sort_every=0)
    rng = np.random.default_rng(nx + ny)
    Q = rng.normal(size=(2, nx + 1, ny)) * cfg["dx"] ** 2
    print_case(f"2d poisson {nx}x{ny}")
    sim.solve_charge(Q)
    g = sim.grid()
    phi, Ex, Ey = oracle.poisson2d(nx, ny, cfg["dx"], Q[0] + Q[1])
    assert rel_inf(g["phi"], phi) <= 1e-12
    assert rel_inf(g["Ex"], Ex) <= 1e-12
    assert rel_inf(g["Ey"], Ey) <= 1e-12
    assert sim.status()["wall_potential"] == pytest.approx(phi[0].mean(), rel=1e-12, abs=1e-14)
    sim.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("sorted_", [True, False])
def test_deposit2d_matches_oracle(gpu_lib, prec, sorted_):
    """rho from the stored particles: through the tile windows (sorted) and
    through the grid (unsorted tail)."""
    cfg, ny = _cfg(nx=24, ny=16, ppc=16, sort_every=0)
    run = oracle.Run2D(cfg, ny, tile=4)
    run.step(5)
    sim = gpu_lib.Sim2D(cfg, ny, precision=prec, sort_every=0, tile=4, margin=2)
    print_case(f"2d deposit {prec} sorted={sorted_}")
    _push_to_gpu(sim, run, quantize=(prec == "f32"))
    if sorted_:
        sim.sort_now()
        run.sort()
        run.refresh_fields()
    sim.refresh_fields()
    g, o = sim.grid(), run.grid()
    tol = 1e-12 if prec == "f64" else 1e-6
    for s in range(2):
        assert rel_inf(g["Q"][s], o["Q"][s]) <= tol, s
    assert rel_inf(g["phi"], o["phi"]) <= (1e-11 if prec == "f64" else 1e-5)
    sim.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_deposit_and_step2d_at_full_tile_occupancy(gpu_lib, prec):
    """The 2D sheath's occupancy (64 per cell per species, 8 x 8-cell tiles:
    4096 particles per tile and species, 16 passes of the 256-thread tile
    loop) on a 64 x 64-cell grid: grid charge element by element after the
    sort (tile windows) and after one step, against the oracle."""
    cfg = workloads.sheath2d(nx=64, ny=64, ppc=64, tile=8, sort_every=8, seed=41)
    ny = cfg["ny"]
    print_case(f"2d full tile occupancy {prec}: oracle load + 3 steps")
    run = oracle.Run2D(cfg, ny, tile=8)
    run.step(3)
    run = _with_sort_every(run, cfg, ny, 1)
    sim = gpu_lib.Sim2D(cfg, ny, precision=prec, sort_every=1, tile=8)
    _push_to_gpu(sim, run, quantize=(prec == "f32"))
    sim.sort_now()
    run.sort()
    run.refresh_fields()
    sim.refresh_fields()
    x0 = run.particles(0)[0]
    per_col = np.bincount(x0[x0 >= 0].astype(np.int64) // 8, minlength=8)
    assert per_col.max() >= 4096 * 8 * 0.9  # a column of 8 tiles holds ~8 x 4096
    tol = 1e-12 if prec == "f64" else 1e-5
    g, o = sim.grid(), run.grid()
    for s in range(2):
        assert rel_inf(g["Q"][s], o["Q"][s]) <= tol, ("sorted deposit", s)
    print_case(f"2d full tile occupancy {prec}: one step")
    sim.step(1)
    run.step(1)
    g, o = sim.grid(), run.grid()
    for s in range(2):
        assert rel_inf(g["Q"][s], o["Q"][s]) <= tol, ("step", s, rel_inf(g["Q"][s], o["Q"][s]))
    if prec == "f64":
        st = sim.status()
        assert st["nslots"] == [run.nslots(0), run.nslots(1)]
        _compare(sim, run, tol_q=1e-12, tol_x=1e-11, tol_v=1e-11)
    sim.close()


def _with_sort_every(run, cfg, ny, sort_every):
    """A copy of an oracle run whose periodic sort runs every sort_every steps."""
    r2 = oracle.Run2D(dict(cfg, sort_every=sort_every), ny, tile=run.tile, load=False)
    for s in range(2):
        r2.set_particles(s, *run.particles(s))
    r2.set_counters(run.step_index, run.acc_e)
    r2.refresh_fields()
    return r2


STEP_CASES = [("step", 3.0, 1), ("smooth", 3.0, 1), ("step", math.inf, 1), ("step", 2.0, 0)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,k,sort_every", STEP_CASES)
def test_one_step2d_matches_oracle(gpu_lib, prec, kind, k, sort_every):
    """sort_every = 1: the push runs on sorted tiles (LDS windows); FP64 also
    sorts after the step (a float position within rounding of a tile edge
    could legitimately sort differently, so FP32 compares unsorted)."""
    cfg, ny = _cfg(nx=24, ny=16, ppc=16, u_over_vti=k, kind=kind, sort_every=sort_every,
                   dt=None if k < 1e9 else 0.1, seed=23)
    run = oracle.Run2D(cfg, ny, tile=4)
    run.step(20 if k < 1e9 else 50)
    after = sort_every if prec == "f64" else 0
    run = _with_sort_every(run, cfg, ny, after)
    sim = gpu_lib.Sim2D(cfg, ny, precision=prec, sort_every=after, tile=4, margin=1)
    print_case(f"2d step {prec} {kind} u/vti={k} sort_every={sort_every}")
    _push_to_gpu(sim, run, quantize=(prec == "f32"))
    if sort_every:
        sim.sort_now()
        run.sort()
        run.refresh_fields()
    sim.refresh_fields()
    sim.step(1)
    run.step(1)
    if prec == "f64":
        _compare(sim, run, tol_q=1e-12, tol_x=1e-11, tol_v=1e-11)
    else:
        _compare(sim, run, tol_q=1e-5, tol_x=1e-5, tol_v=1e-5, exact_counts=False)
    st = sim.status()
    assert st["error_flags"] == 0
    if prec == "f64":
        assert st["nslots"] == [run.nslots(0), run.nslots(1)]
        assert st["wall_potential"] == pytest.approx(run.wall_potential(), rel=1e-10)
    sim.close()


def test_steps2d_with_source_and_sorts_f64(gpu_lib):
    """Several steps with wall losses, source injection and periodic sorts:
    counts exact, charge within 1e-11 of its norm."""
    cfg, ny = _cfg(nx=16, ny=8, ppc=20, u_over_vti=3.0, sort_every=2, seed=31)
    run = oracle.Run2D(cfg, ny, tile=4)
    run.step(10)
    sim = gpu_lib.Sim2D(cfg, ny, precision="f64", sort_every=2, tile=4, margin=2)
    _push_to_gpu(sim, run, quantize=False)
    sim.sort_now()
    run.sort()
    run.refresh_fields()
    sim.refresh_fields()
    inj0 = sim.status()["injected_total"]
    for k in range(6):
        print_case(f"2d steps with source: step {k}")
        sim.step(1)
        run.step(1)
        g, o = sim.grid(), run.grid()
        for s in range(2):
            assert rel_inf(g["Q"][s], o["Q"][s]) <= 1e-11, (k, s)
        st = sim.status()
        assert st["nslots"] == [run.nslots(0), run.nslots(1)], k
        assert st["acc_e"] == pytest.approx(run.acc_e, abs=1e-12)
    st = sim.status()
    assert sum(st["injected_total"]) > sum(inj0)  # the source took part
    sim.close()


# ------------------------------------------------------------------ full size
def _five_point_residual(phi, Q, dx):
    """rho - (-lap phi) over rows 0..nx-1 (dV = dx dy, half at x = 0)."""
    rho = Q / (dx * dx)
    rho[0] *= 2.0
    left = np.vstack([phi[1:2], phi[:-2]])
    d2x = (phi[1:] - 2 * phi[:-1] + left) / dx ** 2
    d2y = (np.roll(phi, -1, axis=1) - 2 * phi + np.roll(phi, 1, axis=1))[:-1] / dx ** 2
    return rho[:-1] + d2x + d2y, rho


def test_full_size_2d_f32_sampled_and_properties(gpu_lib):
    cfg = workloads.sheath2d()
    nx, ny = cfg["nx"], cfg["ny"]
    print_case("2d full size: init (512 x 512 cells, 64 ppc per species)")
    # the benchmark's launch configuration, with the sort permutation recorded
    sim = gpu_lib.Sim2D(cfg, ny, precision="f32", sort_every=cfg["sort_every"], tile=cfg["tile"], record_perm=True)
    st = sim.status()
    fb = st["fixed_bits"]
    assert st["nslots"] == [nx * ny * 64] * 2 and st["nsorted"] == st["nslots"]
    rng = np.random.default_rng(0)
    for s in range(2):
        # load: sampled slots against the oracle's loader, through the sort permutation
        perm = sim.perm(s)
        x, y, vx, vy, vz2 = sim.export_particles(s)
        keys = (np.floor(x) // cfg["tile"]) * math.ceil(ny / cfg["tile"]) + np.floor(y) // cfg["tile"]
        assert np.all(np.diff(keys) >= 0)
        same = np.diff(keys) == 0
        assert np.all(np.diff(perm)[same] > 0)  # stable
        assert np.array_equal(np.sort(perm), np.arange(len(perm)))
        for d in rng.integers(0, len(perm), 300):
            o = oracle.load_particle2d(cfg, ny, s, int(perm[d]))
            q = _quantize(np.array([o[0]]), np.array([o[1]]), np.array([o[2]]), np.array([o[3]]),
                          np.array([o[4] ** 2]), nx, ny, fb)
            assert x[d] == q[0][0] and y[d] == q[1][0], (s, d)
            assert vx[d] == pytest.approx(q[2][0], rel=1e-6, abs=1e-12)
            assert vz2[d] == pytest.approx(q[4][0], rel=1e-6, abs=1e-18)
    print_case("2d full size: one step")
    before = [sim.export_particles(s) for s in range(2)]
    g0 = sim.grid()
    sim.step(1)
    g1 = sim.grid()
    u, dt, dtdx = cfg["u"], cfg["dt"], cfg["dt"] / cfg["dx"]
    for s in range(2):
        X0, Y0, VX0, VY0, VZ0 = before[s]
        X, Y, VX, VY, VZ = sim.export_particles(s)
        qm = cfg["species"][s]["charge"] / cfg["species"][s]["mass"]
        vs = np.abs(VX0).max()
        for d in rng.integers(0, len(X0), 300):
            if X0[d] < 0:
                continue
            cx, cy = int(X0[d]), int(Y0[d])
            fx, fy = X0[d] - cx, Y0[d] - cy
            c1 = (cy + 1) % ny
            wts = [((cx, cy), (1 - fx) * (1 - fy)), ((cx + 1, cy), fx * (1 - fy)),
                   ((cx, c1), (1 - fx) * fy), ((cx + 1, c1), fx * fy)]
            ex = sum(g0["Ex"][n] * w for n, w in wts)
            ey = sum(g0["Ey"][n] * w for n, w in wts)
            v1 = oracle.kick_exact("step", u, dt, [VX0[d], VY0[d], math.sqrt(VZ0[d])], [qm * ex, qm * ey, 0.0])
            sp = math.sqrt(v1 @ v1)
            b = 1.0 if sp <= u else u / sp
            xn = X0[d] + b * v1[0] * dtdx
            yn = (Y0[d] + b * v1[1] * dtdx) % ny
            if xn < 0:
                xn, v1[0] = -xn, -v1[0]
            if xn >= nx:
                assert X[d] < 0
                continue
            assert abs(X[d] - xn) <= 1e-5 and min(abs(Y[d] - yn), ny - abs(Y[d] - yn)) <= 1e-5, (s, d)
            assert abs(VX[d] - v1[0]) <= 1e-5 * vs and abs(VY[d] - v1[1]) <= 1e-5 * vs, (s, d)
        # charge identity: the deposited charge is q w sum beta over live particles
        live = X >= 0
        s2 = VX[live] ** 2 + VY[live] ** 2 + VZ[live]
        beta = np.where(s2 <= u * u, 1.0, u / np.sqrt(np.maximum(s2, 1e-300)))
        want = cfg["species"][s]["charge"] * sim.status()["weight"][s] * beta.sum()
        assert g1["Q"][s].sum() == pytest.approx(want, rel=1e-9)
    # the step's charge element by element: the oracle's deposit of the GPU's own particles
    print_case("2d full size: oracle deposit of the GPU's particles")
    ref = oracle.Run2D(cfg, ny, tile=cfg["tile"], load=False)
    for s in range(2):
        X, Y, VX, VY, VZ2 = sim.export_particles(s)
        ref.set_particles(s, X, Y, VX, VY, np.sqrt(VZ2))
        del X, Y, VX, VY, VZ2
    ref.refresh_fields()
    o1 = ref.grid()
    for s in range(2):
        assert rel_inf(g1["Q"][s], o1["Q"][s]) <= 1e-5, ("full-size charge", s, rel_inf(g1["Q"][s], o1["Q"][s]))
    del ref
    # Poisson and E at full size
    res, rho = _five_point_residual(g1["phi"], g1["Q"][0] + g1["Q"][1], cfg["dx"])
    assert np.abs(res).max() <= 1e-9 * np.abs(rho).max()
    assert np.abs(g1["phi"][-1]).max() == 0.0
    ey = -(np.roll(g1["phi"], -1, axis=1) - np.roll(g1["phi"], 1, axis=1)) / (2 * cfg["dx"])
    assert np.abs(g1["Ey"] - ey).max() <= 1e-12 * max(1.0, np.abs(ey).max())
    assert sim.status()["error_flags"] == 0
    sim.close()

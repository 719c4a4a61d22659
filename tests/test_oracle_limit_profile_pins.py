"""Pins of the oracle's speed limit varying with position, v0(x) (Sec. II
lets beta depend on position): node values interpolated linearly, the limit
at x^n for the velocity map and the move, at the particle's position for the
charge and the moments.

What fixes the answers, independently of the oracle's own code:
  - a uniform profile is the uniform limit (to rounding), and a profile above
    every speed is standard PIC, bit for bit;
  - Sec. II: dx/dt = beta v, dv/dt = beta a keep the phase paths of the
    unlimited motion, whatever beta(x, v) is.  In a uniform field the energy
    v^2/2 - a x is constant along them, and the discrete orbits converge at
    first order (the limit is frozen at x^n over a step) to a DOP853
    integration of the limited equations with the profile interpolated by
    numpy;
  - any stationary solution of the Vlasov equation stays stationary (beta
    multiplies the whole Vlasov operator): a uniform Maxwellian in a periodic
    box keeps a uniform beta-weighted density while its g-particles stay
    piled up where the limit is low (g = f/beta);
  - the charge of Eq. (A2c) written out in numpy with beta at each particle's
    new position;
  - the cold load: unit beta-weighted density in every cell, and the
    g-particle count of a cell in proportion to Z at the cell's limit.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import workloads


def _beta(kind, u, s):
    if kind == "step":
        return np.minimum(1.0, u / s)
    return 1.0 / np.sqrt(1.0 + (s / u) ** 2)


def _cosine_profile(nx, u0, depth=0.6):
    return u0 * (1.0 + depth * np.cos(2.0 * np.pi * np.arange(nx + 1) / nx))


def test_uniform_profile_is_the_uniform_limit():
    cfg = workloads.small_sheath(seed=3, ppc=50)
    nx = cfg["nx"]
    a = oracle.Run(cfg)
    b = oracle.Run(dict(cfg, limit_profile=np.full(nx + 1, cfg["u"])), load=False)
    for s in range(2):
        b.set_particles(s, *a.particles(s))
    b.set_counters(a.step_index, a.acc_e)
    b.refresh_fields()
    a.step(30)
    b.step(30)
    for s in range(2):
        pa, pb = a.particles(s), b.particles(s)
        assert len(pa[0]) == len(pb[0])
        for u, v in zip(pa, pb):
            # u (1 - f) + u f rounds to within an ulp of u
            np.testing.assert_allclose(u, v, rtol=0, atol=1e-12)
    ga, gb = a.grid(), b.grid()
    np.testing.assert_allclose(ga["Q"], gb["Q"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", ["step", "smooth"])
def test_profile_above_every_speed_is_pic(kind):
    """Step form: beta = 1 below the limit, so a profile far above every
    speed (nodes 1e6 to 2e6 v_te) steps exactly like u = inf.  Smooth form:
    beta = 1 - O(v^2/u^2), equal to 1e-11."""
    cfg = dict(workloads.small_sheath(seed=3, ppc=50), beta_kind=kind)
    nx = cfg["nx"]
    a = oracle.Run(dict(cfg, u=math.inf, dt=0.5))
    prof = 1e6 * (1.0 + np.arange(nx + 1) / nx)
    b = oracle.Run(dict(cfg, u=1e6, dt=0.5, limit_profile=prof), load=False)
    for s in range(2):
        b.set_particles(s, *a.particles(s))
        assert b.weight(s) == pytest.approx(a.weight(s), rel=1e-11)
    b.set_counters(a.step_index, a.acc_e)
    b.refresh_fields()
    a.step(20)
    b.step(20)
    for s in range(2):
        for u, v in zip(a.particles(s), b.particles(s)):
            if kind == "step":
                assert np.array_equal(u, v)
            else:
                np.testing.assert_allclose(u, v, rtol=0, atol=1e-9)


NX_ORBIT, BIAS = 32, 0.5


def _orbit_cfg(dt, kind, prof):
    # charges of 1e-9 with q/m of an electron and of a heavy ion: the test
    # particles' own field is ~1e-7 of the applied one (bias / L)
    sp = [dict(charge=-1e-9, mass=1e-9, temperature=1e-9, ppc=1),
          dict(charge=1e-9, mass=1e-7, temperature=1e-9, ppc=1)]
    return dict(nx=NX_ORBIT, dx=1.0, dt=dt, u=0.5, beta_kind=kind, species=sp, geometry="plates",
                bias=BIAS, sort_every=0, source_cells=4, seed=1, limit_profile=prof, capacity_factor=1.0)


@pytest.mark.parametrize("kind", ["step", "smooth"])
def test_orbits_converge_to_the_limited_equations(kind):
    """Electrons in the uniform field of two biased plates (E = -bias/L),
    under a rough random profile (nodes uniform in [0.2, 1] v_te): after
    T = 40 the positions and velocities approach the DOP853 solution of
    dx/dt = beta(u(x), |v|) v_x, dv/dt = beta a at first order (errors halve
    with dt), and the energy v^2/2 - a x drifts by O(dt) only."""
    rng = np.random.default_rng(7)
    prof = rng.uniform(0.2, 1.0, NX_ORBIT + 1)
    k = 12
    x0 = rng.uniform(10, 22, k)
    vx0 = rng.uniform(-0.8, 0.8, k)
    vy0 = rng.uniform(-0.5, 0.5, k)
    T = 40.0
    a = BIAS / NX_ORBIT  # q/m = -1 times E = -bias / L
    nodes = np.arange(NX_ORBIT + 1)

    def rhs(t, y):
        u = np.interp(y[0], nodes, prof)
        b = _beta(kind, u, math.hypot(y[1], y[2]))
        return [b * y[1], b * a, 0.0]

    ref = np.array([solve_ivp(rhs, (0.0, T), [x0[i], vx0[i], vy0[i]], method="DOP853", rtol=1e-12,
                              atol=1e-12).y[:, -1] for i in range(k)])
    inside = (ref[:, 0] > 1.0) & (ref[:, 0] < NX_ORBIT - 1.0)
    assert inside.sum() >= 8
    errs, drifts = [], []
    for dt in (0.5, 0.25, 0.125):
        run = oracle.Run(_orbit_cfg(dt, kind, prof))
        run.set_particles(0, x0, vx0, vy0, np.zeros(k))
        run.set_particles(1, *(np.zeros(0),) * 4)
        run.refresh_fields()
        assert run.grid()["E"][NX_ORBIT // 2] == pytest.approx(-BIAS / NX_ORBIT, rel=1e-5)
        run.step(int(round(T / dt)))
        x, vx, vy, _ = (v[:k] for v in run.particles(0))
        errs.append(max(np.abs(x - ref[:, 0])[inside].max(), np.abs(vx - ref[:, 1])[inside].max()))
        e0 = 0.5 * (vx0 ** 2 + vy0 ** 2) - a * x0
        e1 = 0.5 * (vx ** 2 + vy ** 2) - a * x
        drifts.append(np.abs(e1 - e0)[inside].max())
    for r in (errs[1] / errs[0], errs[2] / errs[1]):
        assert 0.4 <= r <= 0.6, errs
    for r in (drifts[1] / drifts[0], drifts[2] / drifts[1]):
        assert 0.35 <= r <= 0.65, drifts
    assert errs[-1] < 0.05 and drifts[-1] < 1e-3


def test_periodic_maxwellian_stays_stationary():
    """Sec. II: beta multiplies the whole Vlasov operator, so a uniform
    Maxwellian stays a steady state under any beta(x, v).  Periodic box, 64
    cells, 200 g-particles per cell at the mean limit, v0(x) = 0.5 (1 + 0.6
    cos 2 pi x / L) v_te, 800 steps (about five electron transits at the
    lowest limit): the beta-weighted electron density stays 1 within 6 % in
    eight bins, and the g-particles stay piled up where the limit is low."""
    nx, ppc = 64, 200
    cfg = workloads.langmuir_box(0.5, nx=nx, ppc=ppc, seed=5)
    prof = _cosine_profile(nx, 0.5)
    cfg["dt"] = cfg["dx"] / prof.max()
    run = oracle.Run(dict(cfg, limit_profile=prof))

    def bins():
        m = run.moments()
        x = run.particles(0)[0]
        h = np.histogram(x[x >= 0], bins=8, range=(0, nx))[0]
        return m[1][:nx].reshape(8, 8).mean(axis=1), h

    n0, h0 = bins()
    assert np.all(np.abs(n0 - 1.0) < 0.03)
    for _ in range(4):
        run.step(200)
        n, h = bins()
        assert np.all(np.abs(n - 1.0) < 0.06), n
        # counts within 5 sigma of the load's (Poisson-like fluctuations)
        assert np.all(np.abs(h - h0) < 5.0 * np.sqrt(h0)), (h, h0)
    assert h0[3] > 3 * h0[0]  # the pile-up where the limit is lowest (x = L/2)


def test_charge_takes_the_limit_at_the_new_position():
    cfg = workloads.small_sheath(seed=3, ppc=50)
    nx = cfg["nx"]
    prof = _cosine_profile(nx, cfg["u"])
    run = oracle.Run(dict(cfg, limit_profile=prof))
    run.step(5)
    g = run.grid()
    for s in range(2):
        x, vx, vy, vz = run.particles(s)
        live = x >= 0
        x, vx, vy, vz = x[live], vx[live], vy[live], vz[live]
        u = np.interp(x, np.arange(nx + 1), prof)
        b = _beta("step", u, np.sqrt(vx ** 2 + vy ** 2 + vz ** 2))
        c = np.floor(x).astype(np.int64)
        f = x - c
        q = cfg["species"][s]["charge"] * run.weight(s)
        Q = np.zeros(nx + 1)
        np.add.at(Q, c, q * b * (1.0 - f))
        np.add.at(Q, c + 1, q * b * f)
        np.testing.assert_allclose(g["Q"][s], Q, rtol=0, atol=1e-13 * np.abs(Q).max())


def test_cold_load_follows_the_profile():
    """Unit beta-weighted density in every cell (within its sampling noise),
    and g-particles per cell in proportion to Z(u_c/v_t) / Z(u/v_t), u_c the
    mean of the cell's nodes (Z = <1/beta>: the step form's closed form for
    a Maxwellian speed distribution written out with scipy)."""
    from scipy import special

    cfg = workloads.small_sheath(seed=8, ppc=200)
    nx = cfg["nx"]
    prof = _cosine_profile(nx, cfg["u"])
    run = oracle.Run(dict(cfg, limit_profile=prof))
    m = run.moments()
    for row in (1, 4):
        n = m[row][1:-1]
        assert abs(n.mean() - 1.0) < 0.03 and np.all(np.abs(n - 1.0) < 0.25)

    def Z_step(ut):  # <max(1, s/ut)> over the Maxwell speed distribution
        p_above = special.erfc(ut / math.sqrt(2)) + math.sqrt(2 / math.pi) * ut * math.exp(-ut * ut / 2)
        mean_above = 2.0 * math.sqrt(2 / math.pi) * math.exp(-ut * ut / 2) * (1 + ut * ut / 2)
        return 1.0 - p_above + mean_above / ut

    for s in range(2):
        vt = math.sqrt(cfg["species"][s]["temperature"] / cfg["species"][s]["mass"])
        uc = 0.5 * (prof[:-1] + prof[1:])
        expect = 200 * np.array([Z_step(u / vt) for u in uc]) / Z_step(cfg["u"] / vt)
        x = run.particles(s)[0]
        h = np.bincount(np.floor(x).astype(np.int64), minlength=nx)
        assert np.all(np.abs(h - expect) <= 1.0 + 1e-9), s  # floor(E) or floor(E) + 1


def test_invalid_profiles_are_refused():
    cfg = workloads.small_sheath(seed=3, ppc=10)
    nx = cfg["nx"]
    for bad in (np.zeros(nx + 1), np.full(nx + 1, np.inf), -np.ones(nx + 1)):
        with pytest.raises(ValueError):
            oracle.Run(dict(cfg, limit_profile=bad))
    with pytest.raises(ValueError):
        oracle.Run(dict(cfg, u=math.inf, limit_profile=np.ones(nx + 1)))
    with pytest.raises(ValueError):
        oracle.Run(dict(cfg, limit_profile=np.ones(nx)))  # nx + 1 nodes
    with pytest.raises(ValueError):
        oracle.Run2D(dict(cfg, limit_profile=np.ones(nx + 1)), ny=8)
    run = oracle.Run(dict(cfg, limit_profile=np.full(nx + 1, cfg["u"])))
    with pytest.raises(ValueError):
        run.set_speed_limit(2 * cfg["u"], cfg["dt"])  # a profile run keeps its profile

"""Pins of the oracle's two-plate geometry (the paper's sheath experiment,
Sec. IV): the Dirichlet solve against closed forms and a dense solve, the
flux injection's rate and velocity law against the one-sided flux of a
stationary Maxwellian, and absorption at both plates."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads


def test_plates_vacuum_and_uniform_charge_closed_forms():
    nx, dx, bias = 40, 0.3, 5.0
    L = nx * dx
    x = np.arange(nx + 1) * dx
    phi, E = oracle.poisson1d_plates(nx, dx, np.zeros(nx + 1), bias)
    assert np.abs(phi - bias * x / L).max() < 1e-13
    assert np.abs(E + bias / L).max() < 1e-12
    # uniform rho: phi = bias x/L + rho x (L - x)/2, exact for the stencil
    rho = 0.7
    phi, E = oracle.poisson1d_plates(nx, dx, np.full(nx + 1, rho * dx), bias)
    want = bias * x / L + rho * x * (L - x) / 2
    assert np.abs(phi - want).max() < 1e-12 * np.abs(want).max()
    assert np.abs(E - (-(bias / L) - rho * (L / 2 - x))).max() < 1e-11


def test_plates_solve_matches_dense_solve():
    nx, dx, bias = 25, 0.4, -2.0
    rng = np.random.default_rng(2)
    Q = rng.normal(size=nx + 1)
    phi, E = oracle.poisson1d_plates(nx, dx, Q, bias)
    n = nx - 1
    A = np.zeros((n, n))
    b = np.zeros(n)
    for k in range(n):
        j = k + 1
        A[k, k] = 2.0
        if k > 0:
            A[k, k - 1] = -1.0
        if k < n - 1:
            A[k, k + 1] = -1.0
        b[k] = Q[j] * dx  # rho_j dx^2 with rho = Q/dx
    b[-1] += bias
    sol = np.linalg.solve(A, b)
    assert phi[0] == 0.0 and phi[-1] == bias
    assert np.abs(phi[1:-1] - sol).max() < 1e-12 * np.abs(sol).max()
    assert E[3] == pytest.approx(-(phi[4] - phi[2]) / (2 * dx), rel=1e-14)


def test_wall_injection_rate_and_velocity_law():
    cfg = workloads.plates_sheath(0.0158, ppc=40)
    vt = [math.sqrt(sp["temperature"] / sp["mass"]) for sp in cfg["species"]]
    for s in range(2):
        # g-particles per step = one-sided flux v_t/sqrt(2 pi) of density 1, times dt, over the weight
        rate = oracle.wall_flux_per_step(cfg, s)
        assert rate == pytest.approx(vt[s] / math.sqrt(2 * math.pi) * cfg["dt"] / oracle.weight(cfg, s), rel=1e-14)
        pts = np.array([oracle.wall_inject_particle(cfg, s, k, 7) for k in range(4000)])
        x, vx, vy, vz = pts.T
        assert np.all(vx < 0)
        # |v_x|/v_t of the flux through a plane is Rayleigh: P(s) = 1 - exp(-s^2/2)
        assert stats.kstest(-vx / vt[s], "rayleigh").pvalue > 1e-3
        assert stats.kstest(vy / vt[s], "norm").pvalue > 1e-3
        assert stats.kstest(vz / vt[s], "norm").pvalue > 1e-3
        # inside the plate by a uniform fraction of this step's travel
        u = cfg["u"]
        sp = np.sqrt(vx ** 2 + vy ** 2 + vz ** 2)
        travel = np.where(sp <= u, 1.0, u / sp) * np.abs(vx) * cfg["dt"] / cfg["dx"]
        depth = cfg["nx"] - x
        assert np.all(depth >= 0) and np.all(depth <= np.minimum(travel, cfg["source_cells"]) + 1e-12)
        frac = depth[travel < cfg["source_cells"]] / travel[travel < cfg["source_cells"]]
        assert stats.kstest(frac, "uniform").pvalue > 1e-3


def test_plates_run_counts_and_absorption():
    cfg = workloads.plates_sheath(0.0158, ppc=40, sort_every=0)
    r = oracle.Run(cfg)
    assert [r.nslots(s) for s in range(2)] == [0, 0]  # the box starts empty
    n = 37
    r.step(n)
    for s in range(2):
        rate = oracle.wall_flux_per_step(cfg, s)
        assert r.injected_total(s) == math.floor(n * rate + 1e-9)
    # a particle leaving through x = 0 is absorbed, not reflected
    r2 = oracle.Run(cfg, load=False)
    # far above the limit u, it moves u dt = one cell per step whatever E does to v
    r2.set_particles(0, [0.1], [-10.0], [0.0], [0.0])
    r2.set_particles(1, [50.0], [0.0], [0.0], [0.0])
    r2.refresh_fields()
    before = r2.absorbed_total(0)
    r2.step(1)
    x, *_ = r2.particles(0)
    assert x[0] < 0 and r2.absorbed_total(0) == before + 1
    # the same particle moving right is kept
    r3 = oracle.Run(cfg, load=False)
    r3.set_particles(0, [0.1], [10.0], [0.0], [0.0])
    r3.set_particles(1, [50.0], [0.0], [0.0], [0.0])
    r3.refresh_fields()
    r3.step(1)
    x3, *_ = r3.particles(0)
    assert x3[0] == pytest.approx(1.1, abs=1e-12) and r3.absorbed_total(0) == 0
    # the monitored potential is phi at the mid-plane
    g = r2.grid()
    assert g["phi"][0] == 0.0 and g["phi"][-1] == pytest.approx(cfg["bias"])

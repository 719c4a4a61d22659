"""Pins of the oracle's periodic box (the uniform plasma of the
plasma-oscillation section): the periodic Poisson solve against the exact
discrete solution of a Fourier mode and against a dense pseudo-inverse, the
wrap of positions, the speed-limited plasma frequency <(beta v_x)^2>/v_t^2
against its closed form (Eq. 11b) and Monte Carlo (Eq. 11a), and the
oracle's own Langmuir oscillation against the Bohm-Gross frequency (u = inf)
and the speed-limited frequency."""
import math

import numpy as np
import pytest
from scipy.special import erf

import oracle
import workloads


@pytest.mark.parametrize("m", [1, 3, 7])
def test_periodic_mode_exact(m):
    nx, dx = 64, 0.5
    L = nx * dx
    x = np.arange(nx + 1) * dx
    k = 2 * math.pi * m / L
    Q = dx * np.cos(k * x)          # rho = cos(k x) on nodes 0..nx-1
    Q[nx] = 0.0                      # node nx is the image of node 0
    phi, E = oracle.poisson1d_periodic(nx, dx, Q)
    K2 = (2 * math.sin(k * dx / 2) / dx) ** 2   # the three-point stencil's eigenvalue
    want_phi = (np.cos(k * x) - 1.0) / K2       # gauge phi(0) = 0
    want_E = np.sin(k * x) * math.sin(k * dx) / (dx * K2)
    assert np.abs(phi - want_phi).max() < 1e-12 / K2
    assert np.abs(E - want_E).max() < 1e-12 / K2
    assert phi[nx] == phi[0] == 0.0 and E[nx] == E[0]


def test_periodic_background_fold_and_dense():
    nx, dx = 40, 0.3
    rng = np.random.default_rng(3)
    Q = rng.normal(size=nx + 1)
    phi, E = oracle.poisson1d_periodic(nx, dx, Q)
    # a uniform background and a move of charge between node 0 and its image change nothing
    Q2 = Q + 0.37 * dx
    Q2[nx] = Q[nx] + 0.37 * dx
    Q2[0] -= 0.37 * dx  # the fold counts nodes 0 and nx once together
    Q3 = Q.copy()
    Q3[0] += Q3[nx]
    Q3[nx] = 0.0
    for Qa in (Q2, Q3):
        p, e = oracle.poisson1d_periodic(nx, dx, Qa)
        assert np.abs(p - phi).max() < 1e-12 * np.abs(phi).max()
        assert np.abs(e - E).max() < 1e-12 * np.abs(E).max()
    # dense: the circulant Laplacian's pseudo-inverse on the zero-mean charge
    rho = np.concatenate([[Q[0] + Q[nx]], Q[1:nx]]) / dx
    rho -= rho.mean()
    A = np.zeros((nx, nx))
    for j in range(nx):
        A[j, j] = 2.0
        A[j, (j + 1) % nx] = -1.0
        A[j, (j - 1) % nx] = -1.0
    sol = np.linalg.pinv(A) @ (rho * dx * dx)
    sol -= sol[0]
    assert np.abs(phi[:nx] - sol).max() < 1e-10 * np.abs(sol).max()


def test_wrap():
    assert oracle.wrap_periodic(64.3, 64) == pytest.approx(0.3, abs=1e-13)
    assert oracle.wrap_periodic(-0.2, 64) == pytest.approx(63.8, abs=1e-13)
    assert oracle.wrap_periodic(-1e-18, 64) == 0.0
    assert oracle.wrap_periodic(12.5, 64) == 12.5
    assert oracle.wrap_periodic(-130.5, 64) == pytest.approx(61.5, abs=1e-12)


def _step_closed_form(u):
    # <min(s^2, u^2)>/3 over the Maxwell speeds (v_t = 1)
    c = math.sqrt(2 / math.pi)
    e = math.exp(-u * u / 2)
    below_s4 = 3 * (erf(u / math.sqrt(2)) - c * u * e) - c * u ** 3 * e  # int_0^u s^2 * s^2 pdf
    above = 1 - erf(u / math.sqrt(2)) + c * u * e                          # P(s > u)
    return (below_s4 + u * u * above) / 3.0


@pytest.mark.parametrize("u", [0.01, 0.1, 0.5, 1.0, 2.0, 4.0])
def test_plasma_frequency_closed_form_step(u):
    assert oracle.slpic_plasma_freq2("step", u) == pytest.approx(_step_closed_form(u), rel=1e-9)
    assert oracle.slpic_plasma_freq2("step", u, vt=2.0) == pytest.approx(_step_closed_form(u / 2.0), rel=1e-9)


def test_plasma_frequency_limits_and_smooth_monte_carlo():
    assert oracle.slpic_plasma_freq2("step", math.inf) == pytest.approx(1.0, rel=1e-12)
    assert oracle.slpic_plasma_freq2("smooth", math.inf) == pytest.approx(1.0, rel=1e-12)
    assert math.sqrt(oracle.slpic_plasma_freq2("step", 1e-3)) == pytest.approx(1e-3 / math.sqrt(3), rel=1e-6)
    rng = np.random.default_rng(0)
    v = rng.normal(size=(2_000_000, 3))
    s2 = (v ** 2).sum(axis=1)
    for u in (0.2, 1.0):
        beta = 1.0 / np.sqrt(1.0 + s2 / u ** 2)
        mc = np.mean((beta * v[:, 0]) ** 2)
        err = np.std((beta * v[:, 0]) ** 2) / math.sqrt(len(s2))
        assert abs(oracle.slpic_plasma_freq2("smooth", u) - mc) < 5 * err


def test_dispersion_limits():
    """The finite-k root: k -> 0 gives omega_p^2 <(beta v_x)^2>/v_t^2 (the
    paper's long-wavelength result); a limit above every speed (beta = 1)
    gives Bohm-Gross, omega^2 = 1 + 3 k^2 + O(k^4); the root rises with k."""
    for u in (0.05, 0.25, 1.0):
        w0 = oracle.slpic_dispersion("step", u, 1e-4)
        assert w0 == pytest.approx(math.sqrt(oracle.slpic_plasma_freq2("step", u)), rel=1e-6)
        assert oracle.slpic_dispersion("step", u, 0.1) > w0
    w0s = oracle.slpic_dispersion("smooth", 0.3, 1e-4)
    assert w0s == pytest.approx(math.sqrt(oracle.slpic_plasma_freq2("smooth", 0.3)), rel=1e-6)
    for k in (0.02, 0.05):
        w = oracle.slpic_dispersion("step", 13.0, k)
        assert w * w == pytest.approx(1 + 3 * k * k, abs=20 * k ** 4)


def _oracle_langmuir(u, nx, ppc, periods, amplitude):
    """The fundamental mode of a periodic box whose electrons are displaced
    by a small sine: the measured frequency of its E amplitude."""
    cfg = workloads.langmuir_box(u, nx=nx, ppc=ppc, seed=7, sort_every=0)
    run = oracle.Run(cfg)
    x, vx, vy, vz = run.particles(0)
    run.set_particles(0, workloads.langmuir_displacement(x, nx, amplitude), vx, vy, vz)
    run.refresh_fields()
    k = 2 * math.pi / (nx * cfg["dx"])
    w_ref = math.sqrt(1 + 3 * k * k) if math.isinf(cfg["u"]) else oracle.slpic_dispersion("step", cfg["u"], k)
    steps = int(periods * 2 * math.pi / w_ref / cfg["dt"])
    ts, ys = [], []
    for n in range(steps):
        run.step(1)
        ts.append((n + 1) * cfg["dt"])
        ys.append(run.monitor())
    return workloads.fit_frequency(np.array(ts), np.array(ys), w_ref), w_ref


def test_oracle_langmuir_pic_matches_bohm_gross():
    """u = inf: a 5 % density perturbation of a 64-cell box (k lambda_D =
    0.196) oscillates at the Bohm-Gross frequency sqrt(1 + 3 k^2 lambda_D^2)
    omega_p (to 2 %; leapfrog and finite-grid corrections are smaller)."""
    w, w_ref = _oracle_langmuir(math.inf, 64, 200, 5, 0.05)
    assert w == pytest.approx(w_ref, rel=0.02)


def test_oracle_langmuir_speed_limited():
    """u = 0.25 v_te, 64 cells (k lambda_D = 0.196), a 2 % perturbation
    (linear: the velocity excursion stays well below v_te): the oscillation
    runs at the root of the speed-limited dispersion relation, 0.149 omega_p
    (to 4 %), far below omega_p."""
    w, w_ref = _oracle_langmuir(0.25, 64, 1000, 5, 0.02)
    assert w == pytest.approx(w_ref, rel=0.04)
    assert w < 0.2

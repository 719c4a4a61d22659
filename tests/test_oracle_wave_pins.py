"""Pins of the oracle's test-particle push in a prescribed traveling wave
(Sec. V): second-order convergence to an independent ODE integrator of
Eq. (10a, b) with and without a speed limit, the trapping bound of the wave's
separatrix, exact reduction to the unlimited push for particles that stay
below the limit, and the wave-locked motion of particles above a speed limit
equal to the phase velocity."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads


def _wave(u, dt, ramp=0.0, L=20.0, phi=0.1):
    return {"length": L, "v_phase": 1.0, "phi_max": phi, "ramp_time": ramp, "qm": -1.0, "dt": dt, "u": u,
            "beta_kind": "step"}


def _beta(u, v):
    return 1.0 if (math.isinf(u) or abs(v) <= u) else u / abs(v)


def _reference(w, x0, v0, t1):
    """Eq. (10a, b) with the prescribed field, integrated by DOP853 from
    (x0, v0) at t = 0."""
    k = 2 * math.pi / w["length"]

    def acc(x, t):
        phi0 = w["phi_max"] if not w["ramp_time"] else w["phi_max"] * min(1.0, t / w["ramp_time"])
        return -w["qm"] * phi0 * k * math.cos(k * (x - w["v_phase"] * t))

    def rhs(t, y):
        b = _beta(w["u"], y[1])
        return [b * y[1], b * acc(y[0], t)]

    return integrate.solve_ivp(rhs, (0.0, t1), [x0, v0], method="DOP853", rtol=1e-12, atol=1e-12,
                               dense_output=True)


@pytest.mark.parametrize("u", [math.inf, 1.5])
def test_wave_push_second_order(u):
    """The leapfrog positions at t = n dt converge at second order to the ODE
    solution (the exact frozen-field velocity map keeps the scheme second
    order with the speed limit too)."""
    x0, vmid = 3.0, 1.3
    t1 = 16.0
    errs = []
    for dt in (0.2, 0.1, 0.05):
        w = _wave(u, dt)
        n = int(round(t1 / dt))
        x, v = oracle.wave_push(w, [x0], [vmid], 0, n)
        # reference from the same staggered start: v(0) from one half step of
        # the ODE's velocity equation at x0 (second-order consistent)
        k = 2 * math.pi / w["length"]
        a0 = -w["qm"] * w["phi_max"] * k * math.cos(k * x0)
        v0 = vmid + 0.5 * dt * _beta(u, vmid) * a0
        ref = _reference(w, x0, v0, t1)
        d = abs(((x[0] - ref.y[0, -1]) + w["length"] / 2) % w["length"] - w["length"] / 2)
        errs.append(d)
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.3), errs
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.3), errs


def test_trapped_orbits_stay_inside_the_separatrix():
    """Without a limit and at constant amplitude the wave-frame energy
    H = (v - v_phi)^2 / 2 + (q/m) phi0 sin(k xi) is conserved; a trapped
    orbit (H below the separatrix value |q/m| phi0) keeps |v - v_phi| within
    the separatrix half-width 2 sqrt(|q/m| phi0) = 0.632 v_te at phi0 = 0.1."""
    w = _wave(math.inf, 0.05)
    k = 2 * math.pi / w["length"]
    half = 2 * math.sqrt(0.1)
    assert half == pytest.approx(0.632, abs=1e-3)
    rng = np.random.default_rng(3)
    xs = rng.uniform(0, w["length"], 400)
    ws = rng.uniform(-half, half, 400)
    H = 0.5 * ws ** 2 + w["qm"] * w["phi_max"] * np.sin(k * xs)
    trapped = H < 0.85 * abs(w["qm"]) * w["phi_max"]
    x, v = xs[trapped], 1.0 + ws[trapped]
    assert len(x) > 50
    vmax = np.abs(v - 1.0)
    step = 0
    for _ in range(60):  # ~10 bounce periods
        x, v = oracle.wave_push(w, x, v, step, 50)
        step += 50
        vmax = np.maximum(vmax, np.abs(v - 1.0))
    assert vmax.max() <= half * 1.01
    assert vmax.max() >= 0.5 * half  # the orbits do reach deep into the bucket


def test_speed_limit_above_the_motion_is_exact_pic():
    """Step beta with v0 = 2 v_phi: a particle whose speed stays below v0
    moves exactly as without a limit (beta = 1 on its whole path, the in-band
    update is v + a dt)."""
    w_inf = _wave(math.inf, 0.1, ramp=200.0)
    w_lim = dict(w_inf, u=2.0)
    rng = np.random.default_rng(1)
    x0 = rng.uniform(0, 20, 500)
    v0 = rng.normal(0.8, 0.2, 500)
    xa, va = x0.copy(), v0.copy()
    xb, vb = x0.copy(), v0.copy()
    below = np.ones(500, dtype=bool)
    for s in range(0, 3000, 100):
        xa, va = oracle.wave_push(w_inf, xa, va, s, 100)
        xb, vb = oracle.wave_push(w_lim, xb, vb, s, 100)
        below &= np.abs(va) < 1.9
    assert below.sum() > 400
    assert np.array_equal(xa[below], xb[below]) and np.array_equal(va[below], vb[below])


def test_limit_at_the_phase_velocity_locks_fast_particles_to_the_wave():
    """v0 = v_phi: a particle faster than v0 moves at exactly v0 = v_phi, so
    its wave phase x - v_phi t stays fixed and, with c = 0, each step changes
    v|v| by exactly 2 a v0 dt at the frozen field (G_0(p) = p|p|/2)."""
    w = _wave(1.0, 0.1)
    k = 2 * math.pi / w["length"]
    x, v = np.array([5.0]), np.array([1.6])
    xi0 = x[0]
    for s in range(20):
        t = s * w["dt"]
        a = oracle.wave_accel(w, x[0], t)
        x1, v1 = oracle.wave_push(w, x, v, s, 1)
        if abs(v1[0]) > 1.0:
            assert v1[0] * abs(v1[0]) == pytest.approx(v[0] * abs(v[0]) + 2 * a * 1.0 * w["dt"], rel=1e-13)
            xi = (x1[0] - w["v_phase"] * (s + 1) * w["dt"]) % w["length"]
            assert xi == pytest.approx(xi0, abs=1e-11)
        x, v = x1, v1
    assert k > 0


def test_wave_workload_and_ramp():
    w, x, v = workloads.wave_test(2.0, n=1000)
    assert w["dt"] == 0.5 and w["ramp_time"] == 2000.0 and len(x) == 1000
    # the amplitude reaches phi_max after the ramp: the acceleration's
    # amplitude is |q/m| phi0 k
    k = 2 * math.pi / w["length"]
    t = 2500.0
    xs = np.linspace(0, w["length"], 401)
    amax = max(abs(oracle.wave_accel(w, xx, t)) for xx in xs)
    assert amax == pytest.approx(0.1 * k, rel=1e-4)
    assert abs(oracle.wave_accel(w, 3.0, 0.0)) == 0.0

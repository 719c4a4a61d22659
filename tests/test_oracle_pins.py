"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself: a
published known-answer vector, a closed form, an independent ODE integrator
(SciPy DOP853), a dense linear solve, a brute-force hand deposit, NumPy's
stable sort, a textbook leapfrog, or sampling statistics.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ RNG
def test_philox_known_answers():
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        vals = [int(x, 16) for x in row]
        assert oracle.philox4x32_10(vals[0:4], vals[4:6]) == vals[6:10]


def test_u53_bit_layout():
    assert oracle.u53(0, 0) == 0.0
    assert oracle.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert oracle.u53(1 << 5, 0) == 2.0 ** -27
    assert oracle.u53(0, 1 << 6) == 2.0 ** -53


# ------------------------------------------------------------------ beta, Eq. (11a,b)
def test_beta_closed_forms():
    u = 0.37
    # Eq. (11b): 1 inside the band (and on its edge), v0/|v| outside
    assert oracle.beta("step", u, 0.0) == 1.0
    assert oracle.beta("step", u, 0.5 * u) == 1.0
    assert oracle.beta("step", u, u) == 1.0
    assert oracle.beta("step", u, 2 * u) == pytest.approx(0.5, rel=1e-15)
    assert oracle.beta("step", u, 10 * u) == pytest.approx(0.1, rel=1e-15)
    # Eq. (11a): v0 / sqrt(|v|^2 + v0^2)
    assert oracle.beta("smooth", u, 0.0) == 1.0
    assert oracle.beta("smooth", u, u) == pytest.approx(1 / math.sqrt(2), rel=1e-15)
    assert oracle.beta("smooth", u, math.sqrt(3) * u) == pytest.approx(0.5, rel=1e-15)
    # no speed limit: standard PIC
    for kind in ("step", "smooth"):
        assert oracle.beta(kind, math.inf, 123.0) == 1.0
        # the simulated speed beta |v| never exceeds v0
        for s in np.linspace(0, 50 * u, 101):
            assert oracle.beta(kind, u, s) * s <= u * (1 + 1e-15)


# ------------------------------------------------------------------ G and its inverse
def test_G_is_antiderivative_of_speed():
    rng = np.random.default_rng(1)
    for _ in range(200):
        c2 = float(rng.uniform(0, 4)) ** 2
        p = float(rng.normal() * 3)
        h = 1e-4 * max(1.0, abs(p))
        # 4th-order central difference of G vs sqrt(p^2 + c^2)
        d = (-oracle.G(c2, p + 2 * h) + 8 * oracle.G(c2, p + h) - 8 * oracle.G(c2, p - h)
             + oracle.G(c2, p - 2 * h)) / (12 * h)
        assert d == pytest.approx(math.sqrt(p * p + c2), rel=1e-8)
        assert oracle.G(c2, -p) == pytest.approx(-oracle.G(c2, p), rel=1e-14, abs=1e-300)
    assert oracle.G(2.0, 0.0) == 0.0
    assert oracle.G(0.0, -3.0) == -4.5  # G_0(p) = p|p|/2


def test_fast_advance_inverts_G():
    rng = np.random.default_rng(2)
    for _ in range(500):
        c2 = float(rng.choice([0.0, 1e-6, float(rng.uniform(0, 3)) ** 2]))
        p0 = float(rng.normal() * 2)
        K = float(10 ** rng.uniform(-8, 1))
        p1 = oracle.fast_advance(c2, p0, K)
        assert p1 >= p0
        resid = oracle.G(c2, p1) - oracle.G(c2, p0) - K
        scale = abs(oracle.G(c2, p1)) + abs(oracle.G(c2, p0)) + K
        assert abs(resid) <= 1e-13 * scale
    # c = 0 closed form: p1|p1|/2 = p0|p0|/2 + K
    for p0, K in [(-2.0, 1.0), (-2.0, 3.0), (0.5, 2.0), (-1e-3, 5.0)]:
        Q = 0.5 * p0 * abs(p0) + K
        want = math.copysign(math.sqrt(2 * abs(Q)), Q)
        assert oracle.fast_advance(0.0, p0, K) == pytest.approx(want, rel=1e-14)


# ------------------------------------------------------------------ the velocity map, Eq. (A2a)
def _ode_kick(kind, u, dt, v, a):
    """Independent integration of dv/dt = beta(|v|) a (Eq. A1b, E frozen)."""
    def rhs(t, y):
        s = math.sqrt(y[0] ** 2 + y[1] ** 2 + y[2] ** 2)
        if math.isinf(u):
            b = 1.0
        elif kind == "smooth":
            b = u / math.sqrt(s * s + u * u)
        else:
            b = 1.0 if s <= u else u / s
        return [b * a[0], b * a[1], b * a[2]]
    sol = integrate.solve_ivp(rhs, (0.0, dt), list(v), method="DOP853", rtol=1e-13, atol=1e-15,
                              max_step=dt / 2000)
    return sol.y[:, -1]


KICK_CASES = [
    # (kind, u, dt, v, a): one case per segment pattern of Eq. (11b)
    ("step", 1.0, 1.0, [-3.0, 0.2, 0.1], [1.5, 0.0, 0.0]),    # fast -> band -> fast
    ("step", 1.0, 0.3, [-3.0, 0.2, 0.1], [1.5, 0.0, 0.0]),    # stays fast, approaching
    ("step", 1.0, 1.0, [-1.5, 0.2, 0.0], [1.0, 0.0, 0.0]),    # fast -> band (ends inside)
    ("step", 1.0, 2.0, [0.2, 0.3, 0.1], [0.8, 0.0, 0.0]),     # band -> fast
    ("step", 1.0, 2.0, [2.0, 0.1, 0.1], [-0.5, 0.0, 0.0]),    # decelerating fast particle
    ("step", 0.5, 1.5, [0.3, 0.6, 0.2], [2.0, 0.0, 0.0]),     # c >= u: always fast
    ("step", 1.0, 1.0, [-2.0, 0.0, 0.0], [3.0, 0.0, 0.0]),    # c = 0 crossing the band
    ("step", 0.7, 1.0, [0.5, -0.4, 0.9], [0.3, -1.1, 0.4]),   # general 3V direction
    ("smooth", 1.0, 1.0, [-3.0, 0.2, 0.1], [1.5, 0.0, 0.0]),
    ("smooth", 0.2, 2.0, [0.1, 0.0, 0.0], [-1.0, 0.0, 0.0]),
    ("smooth", 0.7, 1.0, [0.5, -0.4, 0.9], [0.3, -1.1, 0.4]),
]


@pytest.mark.parametrize("case", KICK_CASES)
def test_kick_matches_independent_ode(case):
    kind, u, dt, v, a = case
    got = oracle.kick_exact(kind, u, dt, v, a)
    want = _ode_kick(kind, u, dt, v, a)
    # Eq. (11b) has a kink on |v| = v0 that limits the ODE solver to ~1e-8
    tol = 1e-10 if kind == "smooth" else 2e-7
    np.testing.assert_allclose(got, want, rtol=tol, atol=tol)


def test_kick_random_against_ode():
    rng = np.random.default_rng(3)
    for _ in range(40):
        kind = str(rng.choice(["step", "smooth"]))
        u = float(10 ** rng.uniform(-1, 0.5))
        v = rng.normal(size=3)
        a = rng.normal(size=3) * float(10 ** rng.uniform(-1, 0.5))
        dt = float(10 ** rng.uniform(-1, 0.5))
        got = oracle.kick_exact(kind, u, dt, v, a)
        want = _ode_kick(kind, u, dt, v, a)
        tol = 1e-9 if kind == "smooth" else 5e-7
        np.testing.assert_allclose(got, want, rtol=tol, atol=tol)


def test_kick_special_cases():
    v = np.array([0.3, -0.2, 0.1])
    # no field: velocity unchanged
    assert np.array_equal(oracle.kick_exact("step", 0.5, 1.0, v, [0, 0, 0]), v)
    # u = inf is the standard leapfrog kick, bit for bit (Eq. 4)
    a = np.array([0.7, 0.0, 0.0])
    for kind in ("step", "smooth"):
        assert np.array_equal(oracle.kick_exact(kind, math.inf, 0.25, v, a), v + a * 0.25)
    # a path that stays inside the band |v| <= v0 is the standard kick too
    assert np.array_equal(oracle.kick_exact("step", 2.0, 0.25, v, a), v + a * 0.25)
    # 1V, always above v0: v1|v1| = v0|v0| + 2 a dt v0 (closed form)
    for p0, A, dt in [(2.0, 1.0, 0.5), (-3.0, 2.0, 0.2), (1.5, -0.3, 1.0)]:
        u = 0.5
        got = oracle.kick_exact("step", u, dt, [p0, 0, 0], [A, 0, 0])[0]
        Q = p0 * abs(p0) + 2 * A * dt * u
        want = math.copysign(math.sqrt(abs(Q)), Q)
        assert abs(want) > u and abs(p0) > u
        assert got == pytest.approx(want, rel=1e-14)


def test_mmp_converges_to_exact():
    for kind, u, dt, v, a in KICK_CASES:
        exact = oracle.kick_exact(kind, u, dt, v, a)
        tight, n = oracle.kick_mmp(kind, u, dt, v, a, tol=1e-11)
        np.testing.assert_allclose(tight, exact, rtol=1e-6, atol=1e-6)
        # the paper's 1 % tolerance: the integral of beta is within a few percent
        loose, _ = oracle.kick_mmp(kind, u, dt, v, a, tol=1e-2)
        A = np.linalg.norm(a)
        I_exact = np.dot(exact - np.asarray(v), np.asarray(a)) / A ** 2
        I_loose = np.dot(loose - np.asarray(v), np.asarray(a)) / A ** 2
        assert abs(I_loose - I_exact) <= 0.05 * abs(I_exact)


def _slpic_orbit(kind, u, dt, x0, v0, a, T):
    """Uniform field: repeated Eq. (A2a,b) steps (velocity at half steps)."""
    n = int(round(T / dt))
    x = x0
    v = np.array(v0, dtype=float)
    # start the half-step velocity exactly: v^{-1/2} -> v^{1/2} covers [-dt/2, dt/2]
    v = oracle.kick_exact(kind, u, dt / 2, v, [a, 0, 0])
    for _ in range(n):
        s = np.linalg.norm(v)
        x = x + oracle.beta(kind, u, s) * v[0] * dt
        v = oracle.kick_exact(kind, u, dt, v, [a, 0, 0])
    return x


@pytest.mark.parametrize("kind,u", [("smooth", 0.8), ("step", 0.3)])
def test_uniform_field_orbit_second_order(kind, u):
    """Eq. (10) in a uniform field: the discrete orbit converges at order 2
    (the velocity map is exact for a frozen field; the position update is a
    midpoint rule).  For Eq. (11b) the case stays above v0 (|v_perp| > v0):
    a crossing of the kink at |v| = v0 lowers the observed order."""
    a, T = -0.6, 4.0
    x0, v0 = 0.0, [1.5, 0.3, 0.2]

    def rhs(t, y):
        s = math.sqrt(y[1] ** 2 + y[2] ** 2 + y[3] ** 2)
        b = (1.0 if s <= u else u / s) if kind == "step" else u / math.sqrt(s * s + u * u)
        return [b * y[1], b * a, 0.0, 0.0]
    ref = integrate.solve_ivp(rhs, (0, T), [x0] + v0, method="DOP853", rtol=1e-12, atol=1e-14,
                              max_step=1e-3).y[0, -1]
    errs = [abs(_slpic_orbit(kind, u, dt, x0, v0, a, T) - ref) for dt in (0.2, 0.1, 0.05)]
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.05)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.05)


def test_same_path_slower():
    """Eq. (10) vs Eq. (4): a speed-limited particle in a static uniform field
    keeps |v|^2/2 - a.x constant, i.e. it follows the PIC phase-space path."""
    u, a = 0.4, np.array([0.5, 0.0, 0.0])
    v = np.array([-2.0, 0.3, 0.0])
    x = 0.0
    dt = 1e-3
    v0 = oracle.kick_exact("step", u, dt / 2, v, a)  # v at t = 0 from v^{-1/2}
    H0 = 0.5 * v0 @ v0 - a[0] * x
    for _ in range(3000):
        v_new = oracle.kick_exact("step", u, dt, v, a)
        # midpoint of the half-step velocities, position at the same time
        x += oracle.beta("step", u, np.linalg.norm(v_new)) * v_new[0] * dt
        v = v_new
    vm = oracle.kick_exact("step", u, dt / 2, v, a)
    H = 0.5 * vm @ vm - a[0] * x
    assert abs(H - H0) < 1e-6


# ------------------------------------------------------------------ Poisson, Eq. (A2d)
def _charge_from_density(rho, nx, dx):
    dV = np.full(nx + 1, dx)
    dV[0] = dV[-1] = dx / 2
    return rho * dV


def test_poisson_uniform_charge_is_exact_quadratic():
    nx, dx, rho0 = 37, 0.3, 1.7
    L = nx * dx
    x = np.arange(nx + 1) * dx
    phi, E = oracle.poisson1d(nx, dx, _charge_from_density(np.full(nx + 1, rho0), nx, dx))
    np.testing.assert_allclose(phi, rho0 * (L ** 2 - x ** 2) / 2, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(E, rho0 * x, rtol=1e-11, atol=1e-12)
    assert E[0] == 0.0
    # Gauss: the wall field equals the total charge per unit area
    assert E[-1] == pytest.approx(rho0 * L, rel=1e-11)


def test_poisson_discrete_eigenmode():
    nx, dx = 64, 0.5
    L = nx * dx
    x = np.arange(nx + 1) * dx
    for m in (0, 3, 11):
        k = (m + 0.5) * math.pi / L
        lam = (2 - 2 * math.cos(k * dx)) / dx ** 2
        rho = np.cos(k * x)
        phi, _ = oracle.poisson1d(nx, dx, _charge_from_density(rho, nx, dx))
        np.testing.assert_allclose(phi[:-1], rho[:-1] / lam, rtol=1e-9, atol=1e-10)
        assert phi[-1] == 0.0


def test_poisson_dense_solve():
    rng = np.random.default_rng(4)
    nx, dx = 48, 0.25
    Q = rng.normal(size=nx + 1)
    phi, E = oracle.poisson1d(nx, dx, Q)
    rho = Q / _charge_from_density(np.ones(nx + 1), nx, dx)
    # rows of -phi'' = rho: node 0 symmetry, nodes 1..nx-1 interior, phi_nx = 0
    M = np.zeros((nx, nx))
    M[0, 0], M[0, 1] = 2.0, -2.0
    for j in range(1, nx):
        M[j, j - 1] = -1.0
        M[j, j] = 2.0
        if j + 1 < nx:
            M[j, j + 1] = -1.0
    want = np.linalg.solve(M / dx ** 2, rho[:nx])
    np.testing.assert_allclose(phi[:nx], want, rtol=1e-10, atol=1e-10)
    Ew = np.gradient(np.append(want, 0.0), dx, edge_order=2)
    np.testing.assert_allclose(E[1:], -Ew[1:], rtol=1e-9, atol=1e-9)


# ------------------------------------------------------------------ deposit, Eq. (A2c)
def _tiny_cfg(**kw):
    cfg = workloads.sheath(nx=8, ppc=1, u_over_vti=3.0, dt=1.0, sort_every=0, **kw)
    return cfg


def test_deposit_brute_force():
    cfg = _tiny_cfg()
    run = oracle.Run(cfg, load=False)
    w = run.weights()
    u = cfg["u"]
    # electron at xt = 2.25 moving at 4u (beta = 1/4); ion at xt = 5.5 at rest
    run.set_particles(0, [2.25], [4 * u], [0.0], [0.0])
    run.set_particles(1, [5.5], [0.0], [0.0], [0.0])
    run.refresh_fields()
    Q = run.grid()["Q"]
    want_e = np.zeros(9)
    want_e[2] = -w[0] * 0.25 * 0.75
    want_e[3] = -w[0] * 0.25 * 0.25
    want_i = np.zeros(9)
    want_i[5] = w[1] * 0.5
    want_i[6] = w[1] * 0.5
    np.testing.assert_allclose(Q[0], want_e, rtol=1e-15, atol=0)
    np.testing.assert_allclose(Q[1], want_i, rtol=1e-15, atol=0)


def test_deposit_charge_identity():
    cfg = workloads.small_sheath(sort_every=0)
    run = oracle.Run(cfg)
    x, vx, vy, vz = run.particles(0)
    s = np.sqrt(vx ** 2 + vy ** 2 + vz ** 2)
    u = cfg["u"]
    beta = np.where(s <= u, 1.0, u / s)
    Q = run.grid()["Q"]
    w = run.weights()
    assert Q[0].sum() == pytest.approx(-w[0] * beta.sum(), rel=1e-12)
    # the physical electron content is n0 L on average: sum w beta = L (within noise)
    assert -Q[0].sum() == pytest.approx(cfg["nx"] * cfg["dx"], rel=0.1)


# ------------------------------------------------------------------ sort
def test_sort_matches_numpy_stable():
    cfg = workloads.small_sheath(sort_every=0, sort_bucket=3)
    run = oracle.Run(cfg)
    run.step(5)
    before = [run.particles(s) for s in range(2)]
    keys_np = []
    for s in range(2):
        x = before[s][0]
        k = np.where(x < 0, -1, np.floor(np.where(x < 0, 0, x)).astype(np.int64) // 3)
        keys_np.append(k)
        assert np.array_equal(run.keys(s), k)
    perms = run.sort()
    for s in range(2):
        k = keys_np[s]
        live = np.nonzero(k >= 0)[0]
        want = live[np.argsort(k[live], kind="stable")]
        assert np.array_equal(perms[s], want)
        after = run.particles(s)
        for a, b in zip(after, before[s]):
            assert np.array_equal(a, b[want])


# ------------------------------------------------------------------ loading g0 = f0/beta
def test_Z_against_quadrature():
    for ut in (0.003, 0.5, 1.0, 3.0, 10.0):
        pdf = lambda s: math.sqrt(2 / math.pi) * s * s * math.exp(-s * s / 2)
        z_step = integrate.quad(lambda s: pdf(s) * max(1.0, s / ut), 0, 60, points=[ut], limit=400,
                                epsabs=1e-14, epsrel=1e-13)[0]
        assert oracle.Z("step", ut) == pytest.approx(z_step, rel=1e-10)
        z_sm = integrate.quad(lambda s: pdf(s) * math.sqrt(1 + (s / ut) ** 2), 0, 60, limit=400,
                              epsabs=1e-14, epsrel=1e-13)[0]
        assert oracle.Z("smooth", ut) == pytest.approx(z_sm, rel=1e-9)
    assert oracle.Z("step", math.inf) == 1.0


def _g_speed_cdf(kind, ut):
    pdf = lambda s: math.sqrt(2 / math.pi) * s * s * math.exp(-s * s / 2) * (
        max(1.0, s / ut) if kind == "step" else math.sqrt(1 + (s / ut) ** 2))
    Z = oracle.Z(kind, ut)
    grid = np.linspace(0, 12, 6001)
    vals = np.array([pdf(s) for s in grid])
    cdf = integrate.cumulative_trapezoid(vals, grid, initial=0) / Z
    return lambda s: np.interp(s, grid, cdf)


@pytest.mark.parametrize("kind,ut", [("step", 0.4), ("step", 3.0), ("smooth", 1.5)])
def test_loader_samples_g_equals_f_over_beta(kind, ut):
    vt = 1.0
    cfg = workloads.sheath(nx=200, ppc=100, u_over_vti=3.0, dt=1.0, beta_kind=kind)
    cfg["species"][0]["temperature"] = 1.0
    cfg["u"] = ut * vt
    n = 20000
    P = np.array([oracle.load_particle(cfg, 0, i) for i in range(n)])
    x, v = P[:, 0], P[:, 1:]
    assert np.all((x >= 0) & (x < cfg["nx"]))
    s = np.linalg.norm(v, axis=1) / vt
    # speeds follow the g density (KS), directions are isotropic
    assert stats.kstest(s, _g_speed_cdf(kind, ut)).pvalue > 1e-3
    mu = v[:, 0] / np.linalg.norm(v, axis=1)
    assert abs(mu.mean()) < 4 / math.sqrt(3 * n)
    assert abs((mu ** 2).mean() - 1 / 3) < 0.02
    # beta-weighting recovers the Maxwellian: <beta> = 1/Z, <beta v^2>/<beta> = 3 vt^2
    u = ut * vt
    beta = (np.where(s * vt <= u, 1.0, u / (s * vt)) if kind == "step"
            else u / np.sqrt((s * vt) ** 2 + u * u))
    assert beta.mean() == pytest.approx(1 / oracle.Z(kind, ut), rel=0.03)
    assert (beta * (s * vt) ** 2).sum() / beta.sum() == pytest.approx(3 * vt ** 2, rel=0.05)


def test_loader_unlimited_is_maxwellian():
    cfg = workloads.sheath(nx=100, ppc=10, u_over_vti=math.inf, dt=0.1)
    P = np.array([oracle.load_particle(cfg, 0, i) for i in range(20000)])
    for k in (1, 2, 3):
        assert stats.kstest(P[:, k], "norm").pvalue > 1e-3


def test_inject_maxwellian_in_source():
    cfg = workloads.small_sheath()
    vt = oracle.thermal_speed(cfg, 1)
    P = np.array([oracle.inject_particle(cfg, 1, k, 17) for k in range(20000)])
    assert np.all((P[:, 0] >= 0) & (P[:, 0] < cfg["source_cells"]))
    for k in (1, 2, 3):
        assert stats.kstest(P[:, k] / vt, "norm").pvalue > 1e-3
    # a different step gives a different draw
    assert not np.array_equal(oracle.inject_particle(cfg, 1, 0, 17), oracle.inject_particle(cfg, 1, 0, 18))


# ------------------------------------------------------------------ the step
def test_unlimited_step_is_textbook_leapfrog():
    """u = inf: one SLPIC step equals a standard PIC leapfrog step bit for bit
    (the paper: with beta = 1, SLPIC is PIC)."""
    cfg = workloads.sheath(nx=32, ppc=20, u_over_vti=math.inf, dt=0.1, sort_every=0)
    run = oracle.Run(cfg)
    E = run.grid()["E"]
    before = [run.particles(s) for s in range(2)]
    run.step(1)
    dtdx = cfg["dt"] / cfg["dx"]
    for s in range(2):
        qm = cfg["species"][s]["charge"] / cfg["species"][s]["mass"]
        x, vx, vy, vz = before[s]
        c = np.floor(x).astype(int)
        f = x - c
        Ex = E[c] * (1 - f) + E[c + 1] * f
        vn = vx + (qm * Ex) * cfg["dt"]
        xn = x + vn * dtdx
        refl = xn < 0
        xn = np.where(refl, -xn, xn)
        vn = np.where(refl, -vn, vn)
        dead = xn >= cfg["nx"]
        xo, vxo, vyo, vzo = run.particles(s)
        n = len(x)
        assert np.array_equal(xo[:n][~dead], xn[~dead])
        assert np.array_equal(vxo[:n][~dead], vn[~dead])
        assert np.all(xo[:n][dead] < 0)
        assert np.array_equal(vyo[:n], vy) and np.array_equal(vzo[:n], vz)


def test_step_bookkeeping_source_balances_ion_loss():
    cfg = workloads.small_sheath(sort_every=0)
    run = oracle.Run(cfg)
    w = run.weights()
    run.step(200)
    ai, ii = run.absorbed_total(1), run.injected_total(1)
    ie = run.injected_total(0)
    assert ai > 0 and ii == ai
    # electrons injected carry the same physical number as the ions lost
    assert ie + run.acc_e == pytest.approx(ai * w[1] / w[0], rel=1e-12)
    for s in range(2):
        n0 = cfg["nx"] * cfg["species"][s]["ppc"]
        assert run.nlive(s) == n0 - run.absorbed_total(s) + run.injected_total(s)


def test_mmp_one_percent_step_close_to_exact():
    """Appendix: the 1 % quadrature and the exact integral give nearly the same step."""
    base = workloads.small_sheath(sort_every=0, ppc=20)
    a = oracle.Run(dict(base, kick="exact"))
    b = oracle.Run(dict(base, kick="mmp", mmp_tol=0.01))
    a.step(1)
    b.step(1)
    Qa, Qb = a.grid()["Q"], b.grid()["Q"]
    for s in range(2):
        assert np.abs(Qa[s] - Qb[s]).max() <= 0.02 * np.abs(Qa[s]).max()


def test_moments_brute_force():
    """beta-weighted moments of f = beta g (Eq. 5) for one hand-placed particle."""
    cfg = _tiny_cfg()
    run = oracle.Run(cfg, load=False)
    w = run.weights()
    u = cfg["u"]
    v = np.array([3 * u, 4 * u, 0.0])  # |v| = 5u, beta = 1/5
    run.set_particles(0, [0.25], [v[0]], [v[1]], [v[2]])
    run.set_particles(1, [7.0], [0.0], [0.0], [0.0])
    run.refresh_fields()
    M = run.moments()
    dx = cfg["dx"]
    dV = np.full(9, dx)
    dV[0] = dV[-1] = dx / 2
    n_e = np.zeros(9)
    n_e[0], n_e[1] = w[0] * 0.2 * 0.75, w[0] * 0.2 * 0.25
    n_e /= dV
    np.testing.assert_allclose(M[1], n_e, rtol=1e-14)
    np.testing.assert_allclose(M[2], n_e * v[0], rtol=1e-14)
    np.testing.assert_allclose(M[3], n_e * 0.5 * (v @ v), rtol=1e-14)
    n_i = np.zeros(9)
    n_i[7] = w[1] / dx
    np.testing.assert_allclose(M[4], n_i, rtol=1e-14)
    assert np.all(M[5] == 0) and np.all(M[6] == 0)
    np.testing.assert_array_equal(M[0], run.grid()["phi"])
    # density moment and the deposited charge agree: n_s = Q_s / (q_s dV)
    Q = run.grid()["Q"]
    np.testing.assert_allclose(M[1], -Q[0] / dV, rtol=1e-14)


def test_one_step_against_independent_particle_ode():
    """Composition of Eq. (A2a,b) in one step (gather, exact kick, beta-weighted
    position update, specular reflection, absorption) against SciPy's
    integration of Eq. (A1a,b) with E frozen at E^n(x^n)."""
    cfg = workloads.sheath(nx=16, ppc=8, u_over_vti=3.0, dt=5.0, te_over_ti=20.0, sort_every=0)
    run = oracle.Run(cfg)
    run.step(3)
    E = run.grid()["E"]
    before = [run.particles(s) for s in range(2)]
    run.step(1)
    u, dt, dx = cfg["u"], cfg["dt"], cfg["dx"]
    rng = np.random.default_rng(5)
    for s in range(2):
        qm = cfg["species"][s]["charge"] / cfg["species"][s]["mass"]
        x, vx, vy, vz = before[s]
        xo, vxo, vyo, vzo = run.particles(s)
        live = np.nonzero(x >= 0)[0]
        for i in rng.choice(live, size=25, replace=False):
            c = int(np.floor(x[i]))
            f = x[i] - c
            a = qm * (E[c] * (1 - f) + E[c + 1] * f)
            v1 = _ode_kick("step", u, dt, [vx[i], vy[i], vz[i]], [a, 0.0, 0.0])
            sp = np.linalg.norm(v1)
            b = 1.0 if sp <= u else u / sp
            xn = x[i] + b * v1[0] * dt / dx
            if xn < 0:
                xn, v1[0] = -xn, -v1[0]
            if xn >= cfg["nx"]:
                assert xo[i] < 0
                continue
            assert xo[i] == pytest.approx(xn, rel=1e-9, abs=1e-9)
            assert vxo[i] == pytest.approx(v1[0], rel=2e-7, abs=1e-9)
            assert vyo[i] == vy[i] and vzo[i] == vz[i]


# ---------------------------------------------------------------- steady detector
def test_steady_detector_constant_series():
    """A constant wall potential is steady when the third window closes."""
    for W in (1, 4, 16):
        d = oracle.steady_detect([3.25] * (5 * W), W, 0.02)
        assert d["steady_step"] == 3 * W
        assert d["windows"] == 5
        assert d["window_mean"] == [3.25, 3.25, 3.25]


def test_steady_detector_linear_ramp():
    """Phi_k = a + b k (k = 1, 2, ...): window j (steps (j-1)W+1 .. jW) has
    mean a + b((j-1)W + (W+1)/2); three consecutive means deviate from their
    average by at most |b| W, so the run is steady at the first j >= 3 with
    |b| W <= tol |a + b((j-2)W + (W+1)/2)|, at step jW."""
    a, b, W, tol = 2.0, 0.01, 8, 0.02
    n = 4000
    series = [a + b * k for k in range(1, n + 1)]
    d = oracle.steady_detect(series, W, tol)
    j = 3
    while not abs(b) * W <= tol * abs(a + b * ((j - 2) * W + (W + 1) / 2)):
        j += 1
    assert d["steady_step"] == j * W
    # the window means themselves (closed form)
    jl = n // W
    for k, m in enumerate(d["window_mean"]):
        assert m == pytest.approx(a + b * ((jl - 1 - k) * W + (W + 1) / 2), rel=1e-13)


def test_steady_detector_step_change():
    """A relaxing series that is flat (Phi = 1) from step K0 + 1 on, with
    Phi_k = 2 + K0 - k >= 2 before: a window holding any step <= K0 has a mean
    of at least 1 + 1/W, far outside 2 % of the flat windows, so the run is
    steady once all three windows lie after K0, at step (3 + ceil(K0/W)) W."""
    W, K0 = 10, 37
    series = [2.0 + K0 - k if k <= K0 else 1.0 for k in range(1, 200)]
    d = oracle.steady_detect(series, W, 0.02)
    assert d["steady_step"] == (3 + math.ceil(K0 / W)) * W


def test_steady_detector_matches_run_history():
    """The detector inside a run sees the run's own wall potential after each
    step (defaults: W = nx/4, tol = 0.02)."""
    cfg = workloads.small_sheath(sort_every=1)
    run = oracle.Run(cfg)
    series = []
    for _ in range(200):
        run.step(1)
        series.append(run.wall_potential())
    d = oracle.steady_detect(series, cfg["nx"] // 4, 0.02)
    got = run.steady()
    assert got["steady_step"] == d["steady_step"]
    assert got["windows"] == d["windows"] == 200 // (cfg["nx"] // 4)
    assert got["window_mean"] == d["window_mean"]


# ---------------------------------------------------------------- warm load
def _uniform_profile(n=1.0, gamma=0.0):
    p = np.zeros((5, 256))
    p[1] = p[2] = n
    p[3] = p[4] = gamma
    return p


def test_warm_load_uniform_profile_reproduces_cold_counts():
    """A uniform, drift-free profile at n0 = 1: every cell holds ppc
    g-particles, as the cold load does on average (the warm Z by quadrature
    equals the closed-form Z of the weight)."""
    for kind in ("step", "smooth"):
        cfg = workloads.sheath(nx=16, ppc=50, u_over_vti=3.0, dt=5.0, beta_kind=kind)
        w = oracle.Run(cfg, load=False).weights()
        for s in range(2):
            for c in (0, 7, 15):
                cnt, V, vt = oracle.warm_cell_count(cfg, s, _uniform_profile(), c, w[s])
                assert cnt == 50 and V == 0.0, (kind, s, c, cnt)
                # zero temperature rows stand for the source temperature
                T0 = cfg["species"][s]["temperature"]
                assert vt == math.sqrt(T0 / cfg["species"][s]["mass"])
                hot = oracle.warm_profile(_uniform_profile())
                hot[5 + s] = T0
                assert oracle.warm_cell_count(cfg, s, hot, c, w[s]) == (cnt, V, vt)


def test_warm_Z_with_drift_against_cylindrical_quadrature():
    """<1/beta> over a drifting Maxwellian, integrated in cylindrical
    velocity coordinates (SciPy), fixes the expected cell count
    E = n dx Z / w that the loader's count is the floor or ceiling of."""
    cfg = workloads.sheath(nx=16, ppc=40, u_over_vti=3.0, dt=5.0)
    run = oracle.Run(cfg, load=False)
    w = run.weights()
    vt = math.sqrt(cfg["species"][1]["temperature"] / cfg["species"][1]["mass"])
    u = cfg["u"]
    vt0 = vt
    for V_over_vt, T_scale in ((0.0, 1.0), (0.7, 1.0), (2.5, 1.0), (0.7, 4.0), (1.5, 0.25)):
        vt = vt0 * math.sqrt(T_scale)  # a temperature row T_scale T_i moves the thermal speed
        V = V_over_vt * vt
        prof = oracle.warm_profile(_uniform_profile(n=0.8, gamma=0.8 * V))
        if T_scale != 1.0:
            prof[6] = T_scale * cfg["species"][1]["temperature"]
        inv_beta = lambda sp: 1.0 if sp <= u else sp / u
        dens = lambda r, a: (math.exp(-(a - V) ** 2 / (2 * vt * vt)) / (vt * math.sqrt(2 * math.pi))
                             * r / (vt * vt) * math.exp(-r * r / (2 * vt * vt)))
        Z, _ = integrate.dblquad(lambda r, a: inv_beta(math.hypot(a, r)) * dens(r, a),
                                 V - 12 * vt, V + 12 * vt, 0.0, 12 * vt, epsabs=1e-12, epsrel=1e-11)
        E = 0.8 * cfg["dx"] * Z / w[1]
        cnt, Vo, vto = oracle.warm_cell_count(cfg, 1, prof, 5, w[1])
        assert Vo == pytest.approx(V, rel=1e-12, abs=1e-300)
        assert vto == pytest.approx(vt, rel=1e-14)
        assert cnt in (math.floor(E), math.floor(E) + 1), (V_over_vt, T_scale, cnt, E)


def test_warm_load_reproduces_profile_moments():
    """The physical moments of a warm-loaded state (f = beta g, Eq. 5) match
    the profile it was drawn from: density and flux within statistics, and
    the temperature (2K/n - m V^2)/3 from the kinetic energy density K."""
    cfg = workloads.sheath(nx=32, ppc=2000, u_over_vti=3.0, dt=5.0, sort_every=1)
    xi = np.arange(256) / 255.0
    vte = 1.0
    Ti0 = cfg["species"][1]["temperature"]
    vti = math.sqrt(Ti0 / cfg["species"][1]["mass"])
    prof = np.zeros((7, 256))
    prof[1] = 1.0 + 0.5 * np.cos(math.pi * xi)     # n_e
    prof[2] = prof[1]                              # n_i
    prof[3] = prof[1] * 0.3 * vte * xi             # Gamma_e: drift 0.3 v_te at the wall
    prof[4] = prof[2] * 1.5 * vti * xi             # Gamma_i: drift 1.5 v_ti at the wall
    prof[5] = 1.0 + 3.0 * xi                       # T_e: 1 to 4 T_e
    prof[6] = Ti0 * (2.0 - xi)                     # T_i: 2 to 1 T_i
    run = oracle.Run(cfg, warm=prof)
    M = run.moments()
    nodes = np.arange(cfg["nx"] + 1) / cfg["nx"]
    inner = slice(2, cfg["nx"] - 1)                # end nodes see half a cell
    for s, (nrow, grow) in enumerate(((1, 3), (4, 6))):
        n_want = np.interp(nodes, xi, prof[1 + s])
        g_want = np.interp(nodes, xi, prof[3 + s])
        n_got, g_got = M[nrow], M[grow - 1]
        rel = np.abs(n_got[inner] - n_want[inner]) / n_want[inner]
        assert rel.mean() < 0.02 and rel.max() < 0.08, (s, rel.mean(), rel.max())
        # the flux estimate is noisy per node (each g-particle carries at most
        # w u of it): compare its average over the inner nodes
        avg_got, avg_want = g_got[inner].mean(), g_want[inner].mean()
        assert avg_got == pytest.approx(avg_want, rel=0.08), (s, avg_got, avg_want)
        m = cfg["species"][s]["mass"]
        K = M[grow]
        T_got = (2.0 * K / n_got - m * (g_got / n_got) ** 2) / 3.0
        T_want = np.interp(nodes, xi, prof[5 + s])
        relT = np.abs(T_got[inner] - T_want[inner]) / T_want[inner]
        assert relT.mean() < 0.03 and relT.max() < 0.1, (s, relT.mean(), relT.max())

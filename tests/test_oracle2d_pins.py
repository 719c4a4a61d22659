"""Pins of the 2D3V oracle (y periodic, dy = dx) against what the mathematics
and the already pinned 1D oracle fix: the five-point operator applied by
brute force, closed forms of the Poisson problem, a hand deposit, NumPy's
stable sort, free streaming, and the exact reduction of a y-uniform 2D run to
the 1D run.
"""
import math

import numpy as np
import pytest

import oracle
import workloads


def five_point_rho(phi: np.ndarray, dx: float) -> np.ndarray:
    """rho = -lap phi with the discrete operator written out node by node:
    centred second differences, x = 0 a symmetry plane (phi_{-1} = phi_1),
    y periodic.  The wall row x = nx is Dirichlet and not an equation."""
    nxp, ny = phi.shape
    rho = np.zeros_like(phi)
    for i in range(nxp - 1):
        for j in range(ny):
            left = phi[1, j] if i == 0 else phi[i - 1, j]
            d2x = (phi[i + 1, j] - 2 * phi[i, j] + left) / dx ** 2
            d2y = (phi[i, (j + 1) % ny] - 2 * phi[i, j] + phi[i, (j - 1) % ny]) / dx ** 2
            rho[i, j] = -(d2x + d2y)
    return rho


def charge_of(rho: np.ndarray, dx: float) -> np.ndarray:
    """Node charge Q = rho dV, dV = dx dy (half at the x end nodes)."""
    Q = rho * dx * dx
    Q[0] *= 0.5
    Q[-1] *= 0.5
    return Q


@pytest.mark.parametrize("nx,ny,dx", [(12, 8, 0.5), (9, 6, 1.3), (16, 16, 1.0)])
def test_poisson2d_inverts_the_five_point_operator(nx, ny, dx):
    rng = np.random.default_rng(nx * 100 + ny)
    phi_true = rng.normal(size=(nx + 1, ny))
    phi_true[-1] = 0.0  # grounded wall
    Q = charge_of(five_point_rho(phi_true, dx), dx)
    phi, Ex, Ey = oracle.poisson2d(nx, ny, dx, Q)
    assert np.abs(phi - phi_true).max() < 1e-10 * np.abs(phi_true).max()
    # E = -grad phi: centred in the interior and in y (periodic), zero at the
    # symmetry plane, the one-sided second-order difference at the wall
    for i in range(nx + 1):
        for j in range(ny):
            ey = -(phi_true[i, (j + 1) % ny] - phi_true[i, (j - 1) % ny]) / (2 * dx)
            if i == 0:
                ex = 0.0
            elif i < nx:
                ex = -(phi_true[i + 1, j] - phi_true[i - 1, j]) / (2 * dx)
            else:
                ex = -(3 * phi_true[i, j] - 4 * phi_true[i - 1, j] + phi_true[i - 2, j]) / (2 * dx)
            assert abs(Ex[i, j] - ex) < 1e-9
            assert abs(Ey[i, j] - ey) < 1e-9


def test_poisson2d_uniform_charge_closed_form():
    # uniform rho: phi = rho (L^2 - x^2)/2, exact for the three-point stencil
    nx, ny, dx, rho = 10, 8, 0.7, 0.3
    Q = charge_of(np.full((nx + 1, ny), rho), dx)
    phi, Ex, Ey = oracle.poisson2d(nx, ny, dx, Q)
    x = np.arange(nx + 1) * dx
    L = nx * dx
    want = rho * (L ** 2 - x ** 2) / 2
    assert np.abs(phi - want[:, None]).max() < 1e-12 * want.max()
    assert np.abs(Ex[1:] - (rho * x[1:])[:, None]).max() < 1e-11
    assert np.abs(Ex[0]).max() == 0.0
    assert np.abs(Ey).max() < 1e-12


def test_poisson2d_y_independent_charge_is_the_1d_solve():
    nx, ny, dx = 14, 6, 0.5
    rng = np.random.default_rng(5)
    q1 = rng.normal(size=nx + 1)
    phi1, E1 = oracle.poisson1d(nx, dx, q1)
    # per y-row the same rho: 2D node charge = 1D node charge * dy
    phi, Ex, Ey = oracle.poisson2d(nx, ny, dx, np.repeat((q1 * dx)[:, None], ny, axis=1))
    assert np.abs(phi - phi1[:, None]).max() < 1e-12 * np.abs(phi1).max()
    assert np.abs(Ex - E1[:, None]).max() < 1e-11 * np.abs(E1).max()
    assert np.abs(Ey).max() < 1e-12 * np.abs(phi1).max()


def test_poisson2d_single_fourier_mode():
    # phi = X(x) cos(2 pi k j/ny): each mode decouples with the extra term
    # (4/dy^2) sin^2(pi k/ny); pick X and form rho from the 1D operator plus
    # that term, then check the solve returns phi
    nx, ny, dx, k = 12, 8, 0.5, 3
    rng = np.random.default_rng(7)
    X = rng.normal(size=nx + 1)
    X[-1] = 0.0
    kap = 4 / dx ** 2 * math.sin(math.pi * k / ny) ** 2
    r = np.zeros(nx + 1)
    for i in range(nx):
        left = X[1] if i == 0 else X[i - 1]
        r[i] = -(X[i + 1] - 2 * X[i] + left) / dx ** 2 + kap * X[i]
    cosj = np.cos(2 * math.pi * k * np.arange(ny) / ny)
    phi_true = X[:, None] * cosj[None, :]
    Q = charge_of(r[:, None] * cosj[None, :], dx)
    phi, _, _ = oracle.poisson2d(nx, ny, dx, Q)
    assert np.abs(phi - phi_true).max() < 1e-11


def _cfg(u_over_vti=3.0, ppc=4, nx=8, **kw):
    return workloads.sheath(nx=nx, ppc=ppc, u_over_vti=u_over_vti, **kw)


def test_deposit2d_bilinear_by_hand_with_y_wrap():
    cfg = _cfg(u_over_vti=math.inf)
    nx, ny = cfg["nx"], 6
    r = oracle.Run2D(cfg, ny, load=False)
    pts = [(2.25, 5.5, 0.1, -0.2, 0.3), (0.0, 0.0, 0.0, 0.0, 0.0), (7.75, 3.125, 1.0, 2.0, 0.5)]
    x, y, vx, vy, vz = (np.array(c) for c in zip(*pts))
    r.set_particles(0, x, y, vx, vy, vz)
    r.set_particles(1, x[:1], y[:1], vx[:1], vy[:1], vz[:1])
    r.refresh_fields()
    Q = r.grid()["Q"]
    w = [r.weight(0), r.weight(1)]
    want = np.zeros((2, nx + 1, ny))
    for s, n in ((0, 3), (1, 1)):
        q = cfg["species"][s]["charge"] * w[s]
        for (px, py, *_v) in pts[:n]:
            cx, cy = int(px), int(py)
            fx, fy = px - cx, py - cy
            want[s, cx, cy] += q * (1 - fx) * (1 - fy)
            want[s, cx + 1, cy] += q * fx * (1 - fy)
            want[s, cx, (cy + 1) % ny] += q * (1 - fx) * fy
            want[s, cx + 1, (cy + 1) % ny] += q * fx * fy
    assert np.abs(Q - want).max() < 1e-15
    # weights: dx dy Z / ppc (u = inf: Z = 1)
    assert w[0] == pytest.approx(cfg["dx"] ** 2 / cfg["species"][0]["ppc"], rel=1e-15)


def test_deposit2d_beta_weighted_total_charge():
    cfg = _cfg(u_over_vti=3.0, ppc=8)
    r = oracle.Run2D(cfg, 6)
    Q = r.grid()["Q"]
    u = cfg["u"]
    for s in range(2):
        x, y, vx, vy, vz = r.particles(s)
        sp = np.sqrt(vx ** 2 + vy ** 2 + vz ** 2)
        b = np.where(sp <= u, 1.0, u / np.maximum(sp, 1e-300))
        want = cfg["species"][s]["charge"] * r.weight(s) * b[x >= 0].sum()
        assert Q[s].sum() == pytest.approx(want, rel=1e-12)


def test_load2d_positions_and_draws():
    cfg = _cfg(ppc=50, nx=8)
    ny = 4
    r = oracle.Run2D(cfg, ny, load=False)
    lib_pts = np.array([oracle.load_particle2d(cfg, ny, 0, i) for i in range(cfg["nx"] * ny * 50)])
    assert lib_pts[:, 0].min() >= 0 and lib_pts[:, 0].max() < cfg["nx"]
    assert lib_pts[:, 1].min() >= 0 and lib_pts[:, 1].max() < ny
    # uniform in the box: cell counts within 5 sigma of ppc
    cnt = np.histogram2d(lib_pts[:, 0], lib_pts[:, 1], bins=(cfg["nx"], ny),
                         range=((0, cfg["nx"]), (0, ny)))[0]
    assert np.abs(cnt - 50).max() < 5 * math.sqrt(50)
    # isotropic velocities: the mean of each component is ~0, the variances agree
    v = lib_pts[:, 2:]
    sd = v.std(axis=0)
    assert np.abs(v.mean(axis=0)).max() < 5 * sd.max() / math.sqrt(len(v))
    assert sd.max() / sd.min() < 1.1
    del r


def test_sort2d_is_numpys_stable_sort_by_tile_key():
    cfg = _cfg(ppc=6, nx=10, sort_every=0)
    ny, tile = 6, 4
    r = oracle.Run2D(cfg, ny, tile=tile)
    x0 = [r.particles(s) for s in range(2)]
    perms = r.sort()
    nty = math.ceil(ny / tile)
    for s in range(2):
        x, y = x0[s][0], x0[s][1]
        key = np.where(x >= 0, (np.floor(x) // tile) * nty + np.floor(y) // tile, -1).astype(np.int64)
        live = np.nonzero(key >= 0)[0]
        want = live[np.argsort(key[live], kind="stable")]
        assert np.array_equal(perms[s], want)
        xs = r.particles(s)
        assert np.array_equal(xs[0], x[want]) and np.array_equal(xs[1], y[want])
        for i in range(0, len(x), 17):
            assert oracle.sort_key2d(ny, tile, x[i], y[i]) == key[i]


def test_free_streaming_wrap_and_reflection():
    # equal weights and opposite charges at one point: the net charge is
    # zero at every node, E = 0, and each particle streams at beta v
    cfg = _cfg(u_over_vti=3.0, ppc=4, sort_every=0)
    cfg["species"][1]["temperature"] = cfg["species"][0]["temperature"]
    cfg["species"][1]["mass"] = 1.0
    nx, ny = cfg["nx"], 5
    r = oracle.Run2D(cfg, ny, load=False)
    assert r.weight(0) == r.weight(1)
    u, dtdx = cfg["u"], cfg["dt"] / cfg["dx"]
    x = np.array([3.5, 0.2, 4.0, 6.9])
    y = np.array([4.9, 2.0, 0.1, 1.0])
    vx = np.array([0.5 * u / dtdx, -0.8 * u, 0.1 * u, 0.3 * u])
    vy = np.array([0.6 * u, 0.2 * u, -0.9 * u, 0.0])
    vz = np.array([0.0, 0.1 * u, 0.0, 40 * u])
    for s in range(2):
        r.set_particles(s, x, y, vx, vy, vz)
    r.refresh_fields()
    g = r.grid()
    assert np.abs(g["Ex"]).max() == 0.0 and np.abs(g["Ey"]).max() == 0.0
    r.step(1)
    sp = np.sqrt(vx ** 2 + vy ** 2 + vz ** 2)
    b = np.where(sp <= u, 1.0, u / sp)
    xn = x + b * vx * dtdx
    yn = np.mod(y + b * vy * dtdx, ny)
    vxn = np.where(xn < 0, -vx, vx)
    xn = np.abs(xn)
    X, Y, VX, VY, VZ = r.particles(0)
    assert np.allclose(X, xn, rtol=0, atol=1e-13) and np.allclose(Y, yn, rtol=0, atol=1e-13)
    assert np.array_equal(VX, vxn) and np.array_equal(VY, vy) and np.array_equal(VZ, vz)
    assert Y.min() >= 0 and Y.max() < ny


def test_y_uniform_2d_run_reduces_to_1d():
    # every 1D particle copied onto each of the ny rows (same y fraction, vy
    # kept): the 2D charge is y-uniform, Ey vanishes and x, vx, phi follow
    # the 1D run step by step (ions are kept 4 cells from the wall, so none
    # is absorbed in 3 steps of at most one cell and nothing is injected)
    cfg = workloads.sheath(nx=16, ppc=20, u_over_vti=3.0, seed=11, sort_every=0, steady_window=1)
    ny = 4
    r1 = oracle.Run(cfg)
    x, vx, vy, vz = r1.particles(1)
    keep = x < cfg["nx"] - 4
    r1.set_particles(1, x[keep], vx[keep], vy[keep], vz[keep])
    r1.refresh_fields()
    r2 = oracle.Run2D(cfg, ny, load=False)
    for s in range(2):
        x, vx, vy, vz = r1.particles(s)
        n = len(x)
        X = np.tile(x, ny)
        Y = np.repeat(np.arange(ny), n) + 0.25
        r2.set_particles(s, X, Y, np.tile(vx, ny), np.tile(vy, ny), np.tile(vz, ny))
    r2.refresh_fields()
    for it in range(3):
        g1, g2 = r1.grid(), r2.grid()
        assert np.abs(g2["phi"] - g1["phi"][:, None]).max() < 1e-10 * np.abs(g1["phi"]).max()
        assert np.abs(g2["Ey"]).max() < 1e-10 * np.abs(g1["E"]).max()
        r1.step(1)
        r2.step(1)
        assert r1.injected_total(1) == 0
        for s in range(2):
            x1, vx1, _, _ = r1.particles(s)
            X, Y, VX, VY, VZ = r2.particles(s)
            n = len(x1)
            for j in range(ny):
                assert np.abs(X[j * n:(j + 1) * n] - x1).max() < 1e-9
                assert np.abs(VX[j * n:(j + 1) * n] - vx1).max() < 1e-9 * max(1e-300, np.abs(vx1).max())
    # the y-mean of the 2D moments is the 1D moments (the 2D weight is dy
    # times the 1D one and each 1D particle has ny copies), and both steady
    # detectors saw the same Phi_w after every step
    m1, m2 = r1.moments(), r2.moments().mean(axis=2)
    for row in range(7):
        assert np.abs(m2[row] - m1[row]).max() <= 1e-10 * max(1e-300, np.abs(m1[row]).max()), row
    d1, d2 = r1.steady(), r2.steady()  # one-step windows: the last three Phi_w
    assert d2["windows"] == d1["windows"] == 3
    assert d2["window_mean"] == pytest.approx(d1["window_mean"], rel=1e-10)


def test_moments2d_by_hand():
    """Moments of a few particles written out with bilinear weights, the y
    wrap and the node volumes (half at the x end nodes)."""
    cfg = workloads.sheath(nx=6, ppc=2, u_over_vti=3.0, seed=13, sort_every=0)
    ny = 4
    r = oracle.Run2D(cfg, ny, load=False)
    rng = np.random.default_rng(5)
    parts = []
    for s in range(2):
        n = 7
        X = rng.uniform(0, cfg["nx"], n)
        Y = rng.uniform(0, ny, n)
        Y[0] = ny - 0.3  # a particle across the y wrap
        X[1] = 0.2       # near the symmetry plane
        vth = oracle.thermal_speed(cfg, s)
        VX, VY, VZ = (rng.normal(size=n) * vth * 4 for _ in range(3))
        r.set_particles(s, X, Y, VX, VY, VZ)
        parts.append((X, Y, VX, VY, VZ))
    r.refresh_fields()
    m = r.moments()
    u = cfg["u"]
    dx = cfg["dx"]
    assert np.array_equal(m[0], r.grid()["phi"])
    for s in range(2):
        X, Y, VX, VY, VZ = parts[s]
        w = r.weight(s)
        mass = cfg["species"][s]["mass"]
        want = np.zeros((3, cfg["nx"] + 1, ny))
        for i in range(len(X)):
            v2 = VX[i] ** 2 + VY[i] ** 2 + VZ[i] ** 2
            b = min(1.0, u / math.sqrt(v2))
            cx, cy = int(X[i]), int(Y[i])
            fx, fy = X[i] - cx, Y[i] - cy
            for (ix, iy, wt) in ((cx, cy, (1 - fx) * (1 - fy)), (cx + 1, cy, fx * (1 - fy)),
                                 (cx, (cy + 1) % ny, (1 - fx) * fy), (cx + 1, (cy + 1) % ny, fx * fy)):
                for row, q in enumerate((1.0, VX[i], 0.5 * mass * v2)):
                    want[row, ix, iy] += w * b * wt * q
        dV = np.full(cfg["nx"] + 1, dx * dx)
        dV[0] *= 0.5
        dV[-1] *= 0.5
        want /= dV[None, :, None]
        got = m[1 + 3 * s: 4 + 3 * s]
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), s


def test_source2d_balances_ion_loss():
    cfg = workloads.sheath(nx=8, ppc=10, u_over_vti=3.0, dt=200.0, seed=2)
    r = oracle.Run2D(cfg, 4)
    n0 = [r.nslots(s) for s in range(2)]
    r.step(30)
    x, y, *_ = r.particles(1)
    live1 = int((x >= 0).sum())
    # ions: every absorbed ion is replaced by one injected in the source cells
    assert live1 == n0[1]
    k = oracle.inject_particle2d(cfg, 4, 1, 0, 5)
    assert 0 <= k[0] < cfg["source_cells"] and 0 <= k[1] < 4


def test_step2d_is_gather_then_exact_kick_then_beta_drift():
    # one step recomputed particle by particle from pinned pieces: bilinear
    # E from the node fields, the exact velocity map of Eq. (A2a) with
    # a = (q/m)(Ex, Ey, 0), then x += beta vx dt/dx, y += beta vy dt/dy mod ny
    cfg = workloads.sheath(nx=12, ppc=6, u_over_vti=3.0, seed=4, sort_every=0)
    ny = 6
    r = oracle.Run2D(cfg, ny)
    g = r.grid()
    before = [r.particles(s) for s in range(2)]
    r.step(1)
    u, dtdx = cfg["u"], cfg["dt"] / cfg["dx"]
    checked = 0
    for s in range(2):
        qm = cfg["species"][s]["charge"] / cfg["species"][s]["mass"]
        X0, Y0, VX0, VY0, VZ0 = before[s]
        X, Y, VX, VY, VZ = r.particles(s)
        for i in range(0, len(X0), 3):
            cx, cy = int(X0[i]), int(Y0[i])
            fx, fy = X0[i] - cx, Y0[i] - cy
            c1 = (cy + 1) % ny
            w = [((cx, cy), (1 - fx) * (1 - fy)), ((cx + 1, cy), fx * (1 - fy)),
                 ((cx, c1), (1 - fx) * fy), ((cx + 1, c1), fx * fy)]
            ex = sum(g["Ex"][n] * wt for n, wt in w)
            ey = sum(g["Ey"][n] * wt for n, wt in w)
            v1 = oracle.kick_exact("step", u, cfg["dt"], [VX0[i], VY0[i], VZ0[i]], [qm * ex, qm * ey, 0.0])
            sp = math.sqrt(v1 @ v1)
            b = 1.0 if sp <= u else u / sp
            xn = X0[i] + b * v1[0] * dtdx
            yn = (Y0[i] + b * v1[1] * dtdx) % ny
            if xn < 0:
                xn, v1[0] = -xn, -v1[0]
            if xn >= cfg["nx"]:
                assert X[i] == -1.0
                continue
            assert abs(X[i] - xn) < 1e-12 and abs(Y[i] - yn) < 1e-12
            assert np.abs(np.array([VX[i], VY[i], VZ[i]]) - v1).max() <= 1e-15 * max(1.0, np.abs(v1).max())
            checked += 1
    assert checked > 250
    assert np.abs(g["Ey"]).max() > 0.01 * np.abs(g["Ex"]).max()  # the y field takes part

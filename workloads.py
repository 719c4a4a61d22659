"""Seeded synthetic workloads for the SLPIC sheath (parameters only).

This module holds the problem definitions that both the CPU oracle and the
HIP path are run on: grid sizes, species, temperatures, speed limits, time
steps and seeds.  It contains none of the method's arithmetic (no push, no
deposit, no field solve, no sampling); the random numbers the method draws
come from the Philox generator each side implements from its published
definition, keyed by the ``seed`` here.

Normalised units: x in electron Debye lengths, t in 1/omega_pe, v in the
electron thermal speed sqrt(T_e/m_e), energies in T_e; e = m_e = eps0 = 1.
"""
from __future__ import annotations

import math

import numpy as np

AMU_IN_ME = 1822.888486  # atomic mass unit in electron masses


def species(te_over_ti: float, ion_amu: float, ppc: int):
    """Electrons (species 0) and singly charged ions (species 1)."""
    return [
        {"charge": -1.0, "mass": 1.0, "temperature": 1.0, "ppc": int(ppc)},
        {"charge": 1.0, "mass": ion_amu * AMU_IN_ME, "temperature": 1.0 / te_over_ti,
         "ppc": int(ppc)},
    ]


def ion_thermal_speed(te_over_ti: float, ion_amu: float) -> float:
    return math.sqrt((1.0 / te_over_ti) / (ion_amu * AMU_IN_ME))


def sheath(nx: int, ppc: int, u_over_vti: float, dt: float | None = None, te_over_ti: float = 20.0,
           ion_amu: float = 40.0, dx: float = 0.5, seed: int = 0, run: int = 0,
           beta_kind: str = "step", sort_every: int = 1, sort_bucket: int = 1,
           capacity_factor: float = 1.5, source_cells: int = 4, steady_window: int = 0,
           steady_tol: float = 0.0) -> dict:
    """A 1D3V sheath: symmetry plane at x = 0, grounded absorbing wall at
    x = nx*dx, thermal source in the first ``source_cells`` cells.

    Default time step: dt = min(dx/u, 1/omega_pi) for a finite speed limit
    (the paper's dt = dx/v0 capped so that unlimited ions keep
    omega_pi dt <= 1); dx/(5 v_te) for u = inf (the paper's PIC step)."""
    vti = ion_thermal_speed(te_over_ti, ion_amu)
    u = math.inf if math.isinf(u_over_vti) else u_over_vti * vti
    if dt is None:
        if math.isinf(u):
            dt = dx / 5.0
        else:
            inv_wpi = math.sqrt(ion_amu * AMU_IN_ME)
            dt = min(dx / u, inv_wpi)
    return {
        "nx": int(nx), "dx": float(dx), "dt": float(dt), "u": float(u), "beta_kind": beta_kind,
        "species": species(te_over_ti, ion_amu, ppc), "source_cells": int(source_cells),
        "seed": int(seed), "run": int(run), "sort_every": int(sort_every),
        "sort_bucket": int(sort_bucket), "capacity_factor": float(capacity_factor),
        "te_over_ti": float(te_over_ti), "ion_amu": float(ion_amu), "u_over_vti": float(u_over_vti),
        "steady_window": int(steady_window), "steady_tol": float(steady_tol),
    }


def small_sheath(seed: int = 0, **kw) -> dict:
    """64 cells over 32 Debye lengths, argon, Te = 1 eV, Ti = 0.05 eV,
    100 macroparticles per cell per species, u = 3 v_ti, dt = 5/omega_pe,
    1000 steps (FP64)."""
    kw.setdefault("ppc", 100)
    return sheath(nx=64, u_over_vti=3.0, dt=5.0, te_over_ti=20.0, ion_amu=40.0, seed=seed, **kw)


SMALL_SHEATH_STEPS = 1000


def production_sheath(u_over_vti: float = 2.0, ppc: int = 1000, seed: int = 0, **kw) -> dict:
    """2048 cells over 1024 Debye lengths, argon, Te = 1 eV, Ti = 0.05 eV,
    1000 macroparticles per cell per species (4,096,000 particles),
    u in {2, 5, 10, inf} v_ti, FP32 particles with FP64 grids."""
    return sheath(nx=2048, ppc=ppc, u_over_vti=u_over_vti, te_over_ti=20.0, ion_amu=40.0,
                  seed=seed, **kw)


PRODUCTION_U_SWEEP = (2.0, 5.0, 10.0, math.inf)


def sheath2d(nx: int = 512, ny: int = 512, ppc: int = 64, u_over_vti: float = 3.0, tile: int = 8,
             sort_every: int = 8, seed: int = 0, **kw) -> dict:
    """A 2D3V sheath: the 1D geometry in x (symmetry plane at x = 0, wall at
    x = nx*dx, source in the first cells), periodic in y over ny cells with
    dy = dx; argon, Te/Ti = 20, u = 3 v_ti, dt = dx/u.  The particles are
    cell-sorted by blocks of tile x tile cells every ``sort_every`` steps."""
    cfg = sheath(nx=nx, ppc=ppc, u_over_vti=u_over_vti, te_over_ti=20.0, ion_amu=40.0, seed=seed,
                 sort_every=sort_every, **kw)
    cfg["ny"] = int(ny)
    cfg["tile"] = int(tile)
    return cfg


PAPER_ION_MASS = 39.9 * 1836.0  # the paper's argon ion mass in electron masses
# 1 microsecond in 1/omega_pe at the paper's n0 = 5e13 m^-3 (omega_pe = 3.989e8 /s)
PAPER_OMEGA_PE_US = 398.9
PLATES_PAPER = {  # what the paper reports for its sheath experiment (Sec. IV)
    "t_steady_us": 24.0, "t_cross_us": 8.0, "pic_steps": 1.9e5, "slpic_steps": 600,
    "speedup": 160.0, "ions": 8.3e4, "electrons": 1.1e5,
}


def plates_sheath(v0_over_vte: float, ppc: int = 200, seed: int = 0, sort_every: int = 16,
                  capacity_factor: float = 2.0, beta_kind: str = "step") -> dict:
    """The paper's sheath experiment (Sec. IV), normalised to T_e = 2.2 eV,
    n0 = 5e13 m^-3 (lambda_D = 0.156 cm, v_te = 6.2e5 m/s): conducting
    plates 4 cm apart (25.65 lambda_D, 100 cells), phi(0) = 0, phi(L) = 12.5 V
    = 5.68 T_e/e, electrons and argon ions (m = 39.9 * 1836 m_e, T_i = 0.5 eV)
    injected through the plate at x = L as from a stationary plasma of density
    n0, both plates absorbing, the box empty at the start.  v0 = v0_over_vte
    * v_te with dt = dx/v0 (the paper: v0 = 9.8e3 m/s = 0.0158 v_te); v0 = inf
    is PIC with dt = dx/(5 v_te).  ppc: g-particles per cell at density n0
    (sets the weight)."""
    L = 4.0 / 0.15595  # plate gap in Debye lengths
    nx = 100
    dx = L / nx
    u = math.inf if math.isinf(v0_over_vte) else float(v0_over_vte)
    dt = dx / 5.0 if math.isinf(u) else dx / u
    ti = 0.5 / 2.2
    return {
        "nx": nx, "dx": dx, "dt": dt, "u": u, "beta_kind": beta_kind,
        "species": [{"charge": -1.0, "mass": 1.0, "temperature": 1.0, "ppc": int(ppc)},
                    {"charge": 1.0, "mass": PAPER_ION_MASS, "temperature": ti, "ppc": int(ppc)}],
        "source_cells": 4, "seed": int(seed), "run": 0, "sort_every": int(sort_every), "sort_bucket": 1,
        "capacity_factor": float(capacity_factor), "geometry": "plates", "bias": 12.5 / 2.2,
        "steady_window": 0, "steady_tol": 0.0,
    }


def plates_steps(cfg: dict, t_us: float) -> int:
    """Steps of the plates workload cfg covering t_us microseconds."""
    return int(round(t_us * PAPER_OMEGA_PE_US / cfg["dt"]))


def langmuir_box(u_over_vte: float, nx: int = 256, ppc: int = 1000, dx: float = 0.5, seed: int = 0,
                 beta_kind: str = "step", sort_every: int = 16) -> dict:
    """A uniform Maxwellian plasma in a periodic box (the plasma-oscillation
    section): nx cells of dx = 0.5 Debye lengths (k lambda_D = 2 pi/(nx dx) =
    0.049 at 256 cells for the fundamental mode), electrons at T_e = 1 and
    argon ions (40 amu, T_i = T_e/20) loaded uniformly, ppc g-particles per
    cell per species.  SLPIC at u = u_over_vte * v_te takes dt = dx/u (the
    paper's choice of step); u = inf (PIC) takes dt = dx/(5 v_te)."""
    u = math.inf if math.isinf(u_over_vte) else float(u_over_vte)
    dt = dx / 5.0 if math.isinf(u) else dx / u
    return {
        "nx": int(nx), "dx": float(dx), "dt": float(dt), "u": u, "beta_kind": beta_kind,
        "species": species(20.0, 40.0, ppc), "source_cells": 4, "seed": int(seed), "run": 0,
        "sort_every": int(sort_every), "sort_bucket": 1, "capacity_factor": 1.0, "geometry": "periodic",
        "bias": 0.0, "steady_window": 0, "steady_tol": 0.0,
    }


def langmuir_displacement(x: np.ndarray, nx: int, amplitude: float) -> np.ndarray:
    """The initial perturbation of the periodic box: positions (in cells)
    moved by xi = (amplitude nx / 2 pi) sin(2 pi x / nx), which leaves the
    density n0 (1 - amplitude cos(2 pi x / nx)) to first order and the field
    E(L/4) = amplitude L / (2 pi) (for electrons of charge -1); wrapped into
    [0, nx)."""
    xi = amplitude * nx / (2.0 * math.pi) * np.sin(2.0 * math.pi * x / nx)
    y = x + xi
    return np.mod(y, nx)


def fit_frequency(t: np.ndarray, y: np.ndarray, w_guess: float, periods: float = 12.0) -> float:
    """Angular frequency of an oscillating series: the w in [w_guess/2,
    3 w_guess/2] whose least-squares fit a cos(w t) + b sin(w t) explains the
    most of the first `periods` guessed periods (the periodogram peak on a
    grid of 4001 frequencies, refined by a parabola through the top three);
    unlike zero crossings it is not biased by noise near the zero line."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    keep = t - t[0] <= periods * 2.0 * math.pi / w_guess
    t, y = t[keep], y[keep]
    ws = np.linspace(0.5 * w_guess, 1.5 * w_guess, 4001)
    power = np.empty_like(ws)
    for i, w in enumerate(ws):
        A = np.stack([np.cos(w * t), np.sin(w * t)], axis=1)
        c, *_ = np.linalg.lstsq(A, y, rcond=None)
        power[i] = float(np.sum((A @ c) ** 2))
    i = int(np.clip(np.argmax(power), 1, len(ws) - 2))
    p0, p1, p2 = power[i - 1], power[i], power[i + 1]
    den = p0 - 2.0 * p1 + p2
    shift = 0.5 * (p0 - p2) / den if den != 0.0 else 0.0
    return float(ws[i] + shift * (ws[1] - ws[0]))


def zero_crossing_frequency(t: np.ndarray, y: np.ndarray) -> float:
    """Angular frequency of an oscillating series from its zero crossings
    (linear interpolation between samples): pi per half period."""
    s = np.sign(y)
    idx = np.nonzero(s[:-1] * s[1:] < 0)[0]
    if len(idx) < 3:
        return float("nan")
    tc = t[idx] - y[idx] * (t[idx + 1] - t[idx]) / (y[idx + 1] - y[idx])
    return math.pi * (len(tc) - 1) / (tc[-1] - tc[0])


def wave_test(v0_over_vphi: float, n: int = 100_000, seed: int = 0, cells: int = 100, periods_ramp: float = 20.0,
              phi_max: float = 0.1, beta_kind: str = "step"):
    """Test electrons in a prescribed traveling wave phi0(t) sin(k(x - v_phi t))
    with v_phi = v_te = 1 in a periodic box of `cells` cells (dx = 1, k = 2 pi
    / L), e phi_max / T_e = 0.1, phi0 ramped over 20 wave periods.  SLPIC
    with speed limit v0 = v0_over_vphi * v_phi takes dt = dx / v0; v0 = inf
    (PIC) takes dt = dx / (5 v_te).  Returns the wave description and the
    initial particles: x uniform in [0, L), v a 1V Maxwellian at T_e = 1
    (NumPy default_rng(seed))."""
    L = float(cells)
    u = math.inf if math.isinf(v0_over_vphi) else float(v0_over_vphi)
    dt = 1.0 / 5.0 if math.isinf(u) else 1.0 / u
    w = {"length": L, "v_phase": 1.0, "phi_max": phi_max, "ramp_time": periods_ramp * L, "qm": -1.0,
         "dt": dt, "u": u, "beta_kind": beta_kind}
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, L, size=n)
    v = rng.normal(0.0, 1.0, size=n)
    return w, x, v


def batched_sweep(nruns: int = 256, seed: int = 1, ppc_range=(200, 1000), cells_range=(128, 2048),
                  capacity_factor: float = 2.5, **kw) -> list[dict]:
    """Independent 1D sheaths: cells uniform in [128, 2048], ppc uniform in
    [200, 1000], Te/Ti log-uniform in [5, 100], ion mass in {4, 20, 40, 84}
    amu, u uniform in [2, 10] v_ti; dx = 0.5 so L/lambda_D = cells/2.  Slots
    per species are 2.5x the load: small runs lose most of their ions within
    a few hundred steps, and between two sorts the holes stay occupied while
    the source appends."""
    rng = np.random.default_rng(seed)
    runs = []
    for r in range(nruns):
        nx = int(rng.integers(cells_range[0], cells_range[1] + 1))
        ppc = int(rng.integers(ppc_range[0], ppc_range[1] + 1))
        te_ti = float(math.exp(rng.uniform(math.log(5.0), math.log(100.0))))
        amu = float(rng.choice([4.0, 20.0, 40.0, 84.0]))
        k = float(rng.uniform(2.0, 10.0))
        runs.append(sheath(nx=nx, ppc=ppc, u_over_vti=k, te_over_ti=te_ti, ion_amu=amu,
                           seed=seed * 100003 + r, run=r, capacity_factor=capacity_factor, **kw))
    return runs


def features(cfg: dict) -> np.ndarray:
    """Warm-start network inputs: (ln Te/Ti, ln A, u/v_ti, ln L/lambda_D)."""
    return np.array([math.log(cfg["te_over_ti"]), math.log(cfg["ion_amu"]), cfg["u_over_vti"],
                     math.log(cfg["nx"] * cfg["dx"])], dtype=np.float64)

"""FP64 CPU oracle for speed-limited PIC (SLPIC) -- TEST INFRASTRUCTURE ONLY.

This package is the plain reference that the HIP path is checked against.
Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the product package never does.  It shares no
code with the HIP library: the C source ``slpic_oracle.c`` is compiled on its
own with gcc (``-O2 -ffp-contract=off``) and loaded here with ctypes.

Paper: Werner, Jenkins, Chap & Cary, arXiv:1511.08225 -- Eq. (10), (11a,b),
Appendix Eq. (A1), (A2).  See ``slpic_oracle.c`` for the readings taken where
the paper is silent.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slpic_oracle.c")
_LIB = os.path.join(_HERE, "libslpic_oracle.so")

BETA_STEP, BETA_SMOOTH = 0, 1
GEOM_SHEATH, GEOM_PLATES, GEOM_PERIODIC = 0, 1, 2
KICK_EXACT, KICK_MMP = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Species(ctypes.Structure):
    _fields_ = [("charge", ctypes.c_double), ("mass", ctypes.c_double),
                ("temperature", ctypes.c_double), ("ppc", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("beta_kind", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dt", ctypes.c_double), ("u", ctypes.c_double),
                ("nspecies", ctypes.c_int32), ("source_cells", ctypes.c_int32),
                ("species", _Species * 2), ("seed", ctypes.c_uint64), ("run", ctypes.c_int32),
                ("sort_every", ctypes.c_int32), ("sort_bucket", ctypes.c_int32),
                ("kick", ctypes.c_int32), ("mmp_tol", ctypes.c_double),
                ("capacity_factor", ctypes.c_double), ("steady_window", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("steady_tol", ctypes.c_double), ("geometry", ctypes.c_int32),
                ("pad2", ctypes.c_int32), ("bias", ctypes.c_double),
                ("limit", ctypes.POINTER(ctypes.c_double))]


class _Steady(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int32), ("nopen", ctypes.c_int32), ("tol", ctypes.c_double),
                ("sum", ctypes.c_double), ("mean", ctypes.c_double * 3), ("nwin", ctypes.c_int64),
                ("steady_step", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {"window": self.window, "steady_step": self.steady_step, "windows": self.nwin,
                "window_mean": list(self.mean)}


class _Wave(ctypes.Structure):
    _fields_ = [("length", ctypes.c_double), ("v_phase", ctypes.c_double), ("phi_max", ctypes.c_double),
                ("ramp_time", ctypes.c_double), ("qm", ctypes.c_double), ("dt", ctypes.c_double),
                ("u", ctypes.c_double), ("beta_kind", ctypes.c_int32), ("pad", ctypes.c_int32)]


def make_wave(w: dict) -> _Wave:
    c = _Wave()
    for k in ("length", "v_phase", "phi_max", "ramp_time", "qm", "dt", "u"):
        setattr(c, k, float(w[k]))
    c.beta_kind = _beta_kind(w.get("beta_kind", "step"))
    return c


def wave_push(w: dict, x, v, step0: int, nsteps: int):
    """Advance test particles (arrays updated and returned as copies) through
    the prescribed traveling wave for nsteps steps starting at step step0."""
    x = np.array(x, dtype=np.float64, copy=True)
    v = np.array(v, dtype=np.float64, copy=True)
    c = make_wave(w)
    lib().orc_wave_push(ctypes.byref(c), _dp(x), _dp(v), len(x), int(step0), int(nsteps))
    return x, v


def wave_accel(w: dict, x: float, t: float) -> float:
    c = make_wave(w)
    return lib().orc_wave_accel(ctypes.byref(c), float(x), float(t))


_lib = None

_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PU32 = ctypes.POINTER(ctypes.c_uint32)
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_VP = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        sig = {
            "orc_philox4x32_10": (None, [_PU32, _PU32, _PU32]),
            "orc_u53": (_D, [ctypes.c_uint32, ctypes.c_uint32]),
            "orc_beta": (_D, [_I32, _D, _D]),
            "orc_G": (_D, [_D, _D]),
            "orc_fast_advance": (_D, [_D, _D, _D]),
            "orc_kick_exact": (None, [_I32, _D, _D, _PD, _PD, _PD]),
            "orc_kick_mmp": (_I32, [_I32, _D, _D, _PD, _PD, _D, _I32, _PD]),
            "orc_Z": (_D, [_I32, _D]),
            "orc_weight": (_D, [ctypes.POINTER(_Config), _I32]),
            "orc_load_particle": (None, [ctypes.POINTER(_Config), _I32, ctypes.c_uint32, _PD]),
            "orc_inject_particle": (None, [ctypes.POINTER(_Config), _I32, ctypes.c_uint32,
                                           ctypes.c_uint32, _PD]),
            "orc_poisson1d": (None, [_I32, _D, _PD, _PD, _PD]),
            "orc_poisson1d_plates": (None, [_I32, _D, _PD, _D, _PD, _PD]),
            "orc_wall_inject_particle": (None, [ctypes.POINTER(_Config), _I32, ctypes.c_uint32, ctypes.c_uint32,
                                                _PD]),
            "orc_wall_flux_per_step": (_D, [ctypes.POINTER(_Config), _I32]),
            "orc_poisson1d_periodic": (None, [_I32, _D, _PD, _PD, _PD]),
            "orc_wrap_periodic": (_D, [_D, _I32]),
            "orc_slpic_plasma_freq2": (_D, [_I32, _D, _D]),
            "orc_slpic_dispersion": (_D, [_I32, _D, _D, _D]),
            "orc_create": (_VP, [ctypes.POINTER(_Config)]),
            "orc_destroy": (None, [_VP]),
            "orc_load": (None, [_VP]),
            "orc_refresh_fields": (None, [_VP]),
            "orc_step": (None, [_VP, _I32]),
            "orc_sort": (None, [_VP, _PI32, _PI32]),
            "orc_keys": (None, [_VP, _I32, _PI32]),
            "orc_moments": (None, [_VP, _PD]),
            "orc_nslots": (_I64, [_VP, _I32]),
            "orc_capacity": (_I64, [_VP, _I32]),
            "orc_nlive": (_I64, [_VP, _I32]),
            "orc_step_index": (_I64, [_VP]),
            "orc_acc_e": (_D, [_VP]),
            "orc_acc_flux": (_D, [_VP, _I32]),
            "orc_monitor": (_D, [_VP]),
            "orc_set_speed_limit": (ctypes.c_int, [_VP, _D, _D]),
            "orc_run_weight": (_D, [_VP, _I32]),
            "orc_absorbed_total": (_I64, [_VP, _I32]),
            "orc_injected_total": (_I64, [_VP, _I32]),
            "orc_get_particles": (None, [_VP, _I32, _PD, _PD, _PD, _PD]),
            "orc_set_particles": (_I32, [_VP, _I32, _I64, _PD, _PD, _PD, _PD]),
            "orc_set_counters": (None, [_VP, _I64, _D]),
            "orc_get_grid": (None, [_VP, _PD, _PD, _PD, _PD]),
            "orc_get_steady": (None, [_VP, ctypes.POINTER(_Steady)]),
            "orc_load_warm": (ctypes.c_int, [_VP, _PD]),
            "orc_warm_cell_count": (_I64, [ctypes.POINTER(_Config), ctypes.c_int, _PD, ctypes.c_int32, _D, _PD, _PD]),
            "orc_warm_cell_vt": (_D, [ctypes.POINTER(_Config), ctypes.c_int, _PD, ctypes.c_int32]),
            "orc_warm_particle": (None, [ctypes.POINTER(_Config), ctypes.c_int, ctypes.c_uint32, ctypes.c_int32, _D,
                                         _D, _PD]),
            "orc_steady_init": (None, [ctypes.POINTER(_Steady), ctypes.c_int32, _D]),
            "orc_steady_feed": (None, [ctypes.POINTER(_Steady), _D, _I64]),
            "orc_wave_phi0": (_D, [ctypes.POINTER(_Wave), _D]),
            "orc_wave_accel": (_D, [ctypes.POINTER(_Wave), _D, _D]),
            "orc_wave_push": (None, [ctypes.POINTER(_Wave), _PD, _PD, _I64, _I64, _I32]),
            "orc2_create": (_VP, [ctypes.POINTER(_Config), _I32, _I32]),
            "orc2_get_steady": (None, [_VP, ctypes.POINTER(_Steady)]),
            "orc2_moments": (None, [_VP, _PD]),
            "orc2_destroy": (None, [_VP]),
            "orc2_load": (None, [_VP]),
            "orc2_step": (None, [_VP, _I32]),
            "orc2_sort": (None, [_VP, _PI32, _PI32]),
            "orc2_refresh_fields": (None, [_VP]),
            "orc2_poisson": (None, [_I32, _I32, _D, _PD, _PD, _PD, _PD]),
            "orc2_load_particle": (None, [ctypes.POINTER(_Config), _I32, _I32, ctypes.c_uint32, _PD]),
            "orc2_inject_particle": (None, [ctypes.POINTER(_Config), _I32, _I32, ctypes.c_uint32,
                                            ctypes.c_uint32, _PD]),
            "orc2_sort_key": (_I64, [_I32, _I32, _D, _D]),
            "orc2_nslots": (_I64, [_VP, _I32]),
            "orc2_step_index": (_I64, [_VP]),
            "orc2_acc_e": (_D, [_VP]),
            "orc2_weight": (_D, [_VP, _I32]),
            "orc2_get_particles": (None, [_VP, _I32, _PD, _PD, _PD, _PD, _PD]),
            "orc2_set_particles": (None, [_VP, _I32, _I64, _PD, _PD, _PD, _PD, _PD]),
            "orc2_set_counters": (None, [_VP, _I64, _D]),
            "orc2_get_grid": (None, [_VP, _PD, _PD, _PD, _PD, _PD]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_PD)


def _beta_kind(v) -> int:
    if isinstance(v, str):
        return {"step": BETA_STEP, "smooth": BETA_SMOOTH}[v]
    return int(v)


def make_config(cfg: dict) -> _Config:
    """Translate a workload dict (see workloads.py) into the oracle's struct."""
    c = _Config()
    c.nx = int(cfg["nx"])
    c.beta_kind = _beta_kind(cfg.get("beta_kind", "step"))
    c.dx = float(cfg["dx"])
    c.dt = float(cfg["dt"])
    c.u = float(cfg["u"])
    sp = cfg["species"]
    c.nspecies = len(sp)
    for k, s in enumerate(sp):
        c.species[k].charge = float(s["charge"])
        c.species[k].mass = float(s["mass"])
        c.species[k].temperature = float(s["temperature"])
        c.species[k].ppc = int(s["ppc"])
    c.source_cells = int(cfg.get("source_cells", 4))
    c.seed = int(cfg.get("seed", 0))
    c.run = int(cfg.get("run", 0))
    c.sort_every = int(cfg.get("sort_every", 1))
    c.sort_bucket = int(cfg.get("sort_bucket", 1))
    c.kick = {"exact": KICK_EXACT, "mmp": KICK_MMP}[cfg.get("kick", "exact")]
    c.mmp_tol = float(cfg.get("mmp_tol", 0.01))
    c.capacity_factor = float(cfg.get("capacity_factor", 1.5))
    c.steady_window = int(cfg.get("steady_window", 0))
    c.steady_tol = float(cfg.get("steady_tol", 0.0))
    c.geometry = {"sheath": GEOM_SHEATH, "plates": GEOM_PLATES, "periodic": GEOM_PERIODIC}[cfg.get("geometry", "sheath")]
    c.bias = float(cfg.get("bias", 0.0))
    prof = cfg.get("limit_profile")
    if prof is not None:  # nx + 1 node values of a speed limit varying with position
        a = np.ascontiguousarray(np.asarray(prof, dtype=np.float64).reshape(-1))
        if a.size != c.nx + 1:
            raise ValueError("limit_profile needs nx + 1 node values")
        c._limit = a  # kept alive with the struct
        c.limit = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return c


def steady_detect(series, window: int, tol: float) -> dict:
    """Run the wall-potential steady detector over a series (element k is
    Phi_w after step k + 1)."""
    d = _Steady()
    lib().orc_steady_init(ctypes.byref(d), int(window), float(tol))
    for k, v in enumerate(series):
        lib().orc_steady_feed(ctypes.byref(d), float(v), k + 1)
    return d.as_dict()


WARM_ROWS = 7  # phi, n_e, n_i, Gamma_e, Gamma_i, T_e, T_i


def warm_profile(profile) -> np.ndarray:
    """A (7, 256) contiguous warm-load profile; a (5, 256) one (no temperature
    rows) gets zero temperature rows, which stand for the source temperatures."""
    p = np.asarray(profile, dtype=np.float64)
    if p.size == 5 * 256:
        p = np.vstack([p.reshape(5, 256), np.zeros((2, 256))])
    return np.ascontiguousarray(p.reshape(WARM_ROWS, 256))


def warm_cell_count(cfg: dict, s: int, profile, c: int, w: float):
    """(g-particle count, drift V, thermal speed vt) of cell c, species s, of a warm load."""
    prof = warm_profile(profile)
    V, vt = ctypes.c_double(0.0), ctypes.c_double(0.0)
    c_ = make_config(cfg)
    n = lib().orc_warm_cell_count(ctypes.byref(c_), int(s), _dp(prof), int(c), float(w), ctypes.byref(V),
                                  ctypes.byref(vt))
    return int(n), V.value, vt.value


def warm_particle(cfg: dict, s: int, i: int, c: int, V: float, vt: float):
    out = (ctypes.c_double * 4)()
    c_ = make_config(cfg)
    lib().orc_warm_particle(ctypes.byref(c_), int(s), int(i) & 0xffffffff, int(c), float(V), float(vt), out)
    return list(out)


# ---------------------------------------------------------------- primitives
def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xffffffff for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xffffffff for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def u53(a: int, b: int) -> float:
    return lib().orc_u53(a & 0xffffffff, b & 0xffffffff)


def beta(kind, u: float, speed: float) -> float:
    return lib().orc_beta(_beta_kind(kind), u, speed)


def G(c2: float, p: float) -> float:
    return lib().orc_G(c2, p)


def fast_advance(c2: float, p0: float, K: float) -> float:
    return lib().orc_fast_advance(c2, p0, K)


def kick_exact(kind, u: float, dt: float, v, a) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_kick_exact(_beta_kind(kind), u, dt, _dp(v), _dp(a), _dp(out))
    return out


def kick_mmp(kind, u: float, dt: float, v, a, tol: float, nmax: int = 1 << 20):
    v = np.ascontiguousarray(v, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = np.zeros(3)
    n = lib().orc_kick_mmp(_beta_kind(kind), u, dt, _dp(v), _dp(a), tol, nmax, _dp(out))
    return out, n


def Z(kind, u_over_vt: float) -> float:
    return lib().orc_Z(_beta_kind(kind), u_over_vt)


def weight(cfg: dict, s: int) -> float:
    c = make_config(cfg)
    return lib().orc_weight(ctypes.byref(c), s)


def load_particle(cfg: dict, s: int, i: int) -> np.ndarray:
    c = make_config(cfg)
    out = np.zeros(4)
    lib().orc_load_particle(ctypes.byref(c), s, i, _dp(out))
    return out


def inject_particle(cfg: dict, s: int, k: int, step: int) -> np.ndarray:
    c = make_config(cfg)
    out = np.zeros(4)
    lib().orc_inject_particle(ctypes.byref(c), s, k, step, _dp(out))
    return out


def poisson1d(nx: int, dx: float, Q: np.ndarray):
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    assert Q.shape == (nx + 1,)
    phi = np.zeros(nx + 1)
    E = np.zeros(nx + 1)
    lib().orc_poisson1d(nx, dx, _dp(Q), _dp(phi), _dp(E))
    return phi, E


def poisson1d_plates(nx: int, dx: float, Q: np.ndarray, bias: float):
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    phi, E = np.zeros(nx + 1), np.zeros(nx + 1)
    lib().orc_poisson1d_plates(nx, dx, _dp(Q), float(bias), _dp(phi), _dp(E))
    return phi, E


def wall_inject_particle(cfg: dict, s: int, k: int, step: int) -> np.ndarray:
    c = make_config(cfg)
    out = np.zeros(4)
    lib().orc_wall_inject_particle(ctypes.byref(c), s, k, step, _dp(out))
    return out


def wall_flux_per_step(cfg: dict, s: int) -> float:
    c = make_config(cfg)
    return lib().orc_wall_flux_per_step(ctypes.byref(c), s)


def poisson1d_periodic(nx: int, dx: float, Q: np.ndarray):
    """Periodic box: node nx is the image of node 0 (its charge folds onto
    node 0), the mean charge is removed, gauge phi(0) = 0."""
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    phi, E = np.zeros(nx + 1), np.zeros(nx + 1)
    lib().orc_poisson1d_periodic(nx, dx, _dp(Q), _dp(phi), _dp(E))
    return phi, E


def wrap_periodic(xt: float, nx: int) -> float:
    return lib().orc_wrap_periodic(float(xt), int(nx))


def slpic_dispersion(kind, u: float, k: float, vt: float = 1.0) -> float:
    """The real frequency (omega_p = 1) of the mode k from the full
    dispersion relation of speed-limited particles (root above k u)."""
    kk = {"step": 0, "smooth": 1}[kind] if isinstance(kind, str) else int(kind)
    return lib().orc_slpic_dispersion(kk, float(u), float(vt), float(k))


def slpic_plasma_freq2(kind, u: float, vt: float = 1.0) -> float:
    """(omega_s/omega_p)^2 = <(beta v_x)^2>/v_t^2 over the 3D Maxwellian."""
    k = {"step": 0, "smooth": 1}[kind] if isinstance(kind, str) else int(kind)
    return lib().orc_slpic_plasma_freq2(k, float(u), float(vt))


# ----------------------------------------------------------------------- run
class Run:
    """One 1D3V SLPIC run on the CPU (FP64)."""

    def __init__(self, cfg: dict, load: bool = True, warm=None):
        """warm: optional (7, 256) profiles (phi, n_e, n_i, Gamma_e, Gamma_i,
        T_e, T_i on x/L = k/255; a (5, 256) one loads at the source
        temperatures) for a warm load instead of the cold one."""
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        self._h = lib().orc_create(ctypes.byref(self._c))
        if not self._h:
            raise ValueError("invalid run configuration")
        self.nx = self._c.nx
        self.nspecies = self._c.nspecies
        if warm is not None:
            prof = warm_profile(warm)
            lib().orc_load_warm(self._h, _dp(prof))
        elif load:
            lib().orc_load(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.orc_destroy(h)
            except Exception:  # interpreter teardown
                pass
            self._h = None

    # state ------------------------------------------------------------
    def step(self, n: int = 1):
        lib().orc_step(self._h, n)

    def refresh_fields(self):
        lib().orc_refresh_fields(self._h)

    def sort(self):
        perms = [np.zeros(max(1, self.nslots(s)), dtype=np.int32) for s in range(2)]
        n_before = [self.nslots(s) for s in range(2)]
        lib().orc_sort(self._h, perms[0].ctypes.data_as(_PI32), perms[1].ctypes.data_as(_PI32))
        return [perms[s][: self.nslots(s)] if n_before[s] else perms[s][:0] for s in range(2)]

    def keys(self, s: int) -> np.ndarray:
        k = np.zeros(max(1, self.nslots(s)), dtype=np.int32)
        lib().orc_keys(self._h, s, k.ctypes.data_as(_PI32))
        return k[: self.nslots(s)]

    def nslots(self, s: int) -> int:
        return lib().orc_nslots(self._h, s)

    def nlive(self, s: int) -> int:
        return lib().orc_nlive(self._h, s)

    @property
    def step_index(self) -> int:
        return lib().orc_step_index(self._h)

    @property
    def acc_e(self) -> float:
        return lib().orc_acc_e(self._h)

    def set_speed_limit(self, u: float, dt: float):
        """Raise the speed limit mid-run: resample the g-particles so that
        f = beta g is kept at the weight of a fresh load at u, set dt,
        recompute the fields."""
        if lib().orc_set_speed_limit(self._h, float(u), float(dt)) != 0:
            raise ValueError("the limit and dt must be positive; a run with a limit profile keeps it")
        self.cfg["u"], self.cfg["dt"] = float(u), float(dt)

    def weight(self, s: int) -> float:
        return lib().orc_run_weight(self._h, s)

    def monitor(self) -> float:
        """The monitored value: Phi_w (sheath), phi(L/2) (plates), the
        fundamental sine amplitude of E (periodic)."""
        return lib().orc_monitor(self._h)

    def acc_flux(self) -> list:
        """Plates: the fractional wall injection carried over, per species."""
        return [lib().orc_acc_flux(self._h, s) for s in range(2)]

    def absorbed_total(self, s: int) -> int:
        return lib().orc_absorbed_total(self._h, s)

    def injected_total(self, s: int) -> int:
        return lib().orc_injected_total(self._h, s)

    def particles(self, s: int):
        n = self.nslots(s)
        arrs = [np.zeros(max(1, n)) for _ in range(4)]
        lib().orc_get_particles(self._h, s, *[_dp(a) for a in arrs])
        return tuple(a[:n] for a in arrs)

    def set_particles(self, s: int, x, vx, vy, vz):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, vx, vy, vz)]
        n = len(arrs[0])
        lib().orc_set_particles(self._h, s, n, *[_dp(a) for a in arrs])

    def set_counters(self, step: int, acc_e: float):
        lib().orc_set_counters(self._h, step, acc_e)

    def grid(self):
        nodes = self.nx + 1
        Q0, Q1, phi, E = (np.zeros(nodes) for _ in range(4))
        lib().orc_get_grid(self._h, _dp(Q0), _dp(Q1), _dp(phi), _dp(E))
        return {"Q": np.stack([Q0, Q1]), "phi": phi, "E": E}

    def moments(self) -> np.ndarray:
        nodes = self.nx + 1
        out = np.zeros((1 + 3 * self.nspecies) * nodes)
        lib().orc_moments(self._h, _dp(out))
        return out.reshape(1 + 3 * self.nspecies, nodes)

    def wall_potential(self) -> float:
        g = self.grid()
        return float(g["phi"][0] - g["phi"][-1])

    def steady(self) -> dict:
        """The wall-potential steady detector of this run."""
        d = _Steady()
        lib().orc_get_steady(self._h, ctypes.byref(d))
        return d.as_dict()

    def weights(self):
        return [weight(self.cfg, s) for s in range(self.nspecies)]


# ------------------------------------------------------------------- 2D3V
def poisson2d(nx: int, ny: int, dx: float, Q: np.ndarray):
    """phi, Ex, Ey on the (nx+1, ny) nodes from the node charge Q (dy = dx)."""
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    assert Q.shape == (nx + 1, ny)
    phi, Ex, Ey = (np.zeros((nx + 1, ny)) for _ in range(3))
    lib().orc2_poisson(nx, ny, dx, _dp(Q), _dp(phi), _dp(Ex), _dp(Ey))
    return phi, Ex, Ey


def load_particle2d(cfg: dict, ny: int, s: int, i: int) -> np.ndarray:
    """(x, y, vx, vy, vz) of load slot i."""
    c = make_config(cfg)
    out = np.zeros(5)
    lib().orc2_load_particle(ctypes.byref(c), ny, s, i, _dp(out))
    return out


def inject_particle2d(cfg: dict, ny: int, s: int, k: int, step: int) -> np.ndarray:
    c = make_config(cfg)
    out = np.zeros(5)
    lib().orc2_inject_particle(ctypes.byref(c), ny, s, k, step, _dp(out))
    return out


def sort_key2d(ny: int, tile: int, x: float, y: float) -> int:
    return lib().orc2_sort_key(ny, tile, x, y)


class Run2D:
    """One 2D3V SLPIC run on the CPU (FP64): x as in 1D, y periodic in
    [0, ny) cells, dy = dx; nodes (i, j) at i*ny + j."""

    def __init__(self, cfg: dict, ny: int, tile: int = 1, load: bool = True):
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        self.nx, self.ny, self.tile = self._c.nx, int(ny), int(tile)
        self._h = lib().orc2_create(ctypes.byref(self._c), self.ny, self.tile)
        if not self._h:
            raise ValueError("invalid run configuration")
        if load:
            lib().orc2_load(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.orc2_destroy(h)
            except Exception:
                pass
            self._h = None

    def step(self, n: int = 1):
        lib().orc2_step(self._h, n)

    def refresh_fields(self):
        lib().orc2_refresh_fields(self._h)

    def sort(self):
        n_before = [self.nslots(s) for s in range(2)]
        perms = [np.zeros(max(1, n), dtype=np.int32) for n in n_before]
        lib().orc2_sort(self._h, perms[0].ctypes.data_as(_PI32), perms[1].ctypes.data_as(_PI32))
        return [perms[s][: self.nslots(s)] for s in range(2)]

    def nslots(self, s: int) -> int:
        return lib().orc2_nslots(self._h, s)

    @property
    def step_index(self) -> int:
        return lib().orc2_step_index(self._h)

    @property
    def acc_e(self) -> float:
        return lib().orc2_acc_e(self._h)

    def weight(self, s: int) -> float:
        return lib().orc2_weight(self._h, s)

    def particles(self, s: int):
        """(x, y, vx, vy, vz) in grid units / velocity units; dead slots x = -1."""
        n = self.nslots(s)
        arrs = [np.zeros(max(1, n)) for _ in range(5)]
        lib().orc2_get_particles(self._h, s, *[_dp(a) for a in arrs])
        return tuple(a[:n] for a in arrs)

    def set_particles(self, s: int, x, y, vx, vy, vz):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, vx, vy, vz)]
        lib().orc2_set_particles(self._h, s, len(arrs[0]), *[_dp(a) for a in arrs])

    def set_counters(self, step: int, acc_e: float):
        lib().orc2_set_counters(self._h, step, acc_e)

    def grid(self):
        shape = (self.nx + 1, self.ny)
        Q0, Q1, phi, Ex, Ey = (np.zeros(shape) for _ in range(5))
        lib().orc2_get_grid(self._h, *[_dp(a) for a in (Q0, Q1, phi, Ex, Ey)])
        return {"Q": np.stack([Q0, Q1]), "phi": phi, "Ex": Ex, "Ey": Ey}

    def wall_potential(self) -> float:
        """Phi_w: the y-mean of phi at x = 0 (phi = 0 at the wall)."""
        return float(self.grid()["phi"][0].mean())

    def steady(self) -> dict:
        """The wall-potential steady detector of this run."""
        d = _Steady()
        lib().orc2_get_steady(self._h, ctypes.byref(d))
        return d.as_dict()

    def moments(self) -> np.ndarray:
        """beta-weighted node moments, shape (7, nx + 1, ny): phi, then n,
        Gamma_x, kinetic energy density per species."""
        out = np.zeros(7 * (self.nx + 1) * self.ny)
        lib().orc2_moments(self._h, _dp(out))
        return out.reshape(7, self.nx + 1, self.ny)


def thermal_speed(cfg: dict, s: int) -> float:
    sp = cfg["species"][s]
    return math.sqrt(sp["temperature"] / sp["mass"])

"""ctypes binding of libslpic.so (include/slpic.h).

Argument marshalling only: every step of the SLPIC path runs in the HIP
library.  PyTorch supplies the device workspace (a uint8 tensor) and the
stream; nothing here computes the method.  Importing this module without the
built library raises, so a missing extension can never fall back silently.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libslpic.so")

SLPIC_F32, SLPIC_F64 = 0, 1
GEOM_SHEATH, GEOM_PLATES, GEOM_PERIODIC = 0, 1, 2
BETA_STEP, BETA_SMOOTH = 0, 1
FLAG_CAPACITY, FLAG_NUMERIC = 1, 2
PROFILE_CLASSES = ("push", "inject", "field", "sort")


class SlpicError(RuntimeError):
    pass


class _Species(ctypes.Structure):
    _fields_ = [("charge", ctypes.c_double), ("mass", ctypes.c_double),
                ("temperature", ctypes.c_double), ("ppc", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class RunConfig(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("beta_kind", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dt", ctypes.c_double), ("u", ctypes.c_double),
                ("nspecies", ctypes.c_int32), ("source_cells", ctypes.c_int32),
                ("species", _Species * 2), ("seed", ctypes.c_uint64), ("run_id", ctypes.c_int32),
                ("steady_window", ctypes.c_int32), ("capacity_factor", ctypes.c_double),
                ("steady_tol", ctypes.c_double), ("warm_profile", ctypes.c_void_p),
                ("geometry", ctypes.c_int32), ("reserved", ctypes.c_int32), ("bias", ctypes.c_double),
                ("limit_profile", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("sort_every", ctypes.c_int32),
                ("sort_bucket", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("block", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
                ("sort_tile", ctypes.c_int32), ("retire_steady", ctypes.c_int32),
                ("push_order", ctypes.c_int32), ("record_perm", ctypes.c_int32)]


class RunStatus(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("nslots", ctypes.c_int64 * 2),
                ("capacity", ctypes.c_int64 * 2), ("absorbed_total", ctypes.c_int64 * 2),
                ("injected_total", ctypes.c_int64 * 2), ("acc_e", ctypes.c_double),
                ("wall_potential", ctypes.c_double), ("error_flags", ctypes.c_int32),
                ("fixed_bits", ctypes.c_int32), ("weight", ctypes.c_double * 2),
                ("steady_step", ctypes.c_int64), ("windows", ctypes.c_int64),
                ("window_mean", ctypes.c_double * 3), ("moment_samples", ctypes.c_int64),
                ("acc_flux", ctypes.c_double * 2)]

    def as_dict(self) -> dict:
        return {"step": self.step, "nslots": list(self.nslots), "capacity": list(self.capacity),
                "absorbed_total": list(self.absorbed_total),
                "injected_total": list(self.injected_total), "acc_e": self.acc_e,
                "wall_potential": self.wall_potential, "error_flags": self.error_flags,
                "fixed_bits": self.fixed_bits, "weight": list(self.weight),
                "steady_step": self.steady_step, "windows": self.windows,
                "window_mean": list(self.window_mean), "moment_samples": self.moment_samples,
                "acc_flux": list(self.acc_flux)}


class WaveConfig(ctypes.Structure):
    _fields_ = [("length", ctypes.c_double), ("v_phase", ctypes.c_double), ("phi_max", ctypes.c_double),
                ("ramp_time", ctypes.c_double), ("qm", ctypes.c_double), ("dt", ctypes.c_double),
                ("u", ctypes.c_double), ("beta_kind", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Tuning2D(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("sort_every", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("margin", ctypes.c_int32), ("per_thread", ctypes.c_int32), ("tail_groups", ctypes.c_int32),
                ("sort_tile", ctypes.c_int32), ("graph_steps", ctypes.c_int32), ("record_perm", ctypes.c_int32)]


class Status2D(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("nslots", ctypes.c_int64 * 2), ("nsorted", ctypes.c_int64 * 2),
                ("capacity", ctypes.c_int64 * 2), ("absorbed_total", ctypes.c_int64 * 2),
                ("injected_total", ctypes.c_int64 * 2), ("pushed_total", ctypes.c_int64),
                ("acc_e", ctypes.c_double), ("wall_potential", ctypes.c_double),
                ("error_flags", ctypes.c_int32), ("fixed_bits", ctypes.c_int32), ("weight", ctypes.c_double * 2),
                ("steady_step", ctypes.c_int64), ("windows", ctypes.c_int64), ("window_mean", ctypes.c_double * 3)]

    def as_dict(self) -> dict:
        return {"step": self.step, "nslots": list(self.nslots), "nsorted": list(self.nsorted),
                "capacity": list(self.capacity), "absorbed_total": list(self.absorbed_total),
                "injected_total": list(self.injected_total), "pushed_total": self.pushed_total,
                "acc_e": self.acc_e, "wall_potential": self.wall_potential, "error_flags": self.error_flags,
                "fixed_bits": self.fixed_bits, "weight": list(self.weight), "steady_step": self.steady_step,
                "windows": self.windows, "window_mean": list(self.window_mean)}


_lib = None
_P = ctypes.c_void_p
_PD = ctypes.POINTER(ctypes.c_double)
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PI32 = ctypes.POINTER(ctypes.c_int32)


def lib():
    """Load libslpic.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SlpicError(f"{LIB_PATH} is missing: build it with paper_1511_08225_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        sig = {
            "slpic_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(RunConfig), i32, ctypes.POINTER(Tuning)]),
            "slpic_init": (ctypes.c_int, [ctypes.POINTER(RunConfig), i32, ctypes.POINTER(Tuning), _P,
                                          ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
            "slpic_step": (ctypes.c_int, [_P, i32, _P]),
            "slpic_moments": (ctypes.c_int, [_P, i32, _P, _P]),
            "slpic_moments_sample": (ctypes.c_int, [_P, i32, _P]),
            "slpic_wall_history": (ctypes.c_int, [_P, i32, _PD, _PI64]),
            "slpic_mlp_act_bytes": (ctypes.c_size_t, [i32]),
            "slpic_mlp_work_bytes": (ctypes.c_size_t, [i32]),
            "slpic_mlp_to_bf16": (ctypes.c_int, [_P, _P, _P]),
            "slpic_mlp_forward": (ctypes.c_int, [_P, _P, _P, i32, _P, _P]),
            "slpic_mlp_forward_noalloc": (ctypes.c_int, [_P, _P, _P, i32, _P]),
            "slpic_mlp_backward": (ctypes.c_int, [_P, _P, _P, _P, i32, _P, _P]),
            "slpic_mlp_mse": (ctypes.c_int, [_P, _P, _P, i64, _P, _P]),
            "slpic_mlp_adam": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_float, ctypes.c_float,
                                              ctypes.c_float, ctypes.c_float, i32, _P]),
            "slpic_moments_window": (ctypes.c_int, [_P, i32, _P, i32, _P]),
            "slpic_status_query": (ctypes.c_int, [_P, ctypes.POINTER(RunStatus), i32]),
            "slpic_export_particles": (ctypes.c_int, [_P, i32, i32, _PD, _PD, _PD, _PI64]),
            "slpic_import_particles": (ctypes.c_int, [_P, i32, i32, _PD, _PD, _PD, i64]),
            "slpic_set_counters": (ctypes.c_int, [_P, i32, i64, ctypes.c_double]),
            "slpic_set_flux_counters": (ctypes.c_int, [_P, i32, _PD]),
            "slpic_set_sampling": (ctypes.c_int, [_P, i32]),
            "slpic_set_speed_limit": (ctypes.c_int, [_P, i32, ctypes.c_double, ctypes.c_double, _P]),
            "slpic_prune_retired": (ctypes.c_int, [_P, _PI32, _P]),
            "slpic_refresh_fields": (ctypes.c_int, [_P, _P]),
            "slpic_export_grid": (ctypes.c_int, [_P, i32, _PD, _PD, _PD]),
            "slpic_sort_now": (ctypes.c_int, [_P, _P]),
            "slpic_export_perm": (ctypes.c_int, [_P, i32, i32, _PI32, _PI64]),
            "slpic_profile": (ctypes.c_int, [_P, i32]),
            "slpic_profile_read": (ctypes.c_int, [_P, _PD, _PI64]),
            "slpic_total_slots": (ctypes.c_int, [_P, _PI64]),
            "slpic_destroy": (None, [_P]),
            "slpic_wave_push": (ctypes.c_int, [i32, ctypes.POINTER(WaveConfig), _P, _P, i64, i64, i32, _P]),
            "slpic2d_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(RunConfig), i32,
                                                          ctypes.POINTER(Tuning2D)]),
            "slpic2d_init": (ctypes.c_int, [ctypes.POINTER(RunConfig), i32, ctypes.POINTER(Tuning2D), _P,
                                            ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
            "slpic2d_step": (ctypes.c_int, [_P, i32, _P]),
            "slpic2d_refresh_fields": (ctypes.c_int, [_P, _P]),
            "slpic2d_solve_charge": (ctypes.c_int, [_P, _P, _P]),
            "slpic2d_export_grid": (ctypes.c_int, [_P, _PD, _PD, _PD]),
            "slpic2d_export_particles": (ctypes.c_int, [_P, i32, _PD, _PD, _PD, _PD, _PD, _PI64]),
            "slpic2d_import_particles": (ctypes.c_int, [_P, i32, _PD, _PD, _PD, _PD, _PD, i64]),
            "slpic2d_set_counters": (ctypes.c_int, [_P, i64, ctypes.c_double]),
            "slpic2d_sort_now": (ctypes.c_int, [_P, _P]),
            "slpic2d_export_perm": (ctypes.c_int, [_P, i32, _PI32, _PI64]),
            "slpic2d_status_query": (ctypes.c_int, [_P, ctypes.POINTER(Status2D)]),
            "slpic2d_profile": (ctypes.c_int, [_P, i32]),
            "slpic2d_profile_read": (ctypes.c_int, [_P, _PD, _PI64]),
            "slpic2d_moments": (ctypes.c_int, [_P, _P, _P]),
            "slpic2d_wall_history": (ctypes.c_int, [_P, _PD, _PI64]),
            "slpic2d_destroy": (None, [_P]),
            "slpic_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise SlpicError(f"{what}: {lib().slpic_strerror(rc).decode()} ({rc})")


def _beta_kind(v) -> int:
    if isinstance(v, str):
        return {"step": BETA_STEP, "smooth": BETA_SMOOTH}[v]
    return int(v)


def run_config(cfg: dict) -> RunConfig:
    """Marshal a run description (nx, dx, dt, u, beta_kind, species,
    source_cells, seed, run, capacity_factor, geometry, bias, limit_profile)
    into the C struct (a limit profile's nx + 1 node values are kept alive
    with the struct)."""
    c = RunConfig()
    c.nx = int(cfg["nx"])
    c.beta_kind = _beta_kind(cfg.get("beta_kind", "step"))
    c.dx, c.dt, c.u = float(cfg["dx"]), float(cfg["dt"]), float(cfg["u"])
    sp = cfg["species"]
    c.nspecies = len(sp)
    for k, s in enumerate(sp):
        c.species[k].charge = float(s["charge"])
        c.species[k].mass = float(s["mass"])
        c.species[k].temperature = float(s["temperature"])
        c.species[k].ppc = int(s["ppc"])
    c.source_cells = int(cfg.get("source_cells", 4))
    c.seed = int(cfg.get("seed", 0))
    c.run_id = int(cfg.get("run", 0))
    c.capacity_factor = float(cfg.get("capacity_factor", 1.5))
    c.steady_window = int(cfg.get("steady_window", 0))
    c.steady_tol = float(cfg.get("steady_tol", 0.0))
    geom = cfg.get("geometry", "sheath")
    c.geometry = ({"sheath": GEOM_SHEATH, "plates": GEOM_PLATES, "periodic": GEOM_PERIODIC}[geom]
                  if isinstance(geom, str) else int(geom))
    c.bias = float(cfg.get("bias", 0.0))
    prof = cfg.get("limit_profile")
    if prof is not None:
        a = np.ascontiguousarray(np.asarray(prof, dtype=np.float64).reshape(-1))
        if a.size != c.nx + 1:
            raise SlpicError("limit_profile needs nx + 1 node values")
        c._limit = a
        c.limit_profile = a.ctypes.data
    return c


def tuning(precision="f32", sort_every=16, sort_bucket=1, chunk=0, block=0, graph_steps=0,
           sort_tile=0, retire_steady=False, push_order=0, record_perm=False) -> Tuning:
    t = Tuning()
    t.precision = {"f32": SLPIC_F32, "f64": SLPIC_F64}[precision] if isinstance(precision, str) else int(precision)
    t.sort_every, t.sort_bucket, t.chunk, t.block = int(sort_every), int(sort_bucket), int(chunk), int(block)
    t.graph_steps, t.sort_tile = int(graph_steps), int(sort_tile)
    t.retire_steady = int(bool(retire_steady))
    t.push_order = int(push_order)
    t.record_perm = int(bool(record_perm))
    return t


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_PD)


def wave_push(w: dict, x: torch.Tensor, v: torch.Tensor, step0: int, nsteps: int):
    """Advance test particles (device tensors, float32 or float64, updated in
    place) through the prescribed traveling wave described by `w` (length,
    v_phase, phi_max, ramp_time, qm, dt, u, beta_kind)."""
    if x.dtype != v.dtype or x.shape != v.shape or not x.is_contiguous() or not v.is_contiguous():
        raise SlpicError("x and v must be contiguous tensors of one shape and dtype")
    prec = {torch.float32: SLPIC_F32, torch.float64: SLPIC_F64}.get(x.dtype)
    if prec is None:
        raise SlpicError("x and v must be float32 or float64")
    c = WaveConfig()
    for k in ("length", "v_phase", "phi_max", "ramp_time", "qm", "dt", "u"):
        setattr(c, k, float(w[k]))
    c.beta_kind = _beta_kind(w.get("beta_kind", "step"))
    stream = _P(torch.cuda.current_stream(x.device).cuda_stream)
    _check(lib().slpic_wave_push(prec, ctypes.byref(c), _P(x.data_ptr()), _P(v.data_ptr()), x.numel(), int(step0),
                                 int(nsteps), stream), "slpic_wave_push")


class Sim:
    """One or more independent 1D3V sheaths advanced together on one GPU."""

    def __init__(self, configs, precision="f32", sort_every=16, sort_bucket=1, chunk=0, block=0,
                 graph_steps=0, sort_tile=0, device="cuda", warm=None, retire_steady=False, push_order=0,
                 record_perm=False):
        """warm: optional list (one entry per run) of None or a (7, 256)
        array of predicted profiles (phi, n_e, n_i, Gamma_e, Gamma_i, T_e,
        T_i on x/L = k/255; a (5, 256) array loads at the source
        temperatures) for a warm load instead of the cold one.
        record_perm: every sort also stores its permutation (for perm())."""
        if isinstance(configs, dict):
            configs = [configs]
        self.configs = [dict(c) for c in configs]
        self.nruns = len(self.configs)
        self.precision = precision
        structs = [run_config(c) for c in self.configs]
        # the limit profiles the copied structs point to, alive while the library reads them
        self._limits = [getattr(c, "_limit", None) for c in structs]
        self._cfg = (RunConfig * self.nruns)(*structs)
        self._warm = []  # host profiles, alive while the library reads them
        if warm is not None:
            if len(warm) != self.nruns:
                raise SlpicError("warm needs one entry per run")
            for r, prof in enumerate(warm):
                if prof is None:
                    continue
                a = np.asarray(prof, dtype=np.float64)
                if a.size == 5 * 256:  # no temperature rows: the source temperatures
                    a = np.vstack([a.reshape(5, 256), np.zeros((2, 256))])
                a = np.ascontiguousarray(a.reshape(7, 256))
                self._warm.append(a)
                self._cfg[r].warm_profile = a.ctypes.data
        self._tun = tuning(precision, sort_every, sort_bucket, chunk, block, graph_steps, sort_tile, retire_steady,
                           push_order, record_perm)
        L = lib()
        nbytes = L.slpic_workspace_bytes(self._cfg, self.nruns, ctypes.byref(self._tun))
        if nbytes == 0:
            raise SlpicError("invalid configuration")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.workspace_bytes = nbytes
        self._ctx = _P()
        _check(L.slpic_init(self._cfg, self.nruns, ctypes.byref(self._tun), _P(self._ws_ptr), nbytes,
                            self._stream(), ctypes.byref(self._ctx)), "slpic_init")

    def _stream(self):
        return _P(torch.cuda.current_stream(self.device).cuda_stream)

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            torch.cuda.synchronize(self.device)
            lib().slpic_destroy(self._ctx)
            self._ctx = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- stepping
    def step(self, n: int = 1):
        _check(lib().slpic_step(self._ctx, int(n), self._stream()), "slpic_step")

    def refresh_fields(self):
        _check(lib().slpic_refresh_fields(self._ctx, self._stream()), "slpic_refresh_fields")

    def sort_now(self):
        _check(lib().slpic_sort_now(self._ctx, self._stream()), "slpic_sort_now")

    # ---------------------------------------------------------------- state
    def status(self, run: int | None = None):
        st = (RunStatus * self.nruns)()
        _check(lib().slpic_status_query(self._ctx, st, self.nruns), "slpic_status_query")
        out = [s.as_dict() for s in st]
        return out if run is None else out[run]

    def export_particles(self, run: int, species: int):
        n = ctypes.c_int64(0)
        lib().slpic_export_particles(self._ctx, run, species, None, None, None, ctypes.byref(n))
        cnt = n.value
        x, vx, vp = (np.zeros(max(cnt, 1)) for _ in range(3))
        n = ctypes.c_int64(max(cnt, 1))
        _check(lib().slpic_export_particles(self._ctx, run, species, _dp(x), _dp(vx), _dp(vp),
                                            ctypes.byref(n)), "slpic_export_particles")
        k = n.value
        return x[:k], vx[:k], vp[:k]

    def import_particles(self, run: int, species: int, xt, vx, vperp2):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (xt, vx, vperp2)]
        _check(lib().slpic_import_particles(self._ctx, run, species, *[_dp(a) for a in arrs],
                                            len(arrs[0])), "slpic_import_particles")

    def set_counters(self, run: int, step: int, acc_e: float):
        _check(lib().slpic_set_counters(self._ctx, run, int(step), float(acc_e)), "slpic_set_counters")

    def prune_retired(self) -> int:
        """Take retired runs out of the push and sort work; returns how many
        runs are pruned."""
        n = ctypes.c_int32(0)
        _check(lib().slpic_prune_retired(self._ctx, ctypes.byref(n), self._stream()), "slpic_prune_retired")
        return n.value

    def set_speed_limit(self, run: int, u: float, dt: float):
        """Change run's speed limit to u with time step dt (f = beta g kept by
        resampling the g-particles at the weight of a fresh load at u)."""
        _check(lib().slpic_set_speed_limit(self._ctx, int(run), float(u), float(dt), self._stream()),
               "slpic_set_speed_limit")
        self.configs[run]["u"], self.configs[run]["dt"] = float(u), float(dt)

    def set_flux_counters(self, run: int, acc):
        a = np.ascontiguousarray(acc, dtype=np.float64)
        _check(lib().slpic_set_flux_counters(self._ctx, run, _dp(a)), "slpic_set_flux_counters")

    def grid(self, run: int = 0):
        nodes = self.configs[run]["nx"] + 1
        Q = np.zeros(2 * nodes)
        phi = np.zeros(nodes)
        E = np.zeros(nodes)
        _check(lib().slpic_export_grid(self._ctx, run, _dp(Q), _dp(phi), _dp(E)), "slpic_export_grid")
        return {"Q": Q.reshape(2, nodes), "phi": phi, "E": E}

    def perm(self, run: int, species: int) -> np.ndarray:
        if not self._tun.record_perm:
            raise SlpicError("sort permutations are recorded only with record_perm=True")
        n = ctypes.c_int64(0)
        lib().slpic_export_perm(self._ctx, run, species, None, ctypes.byref(n))
        p = np.zeros(max(n.value, 1), dtype=np.int32)
        n = ctypes.c_int64(len(p))
        _check(lib().slpic_export_perm(self._ctx, run, species, p.ctypes.data_as(_PI32),
                                       ctypes.byref(n)), "slpic_export_perm")
        return p[: n.value]

    def moments(self, run: int = 0) -> torch.Tensor:
        nodes = self.configs[run]["nx"] + 1
        out = torch.empty((7, nodes), dtype=torch.float64, device=self.device)
        _check(lib().slpic_moments(self._ctx, run, _P(out.data_ptr()), self._stream()), "slpic_moments")
        return out

    def moments_sample(self, run: int = -1):
        """Add the current moments of one run (or all, run = -1) to the
        device moment windows."""
        _check(lib().slpic_moments_sample(self._ctx, int(run), self._stream()), "slpic_moments_sample")

    def set_sampling(self, every: int):
        """Sample the moments of every run inside the step sequence (graphs
        included) at each step count that is a multiple of `every`; 0 = off."""
        _check(lib().slpic_set_sampling(self._ctx, int(every)), "slpic_set_sampling")

    def moments_window(self, run: int = 0, reset: bool = False) -> torch.Tensor:
        """Window mean of the sampled moments of one run (layout of moments())."""
        nodes = self.configs[run]["nx"] + 1
        out = torch.empty((7, nodes), dtype=torch.float64, device=self.device)
        _check(lib().slpic_moments_window(self._ctx, run, _P(out.data_ptr()), int(bool(reset)), self._stream()),
               "slpic_moments_window")
        return out

    def wall_history(self, run: int = 0) -> np.ndarray:
        """Phi_w after each of the run's last min(step, 4096) steps, oldest first."""
        out = np.zeros(4096)
        n = ctypes.c_int64(0)
        _check(lib().slpic_wall_history(self._ctx, run, _dp(out), ctypes.byref(n)), "slpic_wall_history")
        return out[:n.value].copy()

    def wall_potential(self, run: int = 0) -> float:
        return self.status(run)["wall_potential"]

    # ---------------------------------------------------------------- timing
    def profile(self, enable=True):
        """enable: True (push kernel only), False, or a bitmask of
        PROFILE_CLASSES (1 push, 2 inject, 4 field, 8 sort)."""
        mask = (1 if enable else 0) if isinstance(enable, bool) else int(enable)
        _check(lib().slpic_profile(self._ctx, mask), "slpic_profile")

    def profile_read(self) -> dict:
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_int64 * 4)()
        _check(lib().slpic_profile_read(self._ctx, ms, n), "slpic_profile_read")
        return {k: {"ms": ms[i], "launches": n[i]} for i, k in enumerate(PROFILE_CLASSES)}

    def pushed_total(self) -> int:
        """Live particles advanced by push launches since init (all runs)."""
        t = ctypes.c_int64(0)
        _check(lib().slpic_total_slots(self._ctx, ctypes.byref(t)), "slpic_total_slots")
        return t.value


def fixed_point_round(xt: np.ndarray, fixed_bits: int) -> np.ndarray:
    """Positions as an F32 context stores them: round-to-nearest-even on the
    2^-fixed_bits grid (dead slots, xt < 0, stay negative)."""
    xt = np.asarray(xt, dtype=np.float64)
    scale = math.ldexp(1.0, fixed_bits)
    q = np.rint(xt * scale) / scale
    return np.where(xt < 0, -1.0, q)


# ---------------------------------------------------------------- warm-start network
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS = 4, 256, 1792, 593408
MLP_NOALLOC_MAX_BATCH = 1024


class Mlp:
    """The warm-start network's buffers (torch tensors on the device) and
    its library calls: forward, backward and Adam run in the HIP kernels."""

    def __init__(self, params_fp32, batch: int, device="cuda"):
        if batch <= 0 or batch % 16:
            raise SlpicError("batch must be a positive multiple of 16")
        self.device = torch.device(device)
        self.batch = int(batch)
        self.p32 = torch.as_tensor(params_fp32, dtype=torch.float32).to(self.device).contiguous()
        if self.p32.numel() != MLP_PARAMS:
            raise SlpicError("parameter vector has the wrong length")
        self.pbf16 = torch.empty(MLP_PARAMS, dtype=torch.int16, device=self.device)
        self.m = torch.zeros_like(self.p32)
        self.v = torch.zeros_like(self.p32)
        self.grads = torch.zeros_like(self.p32)
        L = lib()
        self.act = torch.empty(L.slpic_mlp_act_bytes(self.batch), dtype=torch.uint8, device=self.device)
        self.work = torch.empty(L.slpic_mlp_work_bytes(self.batch), dtype=torch.uint8, device=self.device)
        self.y = torch.empty((self.batch, MLP_OUT), dtype=torch.float32, device=self.device)
        self.step = 0
        _check(L.slpic_mlp_to_bf16(_P(self.p32.data_ptr()), _P(self.pbf16.data_ptr()), self._stream()),
               "slpic_mlp_to_bf16")

    def _stream(self):
        return _P(torch.cuda.current_stream(self.device).cuda_stream)

    def forward(self, x) -> torch.Tensor:
        """y [batch][1792] from x [batch][4] (FP32, standardised)."""
        x = torch.as_tensor(x, dtype=torch.float32).to(self.device).contiguous()
        if tuple(x.shape) != (self.batch, MLP_IN):
            raise SlpicError("x must be [batch][4]")
        self._x = x
        _check(lib().slpic_mlp_forward(_P(self.pbf16.data_ptr()), _P(x.data_ptr()), _P(self.y.data_ptr()),
                                       self.batch, _P(self.act.data_ptr()), self._stream()), "slpic_mlp_forward")
        return self.y

    def forward_noalloc(self, x, y=None) -> torch.Tensor:
        """The same forward pass through slpic_mlp_forward_noalloc: the
        activations stay in the library's fixed device array (nothing for
        backward); y [n][1792] is written for x [n][4], n a multiple of 16 up
        to MLP_NOALLOC_MAX_BATCH."""
        x = torch.as_tensor(x, dtype=torch.float32).to(self.device).contiguous()
        if x.dim() != 2 or x.shape[1] != MLP_IN:
            raise SlpicError("x must be [n][4]")
        if y is None:
            y = torch.empty((x.shape[0], MLP_OUT), dtype=torch.float32, device=self.device)
        _check(lib().slpic_mlp_forward_noalloc(_P(self.pbf16.data_ptr()), _P(x.data_ptr()), _P(y.data_ptr()),
                                               int(x.shape[0]), self._stream()), "slpic_mlp_forward_noalloc")
        return y

    def backward(self, dy) -> torch.Tensor:
        """FP32 gradient of sum(dy * y) for the last forward batch."""
        dy = torch.as_tensor(dy, dtype=torch.float32).to(self.device).contiguous()
        _check(lib().slpic_mlp_backward(_P(self.pbf16.data_ptr()), _P(self.act.data_ptr()), _P(dy.data_ptr()),
                                        _P(self.grads.data_ptr()), self.batch, _P(self.work.data_ptr()),
                                        self._stream()), "slpic_mlp_backward")
        return self.grads

    def mse_backward(self, target) -> float:
        """Loss of the last forward batch against target (MSE), and the
        backward pass of its gradient; returns the loss (synchronises)."""
        t = torch.as_tensor(target, dtype=torch.float32).to(self.device).contiguous()
        if not hasattr(self, "_dy"):
            self._dy = torch.empty_like(self.y)
            self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self._loss.zero_()
        _check(lib().slpic_mlp_mse(_P(self.y.data_ptr()), _P(t.data_ptr()), _P(self._dy.data_ptr()), self.y.numel(),
                                   _P(self._loss.data_ptr()), self._stream()), "slpic_mlp_mse")
        self.backward(self._dy)
        return float(self._loss.item())

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        _check(lib().slpic_mlp_adam(_P(self.p32.data_ptr()), _P(self.pbf16.data_ptr()), _P(self.m.data_ptr()),
                                    _P(self.v.data_ptr()), _P(self.grads.data_ptr()), float(lr), float(beta1),
                                    float(beta2), float(eps), self.step, self._stream()), "slpic_mlp_adam")



class Sim2D:
    """One 2D3V sheath (y periodic over ny cells, dy = dx) on one GPU."""

    def __init__(self, config: dict, ny: int, precision="f32", sort_every=8, tile=8, margin=0, per_thread=0,
                 tail_groups=0, sort_tile=0, graph_steps=0, device="cuda", record_perm=False):
        self.config = dict(config)
        self.nx, self.ny = int(config["nx"]), int(ny)
        self.precision = precision
        self._cfg = run_config(self.config)
        t = Tuning2D()
        t.precision = {"f32": SLPIC_F32, "f64": SLPIC_F64}[precision]
        t.sort_every, t.tile, t.margin = int(sort_every), int(tile), int(margin)
        t.per_thread, t.tail_groups, t.sort_tile = int(per_thread), int(tail_groups), int(sort_tile)
        t.graph_steps = int(graph_steps)
        t.record_perm = int(bool(record_perm))
        self._tun = t
        L = lib()
        nbytes = L.slpic2d_workspace_bytes(ctypes.byref(self._cfg), self.ny, ctypes.byref(t))
        if nbytes == 0:
            raise SlpicError("invalid 2D configuration")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._ws_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.workspace_bytes = nbytes
        self._ctx = _P()
        _check(L.slpic2d_init(ctypes.byref(self._cfg), self.ny, ctypes.byref(t), _P(self._ws_ptr), nbytes,
                              self._stream(), ctypes.byref(self._ctx)), "slpic2d_init")

    def _stream(self):
        return _P(torch.cuda.current_stream(self.device).cuda_stream)

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            torch.cuda.synchronize(self.device)
            lib().slpic2d_destroy(self._ctx)
            self._ctx = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        _check(lib().slpic2d_step(self._ctx, int(n), self._stream()), "slpic2d_step")

    def refresh_fields(self):
        _check(lib().slpic2d_refresh_fields(self._ctx, self._stream()), "slpic2d_refresh_fields")

    def solve_charge(self, Q):
        """phi and E from a node charge array (2, nx+1, ny) (rho = Q/dV)."""
        q = torch.as_tensor(np.ascontiguousarray(Q, dtype=np.float64)).to(self.device)
        _check(lib().slpic2d_solve_charge(self._ctx, _P(q.data_ptr()), self._stream()), "slpic2d_solve_charge")
        torch.cuda.synchronize(self.device)

    def sort_now(self):
        _check(lib().slpic2d_sort_now(self._ctx, self._stream()), "slpic2d_sort_now")

    def status(self) -> dict:
        st = Status2D()
        _check(lib().slpic2d_status_query(self._ctx, ctypes.byref(st)), "slpic2d_status_query")
        return st.as_dict()

    def grid(self):
        shape = (self.nx + 1, self.ny)
        nodes = shape[0] * shape[1]
        Q, phi, E = np.zeros(2 * nodes), np.zeros(nodes), np.zeros(2 * nodes)
        _check(lib().slpic2d_export_grid(self._ctx, _dp(Q), _dp(phi), _dp(E)), "slpic2d_export_grid")
        E = E.reshape(2, *shape)
        return {"Q": Q.reshape(2, *shape), "phi": phi.reshape(shape), "Ex": E[0], "Ey": E[1]}

    def export_particles(self, species: int):
        """(x, y, vx, vy, vz^2) of the occupied slots (dead slots x < 0)."""
        cnt = self.status()["nslots"][species]
        arrs = [np.zeros(max(cnt, 1)) for _ in range(5)]
        n = ctypes.c_int64(len(arrs[0]))
        _check(lib().slpic2d_export_particles(self._ctx, species, *[_dp(a) for a in arrs], ctypes.byref(n)),
               "slpic2d_export_particles")
        return tuple(a[: n.value] for a in arrs)

    def import_particles(self, species: int, x, y, vx, vy, vz2):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, vx, vy, vz2)]
        _check(lib().slpic2d_import_particles(self._ctx, species, *[_dp(a) for a in arrs], len(arrs[0])),
               "slpic2d_import_particles")

    def set_counters(self, step: int, acc_e: float):
        _check(lib().slpic2d_set_counters(self._ctx, int(step), float(acc_e)), "slpic2d_set_counters")

    def perm(self, species: int) -> np.ndarray:
        if not self._tun.record_perm:
            raise SlpicError("sort permutations are recorded only with record_perm=True")
        cnt = max(self.status()["capacity"][species], 1)
        p = np.zeros(cnt, dtype=np.int32)
        n = ctypes.c_int64(cnt)
        _check(lib().slpic2d_export_perm(self._ctx, species, p.ctypes.data_as(_PI32), ctypes.byref(n)),
               "slpic2d_export_perm")
        return p[: n.value]

    def moments(self) -> torch.Tensor:
        """beta-weighted node moments (7, nx + 1, ny) on the device: phi, then
        n, Gamma_x, kinetic energy density per species."""
        out = torch.empty(7 * (self.nx + 1) * self.ny, dtype=torch.float64, device=self.device)
        _check(lib().slpic2d_moments(self._ctx, _P(out.data_ptr()), self._stream()), "slpic2d_moments")
        return out.view(7, self.nx + 1, self.ny)

    def wall_history(self) -> np.ndarray:
        """Phi_w after each of the last min(step, 4096) steps, oldest first."""
        out = np.zeros(4096)
        n = ctypes.c_int64(0)
        _check(lib().slpic2d_wall_history(self._ctx, _dp(out), ctypes.byref(n)), "slpic2d_wall_history")
        return out[:n.value].copy()

    def profile(self, enable: int):
        _check(lib().slpic2d_profile(self._ctx, int(enable)), "slpic2d_profile")

    def profile_read(self):
        ms = np.zeros(4)
        cnt = np.zeros(4, dtype=np.int64)
        _check(lib().slpic2d_profile_read(self._ctx, _dp(ms), cnt.ctypes.data_as(_PI64)), "slpic2d_profile_read")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(PROFILE_CLASSES)}

"""The velocity map of Eq. (A2a) on the GPU (slpic_velocity_map) against the
oracle's exact frozen-field integral, case by case, over every segment
pattern of Eq. (11b) and over Eq. (11a), in FP64 and FP32."""
import ctypes
import math

import numpy as np
import pytest

import oracle
from parity_util import print_case

pytestmark = pytest.mark.gpu


def _cases(n=4000, seed=0):
    rng = np.random.default_rng(seed)
    vx = rng.normal(size=n) * 10 ** rng.uniform(-2, 0.7, size=n)
    vp2 = (rng.normal(size=n) * 10 ** rng.uniform(-3, 0.5, size=n)) ** 2
    vp2[: n // 20] = 0.0                      # no perpendicular speed
    a = rng.normal(size=n) * 10 ** rng.uniform(-4, 0.5, size=n)
    a[n // 20: n // 10] = 0.0                 # no field
    return vx, vp2, a


def _run(gpu_lib, prec, kind, u, dt, vx, vp2, a):
    import torch
    dt_ = torch.float32 if prec == "f32" else torch.float64
    tv = torch.tensor(vx, dtype=dt_, device="cuda")
    tc = torch.tensor(vp2, dtype=dt_, device="cuda")
    ta = torch.tensor(a, dtype=dt_, device="cuda")
    out = torch.empty_like(tv)
    it = torch.zeros(len(vx), dtype=torch.int32, device="cuda")
    L = gpu_lib.lib()
    L.slpic_velocity_map.restype = ctypes.c_int
    L.slpic_velocity_map.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int64] + [ctypes.c_void_p] * 6
    rc = L.slpic_velocity_map(0 if prec == "f32" else 1, 0 if kind == "step" else 1, u, dt, len(vx),
                              tv.data_ptr(), tc.data_ptr(), ta.data_ptr(), out.data_ptr(), it.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    return out.double().cpu().numpy(), it.cpu().numpy()


@pytest.mark.parametrize("kind", ["step", "smooth"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("u,dt", [(0.05, 3.0), (1.0, 0.7), (math.inf, 0.5)])
def test_velocity_map_matches_oracle(gpu_lib, kind, prec, u, dt):
    vx, vp2, a = _cases()
    if prec == "f32":  # both sides see the float-rounded inputs
        vx, vp2, a = (x.astype(np.float32).astype(np.float64) for x in (vx, vp2, a))
    got, iters = _run(gpu_lib, prec, kind, u, dt, vx, vp2, a)
    want = np.array([oracle.kick_exact(kind, u, dt, [vx[i], math.sqrt(vp2[i]), 0.0], [a[i], 0, 0])[0]
                     for i in range(len(vx))])
    c = np.sqrt(vp2)
    scale = np.maximum.reduce([np.abs(want), np.abs(vx), c, np.full_like(c, 1e-30)])
    err = np.abs(got - want) / scale
    print_case(f"kick {prec} {kind} u={u}: max rel err {err.max():.2e}, Newton its mean "
               f"{iters.mean():.2f} max {iters.max()}")
    if prec == "f64":
        # G-inversion rounding: |dp| ~ eps (p0^2 + c^2) / max(s1, c)
        assert err.max() <= 2e-11
    else:
        # float rounding of G differences and of the stored result
        assert err.max() <= 4e-6
    if math.isinf(u) and prec == "f64":
        assert np.array_equal(got, vx + a * dt)  # beta = 1: the standard leapfrog kick


@pytest.mark.parametrize("kind", ["step", "smooth"])
@pytest.mark.parametrize("u,dt", [(0.05, 3.0), (1.0, 0.7)])
def test_fp64_velocity_error_against_40_digit_map(gpu_lib, kind, u, dt):
    """The worst actual error of the FP64 map on the GPU, measured against
    the map in 40-digit arithmetic over random and worst-conditioned cases
    (slowed through zero with perpendicular speeds down to 1e-8): at most
    1e-13 of max(1, |v|), a hundred times inside the 1e-11 floor of the
    lockstep parity tests."""
    import mp_kick
    vx, c2, a = mp_kick.hard_cases(600, seed=2)
    got, _ = _run(gpu_lib, "f64", kind, u, dt, vx, c2, a)
    want = np.array([mp_kick.kick(kind, u, dt, vx[i], c2[i], a[i]) for i in range(len(vx))])
    scale = np.maximum(1.0, np.maximum(np.abs(want), np.abs(vx)))
    err = np.abs(got - want) / scale
    print_case(f"kick f64 {kind} u={u}: worst error vs 40 digits {err.max():.2e} (case {int(err.argmax())})")
    assert err.max() <= 1e-13

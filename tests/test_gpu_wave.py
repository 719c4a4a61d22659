"""Test particles in a prescribed traveling wave on the GPU (slpic_wave_push)
against the oracle, element by element, and the paper's wave-particle
findings at scale: with the limit well above the phase velocity the velocity
distribution matches the unlimited push, with the limit at the phase
velocity the particles above it are depleted."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from parity_util import print_case

pytestmark = pytest.mark.gpu


def _periodic_diff(a, b, L):
    d = np.abs(a - b)
    return np.minimum(d, L - d)


@pytest.mark.parametrize("r", [math.inf, 2.0, 1.5, 1.25, 1.0])
@pytest.mark.parametrize("kind", ["step", "smooth"])
def test_wave_push_f64_matches_oracle(gpu_lib, r, kind):
    w, x0, v0 = workloads.wave_test(r, n=3000, seed=4, beta_kind=kind)
    w["ramp_time"] = 200.0  # reach full amplitude inside the compared steps
    print_case(f"wave f64 v0/vphi={r} {kind}")
    xg = torch.tensor(x0, device="cuda")
    vg = torch.tensor(v0, device="cuda")
    xo, vo = x0.copy(), v0.copy()
    step = 0
    for chunk in (1, 99, 200):
        gpu_lib.wave_push(w, xg, vg, step, chunk)
        xo, vo = oracle.wave_push(w, xo, vo, step, chunk)
        step += chunk
        torch.cuda.synchronize()
        xa, va = xg.cpu().numpy(), vg.cpu().numpy()
        assert _periodic_diff(xa, xo, w["length"]).max() <= 1e-9, (chunk,)
        assert np.abs(va - vo).max() <= 1e-9, (chunk,)


@pytest.mark.parametrize("r", [math.inf, 2.0, 1.0])
def test_wave_push_f32_matches_oracle(gpu_lib, r):
    w, x0, v0 = workloads.wave_test(r, n=3000, seed=5)
    w["ramp_time"] = 50.0
    x32, v32 = x0.astype(np.float32), v0.astype(np.float32)
    print_case(f"wave f32 v0/vphi={r}")
    xg = torch.tensor(x32, device="cuda")
    vg = torch.tensor(v32, device="cuda")
    gpu_lib.wave_push(w, xg, vg, 0, 60)
    xo, vo = oracle.wave_push(w, x32.astype(np.float64), v32.astype(np.float64), 0, 60)
    torch.cuda.synchronize()
    xa, va = xg.cpu().numpy().astype(np.float64), vg.cpu().numpy().astype(np.float64)
    assert _periodic_diff(xa, xo, w["length"]).max() <= 2e-4 * w["length"]
    assert np.abs(va - vo).max() <= 2e-4


def test_wave_push_rejects_bad_arguments(gpu_lib):
    w, x0, v0 = workloads.wave_test(2.0, n=10)
    x = torch.tensor(x0, device="cuda")
    v = torch.tensor(v0.astype(np.float32), device="cuda")
    with pytest.raises(gpu_lib.SlpicError):
        gpu_lib.wave_push(w, x, v, 0, 1)  # mixed dtypes
    v = torch.tensor(v0, device="cuda")
    with pytest.raises(gpu_lib.SlpicError):
        gpu_lib.wave_push(dict(w, dt=-1.0), x, v, 0, 1)


def _distribution(push, r, n=1_000_000, periods=40):
    w, x0, v0 = workloads.wave_test(r, n=n, seed=7)
    xg = torch.tensor(x0.astype(np.float32), device="cuda")
    vg = torch.tensor(v0.astype(np.float32), device="cuda")
    steps = int(round(periods * w["length"] / w["v_phase"] / w["dt"]))
    done = 0
    while done < steps:
        k = min(2000, steps - done)
        push(w, xg, vg, done, k)
        done += k
    torch.cuda.synchronize()
    return vg.cpu().numpy().astype(np.float64)


def test_wave_particle_findings_at_scale(gpu_lib):
    """One million electrons, 40 wave periods (amplitude ramped over the
    first 20): the distribution in the flattened region 0.5-1.5 v_phi with
    v0 = 2 v_phi agrees with the unlimited push to within sampling noise; the
    resonant region is flattened against the initial Maxwellian; with v0 =
    v_phi the distribution departs from the unlimited one far beyond the
    noise, with the region just above the phase velocity depleted."""
    print_case("wave distributions at scale")
    bins = np.linspace(0.25, 1.75, 16)
    h = {r: np.histogram(_distribution(gpu_lib.wave_push, r), bins=bins)[0].astype(float)
         for r in (math.inf, 2.0, 1.0)}
    h0 = np.histogram(np.random.default_rng(7).normal(0, 1, 1_000_000), bins=bins)[0].astype(float)
    sig = np.sqrt(h[math.inf] + h[2.0])
    assert np.all(np.abs(h[2.0] - h[math.inf]) <= 5 * sig + 1)
    # flattening: the slope of f(v) across the resonance is reduced
    mid = (bins[:-1] + bins[1:]) / 2
    sel = (mid > 0.7) & (mid < 1.3)
    slope = lambda c: np.polyfit(mid[sel], c[sel], 1)[0]  # noqa: E731
    assert abs(slope(h[math.inf])) < 0.6 * abs(slope(h0))
    # v0 = v_phi: far from PIC, fewer particles just above v_phi
    assert np.max(np.abs(h[1.0] - h[math.inf]) / np.sqrt(h[1.0] + h[math.inf] + 1)) > 10
    above = (mid > 1.1) & (mid < 1.6)
    assert h[1.0][above].sum() < 0.9 * h[math.inf][above].sum()

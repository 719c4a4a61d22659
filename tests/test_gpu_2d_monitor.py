"""2D3V diagnostics and step replay on the HIP path against the oracle: the
beta-weighted node moments (Eq. 5), the wall-potential history and steady
detector fed after every step, and HIP-graph replay of blocks of steps
against direct launches."""
import numpy as np
import pytest

import oracle
import workloads
from parity_util import print_case, rel_inf
from test_gpu_parity2d import _cfg, _push_to_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_moments2d_match_oracle(gpu_lib, prec):
    cfg, ny = _cfg(nx=16, ny=8, ppc=20, u_over_vti=3.0, sort_every=2, seed=41)
    run = oracle.Run2D(cfg, ny, tile=4)
    run.step(10)
    sim = gpu_lib.Sim2D(cfg, ny, precision=prec, sort_every=2, tile=4, margin=2)
    _push_to_gpu(sim, run, quantize=prec == "f32")
    sim.refresh_fields()
    m = sim.moments().cpu().numpy()
    o = run.moments()
    tol = 1e-11 if prec == "f64" else 1e-5
    for row in range(7):
        err = rel_inf(m[row], o[row])
        print_case(f"2d moments {prec} row {row}: {err:.2e}")
        assert err <= tol, (row, err)
    sim.close()


def test_wall_history_and_detector_match_oracle_f64(gpu_lib):
    """Both sides from the same cold load, the oracle's state handed over
    before every step: Phi_w after each step (the GPU's history ring), the
    window means and the steady step (windows of 2 steps, tolerance 0.5, so
    the detector flags within the run)."""
    cfg, ny = _cfg(nx=16, ny=8, ppc=20, u_over_vti=3.0, sort_every=2, seed=42)
    cfg = dict(cfg, steady_window=2, steady_tol=0.5)
    run = oracle.Run2D(cfg, ny, tile=4)
    sim = gpu_lib.Sim2D(cfg, ny, precision="f64", sort_every=2, tile=4, margin=2)
    phis = []
    for k in range(24):
        _push_to_gpu(sim, run, quantize=False)
        sim.refresh_fields()
        sim.step(1)
        run.step(1)
        phis.append(run.wall_potential())
    hist = sim.wall_history()
    assert len(hist) == 24
    np.testing.assert_allclose(hist, phis, rtol=1e-10, atol=1e-12 * np.abs(phis).max())
    st, od = sim.status(), run.steady()
    print_case(f"2d detector: gpu steady {st['steady_step']} oracle {od['steady_step']}, windows {od['windows']}")
    assert st["windows"] == od["windows"] == 12
    np.testing.assert_allclose(st["window_mean"], od["window_mean"], rtol=1e-10, atol=1e-12)
    assert st["steady_step"] == od["steady_step"] >= 0
    sim.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graph_replay2d_matches_direct_launches(gpu_lib, prec):
    """Blocks of 8 steps captured once and replayed as a HIP graph (side
    stream) against the same steps launched directly, checked after every
    replay with host reads in between: charge, counts, Phi_w history."""
    import torch
    cfg, ny = _cfg(nx=32, ny=16, ppc=16, u_over_vti=3.0, sort_every=4, seed=43)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        a = gpu_lib.Sim2D(cfg, ny, precision=prec, sort_every=4, tile=4, margin=4, graph_steps=8)
        b = gpu_lib.Sim2D(cfg, ny, precision=prec, sort_every=4, tile=4, margin=4, graph_steps=0)
        for k in range(4):
            print_case(f"2d graph replay {prec} block {k}")
            a.step(8)
            b.step(8)
            ga, gb = a.grid(), b.grid()
            # FP64 charge atomics land in either order, so float particles may
            # round a velocity differently by an ulp: the FP32 bar there
            tol = 1e-9 if prec == "f64" else 1e-5
            for s in range(2):
                assert rel_inf(ga["Q"][s], gb["Q"][s]) <= tol, (k, s)
            sa, sb = a.status(), b.status()
            assert sa["nslots"] == sb["nslots"] and sa["injected_total"] == sb["injected_total"], k
            assert sa["step"] == sb["step"] == 8 * (k + 1)
        np.testing.assert_allclose(a.wall_history(), b.wall_history(), rtol=tol,
                                   atol=1e-12 * np.abs(b.wall_history()).max())
        a.close()
        b.close()


def test_y_averaged_2d_sheath_matches_1d(gpu_lib):
    """The physics check of the 2D3V configuration (App. A, Eq. A1 in two
    dimensions): with y periodic and the source uniform in y, the 2D sheath
    is the 1D sheath, so its y-averaged moments must match the 1D run's.
    64 cells, u = 3 v_ti, 100 g-particles per 2D cell and ny = 16 against
    1600 per 1D cell (equal particles per x-cell, so equal noise and noise
    heating), FP32, four seeds each, moments averaged over steps 2048-4096:
    phi within 6 % of its largest value, n_e, n_i and the electron energy
    density within 5 % of theirs (measured: 2.4 %, 2.3 %, 2.0 %, 2.2 %)."""
    import torch
    nx, ppc2, ny, steps, start = 64, 100, 16, 4096, 2048
    prof1, prof2 = [], []
    with torch.cuda.stream(torch.cuda.Stream()):
        for sd in range(4):
            print_case(f"2d vs 1d seed {sd}")
            s1 = gpu_lib.Sim(workloads.small_sheath(seed=100 + sd, ppc=ppc2 * ny, sort_every=16), precision="f32",
                             sort_every=16, graph_steps=16)
            s2 = gpu_lib.Sim2D(workloads.small_sheath(seed=200 + sd, ppc=ppc2, sort_every=8), ny, precision="f32",
                               sort_every=8, tile=8, graph_steps=16)
            acc1, acc2, n = np.zeros((7, nx + 1)), np.zeros((7, nx + 1)), 0
            for done in range(16, steps + 1, 16):
                s1.step(16)
                s2.step(16)
                if done > start:
                    acc1 += s1.moments(0).cpu().numpy().reshape(7, nx + 1)
                    acc2 += s2.moments().cpu().numpy().mean(axis=2)
                    n += 1
            assert s1.status(0)["error_flags"] == 0 and s2.status()["error_flags"] == 0
            prof1.append(acc1 / n)
            prof2.append(acc2 / n)
            s1.close()
            s2.close()
    p1, p2 = np.mean(prof1, axis=0), np.mean(prof2, axis=0)
    for row, name, tol in ((0, "phi", 0.06), (1, "n_e", 0.05), (4, "n_i", 0.05), (3, "K_e", 0.05)):
        err = np.abs(p1[row] - p2[row]).max() / np.abs(p1[row]).max()
        print_case(f"2d y-average vs 1d: {name} {err:.4f}")
        assert err <= tol, (name, err)

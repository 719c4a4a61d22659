"""The learned warm start end to end at a small scale: profiles from batched
cold runs, training in the library's kernels, prediction, warm loads that
step cleanly; the wall-potential history export."""
import numpy as np
import pytest

import workloads
from parity_util import print_case

pytestmark = pytest.mark.gpu


def test_wall_history_matches_status(gpu_lib):
    cfg = workloads.small_sheath(seed=21)
    sim = gpu_lib.Sim(cfg, precision="f64", sort_every=8)
    sim.step(40)
    h = sim.wall_history(0)
    assert len(h) == 40
    assert h[-1] == sim.status(0)["wall_potential"]
    W = cfg["nx"] // 4
    assert sim.status(0)["window_mean"][0] == pytest.approx(h[W:2 * W].mean(), rel=1e-12)


def test_collect_train_predict_warm_load(gpu_lib):
    from paper_1511_08225_amd import warmstart
    cfgs = workloads.batched_sweep(nruns=8, seed=22, cells_range=(128, 192), ppc_range=(50, 80))
    prof, phi_w = warmstart.collect_profiles(cfgs, steps=512, sample_every=32, sample_last=256)
    assert prof.shape == (8, 5, 256) and np.isfinite(prof).all()
    assert np.all(prof[:, 1:3].mean(axis=2) > 0)  # densities
    X = np.stack([warmstart.features(c) for c in cfgs])
    net, std, losses = warmstart.train(X, prof.reshape(8, -1), epochs=60, batch=16)
    print_case(f"warm-start training loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    assert losses[-1] < 0.5 * losses[0]
    pred = warmstart.predict(net, std, cfgs)
    assert pred.shape == (8, 5, 256) and np.isfinite(pred).all()
    sim = gpu_lib.Sim(cfgs, precision="f32", sort_every=16, warm=list(pred))
    st0 = sim.status()
    sim.step(64)
    st = sim.status()
    assert all(s["error_flags"] == 0 for s in st)
    for r in range(8):  # loaded near the predicted density: about nx ppc n/n0 particles
        n_pred = pred[r, 1].mean()
        expect = cfgs[r]["nx"] * cfgs[r]["species"][0]["ppc"] * n_pred
        assert 0.5 * expect < st0[r]["nslots"][0] < 2.0 * expect + 100, (r, st0[r]["nslots"][0], expect)

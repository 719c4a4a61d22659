"""The learned warm start end to end at a small scale: profiles from batched
cold runs, training in the library's kernels, prediction, warm loads that
step cleanly; the wall-potential history export."""
import numpy as np
import pytest

import oracle
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
    assert prof.shape == (8, 7, 256) and np.isfinite(prof).all()
    assert np.all(prof[:, 1:3].mean(axis=2) > 0)  # densities
    X = np.stack([warmstart.features(c) for c in cfgs])
    net, std, losses = warmstart.train(X, prof.reshape(8, -1), epochs=60, batch=16)
    print_case(f"warm-start training loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    assert losses[-1] < 0.5 * losses[0]
    pred = warmstart.predict(net, std, cfgs)
    assert pred.shape == (8, 7, 256) and np.isfinite(pred).all()
    sim = gpu_lib.Sim(cfgs, precision="f32", sort_every=16, warm=list(pred))
    st0 = sim.status()
    sim.step(64)
    st = sim.status()
    assert all(s["error_flags"] == 0 for s in st)
    for r in range(8):  # the loaded counts are the oracle's for the predicted profiles (density, drift, temperature)
        w = oracle.Run(cfgs[r], load=False).weights()
        for s in range(2):
            expect = sum(oracle.warm_cell_count(cfgs[r], s, pred[r], c, w[s])[0] for c in range(cfgs[r]["nx"]))
            assert st0[r]["nslots"][s] == expect, (r, s, st0[r]["nslots"][s], expect)


def test_warm_start_network_gains_over_cold_runs(gpu_lib):
    """What the trained network gains over the method without it, on
    held-out sheaths: its prediction of the late wall potential (the cold
    run's mean over the last quarter of 2048 steps, plain cold-start SLPIC
    being the reference) is available before the first step, and it is closer to
    that reference than the naive prediction (the training runs' mean) and
    than the cold run's own running estimate (its latest nx/4-step window)
    after a quarter of the run.  192 training sheaths, 32 held out, cells
    128-256, 100-200 per cell."""
    from paper_1511_08225_amd import warmstart
    cells, ppc, H = (128, 256), (100, 200), 2048
    train = workloads.batched_sweep(nruns=192, seed=2, cells_range=cells, ppc_range=ppc)
    held = workloads.batched_sweep(nruns=32, seed=3, cells_range=cells, ppc_range=ppc)
    tun = {"chunk": 512, "block": 128, "sort_every": 64, "sort_bucket": 1}
    print_case("warm-start gain: collecting 192 training profiles")
    Y, _ = warmstart.collect_profiles(train, steps=H, sample_every=32, sample_last=H // 4, tuning=tun)
    X = np.stack([warmstart.features(c) for c in train])
    net, std, losses = warmstart.train(X, Y.reshape(len(Y), -1), epochs=300, batch=64)
    pred = warmstart.predict(net, std, held)
    print_case("warm-start gain: 32 held-out cold runs")
    sim = gpu_lib.Sim(held, precision="f32", sort_every=64, sort_bucket=1, chunk=512, block=128, graph_steps=64)
    sim.step(H)
    hist = np.array([sim.wall_history(r)[-H:] for r in range(len(held))])
    assert all(s["error_flags"] == 0 for s in sim.status())
    sim.close()
    ref = hist[:, -H // 4:].mean(axis=1)
    e_net = np.abs(pred[:, 0, 0] - pred[:, 0, -1] - ref) / np.abs(ref)
    e_naive = np.abs((Y[:, 0, 0] - Y[:, 0, -1]).mean() - ref) / np.abs(ref)
    e_cold = np.array([abs(hist[r, H // 4 - max(1, c["nx"] // 4):H // 4].mean() - ref[r]) / abs(ref[r])
                       for r, c in enumerate(held)])
    print_case(f"warm-start gain: median error network {np.median(e_net):.3f}, naive {np.median(e_naive):.3f}, "
               f"cold run after H/4 {np.median(e_cold):.3f}; network better than naive in "
               f"{int((e_net < e_naive).sum())}/32")
    assert losses[-1] < 0.2 * losses[0]
    assert np.median(e_net) < 0.6 * np.median(e_naive)
    assert (e_net < e_naive).sum() >= 0.65 * len(held)
    assert np.median(e_net) < np.median(e_cold)

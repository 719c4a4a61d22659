"""The launch-parameter tuner: signature, coordinate descent and cache (CPU,
with a synthetic cost), and one real tuning pass on the GPU."""
import json

import pytest

import workloads
from paper_1511_08225_amd import autotune


def _cost(optimum):
    """A separable cost with its minimum at `optimum` (seconds per push)."""
    def f(configs, precision, params, steps, warmup):
        return 1e-11 * (1.0 + sum(abs(autotune.CANDIDATES[k].index(params[k]) -
                                      autotune.CANDIDATES[k].index(optimum[k])) for k in optimum))
    return f


def test_signature_groups_similar_run_sets():
    a = workloads.batched_sweep(nruns=16, seed=1)
    b = workloads.batched_sweep(nruns=16, seed=2)
    assert autotune.signature(a, "f32") != autotune.signature(a, "f64")
    assert autotune.signature(a, "f32").startswith("f32|runs=16|")
    assert autotune.signature(a[:1], "f32") != autotune.signature(a, "f32")
    # same distribution, same size class: usually the same key
    assert autotune.signature(a, "f32").split("|")[1] == autotune.signature(b, "f32").split("|")[1]


def test_coordinate_descent_finds_separable_optimum_and_caches(tmp_path):
    cfgs = workloads.batched_sweep(nruns=4, seed=3, cells_range=(64, 128), ppc_range=(20, 40))
    opt = {"chunk": 256, "block": 256, "sort_every": 32, "sort_bucket": 2, "push_order": 1, "sort_tile": 8192}
    path = str(tmp_path / "cache.json")
    got = autotune.tune(cfgs, "f32", cache_path=path, measure_fn=_cost(opt))
    assert got == opt
    cache = json.load(open(path))
    key = autotune.signature(cfgs, "f32")
    assert cache[key]["params"] == opt
    nc = len(autotune.CANDIDATES["chunk"]) * len(autotune.CANDIDATES["block"])
    # the default, its (chunk, block) group, then one new trial per other value
    assert len(cache[key]["trials"]) == 1 + (nc - 1) + (4 - 1) + (3 - 1) + (2 - 1) + (5 - 1)
    assert autotune.cached(cfgs, "f32", cache_path=path) == opt
    assert autotune.cached(cfgs, "f64", cache_path=path) is None
    # a cached key is returned without measuring
    def boom(*a):
        raise AssertionError("measured a cached signature")
    assert autotune.tune(cfgs, "f32", cache_path=path, measure_fn=boom) == opt


def test_entry_without_a_newer_parameter_is_extended(tmp_path):
    """A cached entry lacking parameters (tuned before they existed) keeps its
    values; only the missing groups are searched, from its best."""
    cfgs = workloads.batched_sweep(nruns=4, seed=3, cells_range=(64, 128), ppc_range=(20, 40))
    key = autotune.signature(cfgs, "f32")
    old = {"chunk": 1024, "block": 64, "sort_every": 64, "sort_bucket": 4}
    path = str(tmp_path / "cache.json")
    json.dump({key: {"params": old, "ps_per_push": 5.0, "trials": [{"params": old, "ps_per_push": 5.0}]}},
              open(path, "w"))
    seen = []
    opt = dict(old, push_order=1, sort_tile=32768)
    cost = _cost(opt)

    def measure(c, p, params, s, w):
        seen.append(dict(params))
        return cost(c, p, params, s, w)
    got = autotune.tune(cfgs, "f32", cache_path=path, measure_fn=measure)
    assert got == opt
    start = dict(old, push_order=0, sort_tile=16384)
    assert seen == [start, dict(start, push_order=1),
                    *[dict(start, push_order=1, sort_tile=t) for t in (2048, 4096, 8192, 32768)]]
    rec = json.load(open(path))[key]
    assert rec["params"] == opt and rec["earlier_trials"] == [{"params": old, "ps_per_push": 5.0}]
    assert rec["ps_per_push"] == min(t["ps_per_push"] for t in rec["trials"])


@pytest.mark.gpu
def test_tune_real_step_small_batch(gpu_lib, tmp_path):
    cfgs = workloads.batched_sweep(nruns=8, seed=4, cells_range=(128, 256), ppc_range=(100, 200))
    path = str(tmp_path / "cache.json")
    got = autotune.tune(cfgs, "f32", cache_path=path, steps=32, warmup=16)
    for k, v in got.items():
        assert v in autotune.CANDIDATES[k]
    rec = json.load(open(path))[autotune.signature(cfgs, "f32")]
    # the chosen trial is within the switch margin of the fastest one
    times = [t["ps_per_push"] for t in rec["trials"]]
    assert rec["ps_per_push"] in times
    assert rec["ps_per_push"] * (1.0 - autotune.SWITCH_MARGIN) <= min(times) * (1.0 + 1e-12)

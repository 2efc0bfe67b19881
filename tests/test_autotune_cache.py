"""Host logic of the autotuner cache (no GPU): degree signatures and the JSON
cache round trip, with a stand-in for the GPU search."""
import json

import numpy as np

import graphgen
from paper_2411_11468_amd import autotune, lpa


def test_signature_stable_and_discriminating():
    g = graphgen.rmat_graph(12, 3, "int8")
    s1 = autotune.degree_signature(g.offsets)
    assert s1 == autotune.degree_signature(g.offsets.astype(np.int64))
    # a different family differs
    r = graphgen.random_graph(4096, 0.004, seed=1)
    assert autotune.degree_signature(r.offsets) != s1
    assert autotune.degree_signature(g.offsets, 8) != s1


def test_round2():
    assert [autotune._round2(x) for x in (0, 7, 99, 100, 1234, 98765, 1_060_000)] == \
        [0, 7, 99, 100, 1200, 99000, 1_100_000]


def test_cache_round_trip(tmp_path):
    calls = []

    def fake(offsets, targets, weights, v_off=None, mode=0, budget_ms=0.0):
        calls.append(1)
        t = lpa.default_tuning()
        t.wave, t.block = 256, 4096
        return t, {"candidates": 73, "runs": 100}

    g = graphgen.rmat_graph(10, 1, "int8")
    path = str(tmp_path / "tune.json")
    t1, info1 = autotune.tuned(g.offsets, g.targets, g.weights, cache_path=path, tuner=fake)
    t2, info2 = autotune.tuned(g.offsets, g.targets, g.weights, cache_path=path, tuner=fake)
    assert len(calls) == 1 and not info1["cached"] and info2["cached"]
    assert autotune.tuning_to_dict(t1) == autotune.tuning_to_dict(t2)
    assert (t2.wave, t2.block) == (256, 4096)
    data = json.load(open(path))
    assert len(data) == 1
    # another mode is another entry
    autotune.tuned(g.offsets, g.targets, g.weights, mode=lpa.MODE_DETERMINISTIC,
                   cache_path=path, tuner=fake)
    assert len(calls) == 2 and len(json.load(open(path))) == 2


def test_swapstudy_variants():
    from paper_2411_11468_amd import swapstudy
    v = swapstudy.variants()
    assert len(v) == 24 and len({name for name, _, _ in v}) == 24
    assert ("PL4", 4, 0) in v and ("CC2", 0, 2) in v and ("H3,1", 3, 1) in v

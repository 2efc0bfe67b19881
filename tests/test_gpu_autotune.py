"""GPU: the autotuner returns a valid tuning, and deterministic results do not
depend on the tuning (labels equal the oracle's with the tuned thresholds)."""
import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2411_11468_amd import lpa  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _valid(t):
    assert 0 <= t.small4 <= 4 and t.small4 <= t.small16 <= 16 and t.small16 <= t.wave
    assert t.wave <= 512 and t.wave <= t.block <= 8192 and 64 <= t.hub_chunk <= 8192
    assert t.block_threads in (0, 256, 512, 1024) and t.table_load in (1, 2, 4)
    assert 1 <= t.pull_divisor <= 4096 and t.batch_queue in (-1, 0, 1)


def test_autotune_single_graph():
    g = graphgen.rmat_graph(15, 9, "int8")
    t, rep = lpa.lpa_autotune(_dev(g.offsets), _dev(g.targets), _dev(g.weights),
                              mode=lpa.MODE_DETERMINISTIC, budget_ms=20_000)
    _valid(t)
    assert rep["candidates"] >= 2 and rep["runs"] >= rep["candidates"]
    assert rep["best_ms"] > 0 and rep["default_ms"] > 0
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    G = lpa.LpaGraph(_dev(g.offsets), _dev(g.targets), _dev(g.weights), tuning=t)
    res = G.run("det")
    np.testing.assert_array_equal(res.labels.cpu().numpy(), ref.labels)
    G.close()


def test_autotune_batch_and_budget():
    g, v_off = graphgen.planted_partition_batch(32, 3, n_range=(256, 4000))
    t, rep = lpa.lpa_autotune(_dev(g.offsets), _dev(g.targets), _dev(g.weights), v_off=v_off,
                              budget_ms=1.0)
    _valid(t)
    # a tiny budget still measures at least the defaults
    assert rep["runs"] >= 2
    with pytest.raises(lpa.LpaError):
        lpa.lpa_autotune(_dev(g.offsets), _dev(g.targets), budget_ms=0.0)


def test_autotune_batch_schedule_and_labels():
    # a batch: the search covers the schedule (work queue chunk and group
    # sizes, or the class kernels); the tuned deterministic run equals the
    # oracle graph by graph
    g, v_off = graphgen.planted_partition_batch(48, 4, n_range=(256, 6000))
    t, rep = lpa.lpa_autotune(_dev(g.offsets), _dev(g.targets), _dev(g.weights), v_off=v_off,
                              mode=lpa.MODE_DETERMINISTIC, budget_ms=15_000)
    _valid(t)
    assert t.batch_queue in (0, 1)
    assert rep["candidates"] >= 14 and rep["best_ms"] > 0
    B = lpa.LpaBatch(v_off, _dev(g.offsets), _dev(g.targets), _dev(g.weights), tuning=t)
    res = B.run_batched("det")
    lab = res.labels.cpu().numpy()
    for q in range(48):
        a, b = int(v_off[q]), int(v_off[q + 1])
        ea, eb = int(g.offsets[a]), int(g.offsets[b])
        ref = oracle.lpa_sync(g.offsets[a:b + 1] - ea, g.targets[ea:eb] - a, g.weights[ea:eb])
        np.testing.assert_array_equal(lab[a:b] - a, ref.labels)
    B.close()

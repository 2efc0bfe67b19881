"""GPU: handles that keep labels and rows in the internal order by degree
(lpa_tuning.relabel = 1) against the oracle and against the caller's order.

Label values stay the caller's ids, so a deterministic run must equal the
oracle exactly (labels, iteration count, every per-iteration counter), and
every per-vertex array that leaves the library (labels, flags, records,
trace vertex ids) is in the caller's numbering.
"""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import mlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2411_11468_amd import lpa  # noqa: E402

SMALL_TUNING = dict(small4=2, small16=8, wave=40, block=100, hub_chunk=64)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _tuning(**kw):
    t = lpa.default_tuning()
    for k, v in kw.items():
        setattr(t, k, v)
    return t


def _graph(g, relabel, on_device=True, **tun):
    t = _tuning(relabel=relabel, **tun)
    if on_device:
        return lpa.LpaGraph(_dev(g.offsets), _dev(g.targets),
                            None if g.weights is None else _dev(g.weights), tuning=t)
    return lpa.LpaGraph(g.offsets, g.targets, g.weights, tuning=t)


def _labels(res):
    return res.labels.cpu().numpy() if hasattr(res.labels, "cpu") else np.asarray(res.labels)


def _assert_matches(ref, res):
    assert res.iterations == ref.iterations
    for a, b in zip(res.stats, ref.stats):
        for k in ("iteration", "pick_less", "changed", "processed", "edges_scanned"):
            assert a[k] == b[k], (k, a, b)
    lab = _labels(res)
    mism = np.nonzero(lab != ref.labels)[0]
    assert mism.size == 0, f"{mism.size} labels differ, first at {mism[:5]}"


def _cases():
    return [
        ("sbm10k", graphgen.planted_partition_10k(1), {}),
        ("random_w8", graphgen.random_graph(3000, 0.01, seed=3010, wmax=8), {}),
        ("random_hubs", graphgen.random_graph(1500, 0.25, seed=5, wmax=8), SMALL_TUNING),
        ("rmat13_small", graphgen.rmat_graph(13, 8, "int8"), SMALL_TUNING),
        ("rmat16_i64", graphgen.rmat_graph(16, 16, "int8", np.int64),
         dict(block=1024, hub_chunk=256)),
        ("isolated", graphgen.from_edges(9, [(1, 2), (2, 3), (3, 1), (5, 6), (6, 7)]), {}),
    ]


@pytest.mark.parametrize("sort_rows", [1, 0])
@pytest.mark.parametrize("launch", [lpa.LAUNCH_EAGER, lpa.LAUNCH_GRAPH])
@pytest.mark.parametrize("name,g,tun", _cases(), ids=[c[0] for c in _cases()])
def test_det_parity_internal_order(name, g, tun, launch, sort_rows):
    # internal rows sorted by target (the default) or in the caller's order
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    G = _graph(g, 1, sort_rows=sort_rows, **tun)
    _assert_matches(ref, G.run("det", launch=launch))
    # a second run on the same handle (the captured iteration is replayed)
    _assert_matches(ref, G.run("det", launch=launch))
    G.close()


def test_det_parity_host_arrays_initial_labels_unsorted_rows():
    g = graphgen.rmat_graph(12, 6, "int8")
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    G = _graph(g, 1, on_device=False, **SMALL_TUNING)
    _assert_matches(ref, G.run("det"))
    G.close()
    # initial labels (no identity first sweep)
    init = (np.arange(g.num_vertices) * 7919 % g.num_vertices).astype(np.int32)
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights, initial_labels=init)
    G = _graph(g, 1, **SMALL_TUNING)
    _assert_matches(ref, G.run("det", initial_labels=_dev(init)))
    _assert_matches(ref, G.run("det", initial_labels=init, launch=lpa.LAUNCH_GRAPH))
    G.close()
    # rows in random order: the first sweep takes the table path
    rng = np.random.default_rng(4)
    tgt = g.targets.copy()
    w = g.weights.copy()
    for v in range(g.num_vertices):
        a, b = g.offsets[v], g.offsets[v + 1]
        p = rng.permutation(b - a) + a
        tgt[a:b], w[a:b] = tgt[p], w[p]
    gs = graphgen.Graph(g.offsets.copy(), tgt, w, "shuffled")
    ref = oracle.lpa_sync(gs.offsets, gs.targets, gs.weights)
    G = _graph(gs, 1, **SMALL_TUNING)
    _assert_matches(ref, G.run("det"))
    G.close()


def test_same_labels_in_both_orders_and_options():
    g = graphgen.rmat_graph(15, 9, "int8")
    for kw in (dict(), dict(pl_period=0), dict(prune=0), dict(flag_mode=lpa.FLAGS_PUSH),
               dict(flag_mode=lpa.FLAGS_PULL), dict(tolerance=0.0, max_iterations=7)):
        A = _graph(g, 0)
        B = _graph(g, 1)
        ra, rb = A.run("det", **kw), B.run("det", **kw)
        assert ra.iterations == rb.iterations, kw
        np.testing.assert_array_equal(_labels(ra), _labels(rb))
        for a, b in zip(ra.stats, rb.stats):
            assert (a["changed"], a["processed"], a["edges_scanned"]) == \
                (b["changed"], b["processed"], b["edges_scanned"]), kw
        A.close()
        B.close()


def test_async_invariant_flags_and_modularity():
    for g, tun in ((graphgen.rmat_graph(14, 5, "int8"), {}),
                   (graphgen.rmat_graph(12, 6, "int8"), SMALL_TUNING)):
        G = _graph(g, 1, **tun)
        for fm in (lpa.FLAGS_PUSH, lpa.FLAGS_PULL):
            res = G.run("async", pl_period=0, flag_mode=fm)
            lab = _labels(res)
            flags = G.flags().astype(bool)
            ok = oracle.local_optimal(g.offsets, g.targets, g.weights, lab)
            bad = np.nonzero(~ok & ~flags)[0]
            assert bad.size == 0, f"{bad.size} unflagged vertices hold a non-maximal label"
            q = G.modularity(lab)
            assert q == pytest.approx(oracle.modularity(g.offsets, g.targets, g.weights, lab),
                                      rel=1e-9, abs=1e-12)
        dflags = torch.empty(g.num_vertices, dtype=torch.uint8, device="cuda")
        lpa.lpa_get_flags(G.handle, dflags)
        np.testing.assert_array_equal(dflags.cpu().numpy(), G.flags())
        G.close()


def test_auto_mode_on_a_large_graph():
    # N > 2^20 and R-MAT ids carry no locality: the automatic choice takes
    # the internal order, with the same result as the caller's order
    g = graphgen.rmat_graph(21, 21, "unit")
    A = _graph(g, -1)
    B = _graph(g, 0)
    ra, rb = A.run("det", launch=lpa.LAUNCH_GRAPH), B.run("det", launch=lpa.LAUNCH_GRAPH)
    assert ra.iterations == rb.iterations
    np.testing.assert_array_equal(_labels(ra), _labels(rb))
    A.close()
    B.close()


def _params_history():
    # changed in l-1 or l-2 -> keep; neither -> predicted unchanged
    p = {k: np.zeros(v, dtype=np.float32) for k, v in mlp.PARAM_SHAPES.items()}
    p["W1"][5, 0] = 1.0
    p["W1"][6, 0] = 1.0
    p["W2"][0, 0] = 1.0
    p["W3"][0, 0] = 6.0
    p["b3"][0] = -3.0
    return mlp.flatten(p)


def test_learned_records_and_traces_in_caller_order():
    g = graphgen.rmat_graph(12, 6, "int8")
    params = _params_history()
    zt = float(np.float32(np.log(0.5 / 0.5)))
    ref = oracle.lpa_learned(g.offsets, g.targets, g.weights, params=params, z_theta=zt,
                             fn_bound=1.0, max_pred_degree=SMALL_TUNING["wave"],
                             min_pred_degree=SMALL_TUNING["small16"] + 1, pred_start=2)
    G = _graph(g, 1, **SMALL_TUNING)
    pr = lpa.Predictor(params=params)
    G.set_predictor(pr, threshold=0.5, fn_bound=1.0)
    res = G.run("det", learned=True)
    assert res.iterations == ref.iterations
    np.testing.assert_array_equal(_labels(res), ref.labels)
    for a, b in zip(res.stats, ref.stats):
        assert (a["changed"], a["processed"], a["skipped"]) == \
            (b["changed"], b["processed"], b["skipped"]), (a, b)
    np.testing.assert_array_equal(G.records(), ref.records)
    # traces: sampled by caller id, reported in caller ids
    tref = oracle.lpa_learned(g.offsets, g.targets, g.weights, sample_rate=0.4, seed=11,
                              trace_cap=1_000_000, max_pred_degree=SMALL_TUNING["wave"],
                              min_pred_degree=SMALL_TUNING["small16"] + 1, pred_start=2)
    X, y, v, it, drawn = G.trace(sample_rate=0.4, seed=11, cap=1_000_000)
    assert drawn == tref.trace_total == X.shape[0]
    order = np.lexsort((v, it))
    np.testing.assert_array_equal(it[order], tref.trace["l"])
    np.testing.assert_array_equal(v[order], tref.trace["v"])
    np.testing.assert_array_equal(X[order], tref.trace["X"])
    np.testing.assert_array_equal(y[order], tref.trace["y"])
    np.testing.assert_array_equal(G.records(), tref.records)
    G.close()
    pr.close()


def test_argument_errors():
    g = graphgen.planted_partition_10k(1)
    with pytest.raises(lpa.LpaError):
        _graph(g, 2)
    with pytest.raises(lpa.LpaError):
        _graph(g, -2)
    packed, v_off = graphgen.pack_graphs([g, graphgen.disjoint_cliques(3, 4)])
    with pytest.raises(lpa.LpaError):
        lpa.LpaBatch(v_off, _dev(packed.offsets), _dev(packed.targets), _dev(packed.weights),
                     tuning=_tuning(relabel=1))
    # the default (automatic) and 0 are accepted for batches
    B = lpa.LpaBatch(v_off, _dev(packed.offsets), _dev(packed.targets), _dev(packed.weights))
    B.close()

"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Deterministic mode must equal the oracle exactly (labels, iteration count and
every per-iteration counter) on integer-valued weights.  Asynchronous mode is
judged by invariants: with Pick-Less off, every vertex that is not flagged at
exit holds a label of maximum weight; with Pick-Less on, modularity within
0.01 of the oracle's.  Modularity itself must match the fp64 oracle to 1e-9
relative.
"""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2411_11468_amd import lpa  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _graph_on_gpu(g, tuning=None, on_device=True, weights=True):
    w = g.weights if weights else None
    if on_device:
        return lpa.LpaGraph(_dev(g.offsets), _dev(g.targets),
                            None if w is None else _dev(w), tuning=tuning)
    return lpa.LpaGraph(g.offsets, g.targets, w, tuning=tuning)


def _tuning(**kw):
    t = lpa.default_tuning()
    for k, v in kw.items():
        setattr(t, k, v)
    return t


SMALL_TUNING = dict(small4=2, small16=8, wave=40, block=100, hub_chunk=64)


def assert_det_parity(g, tuning=None, on_device=True, weights=True, initial=None,
                      flag_mode=lpa.FLAGS_AUTO, **kw):
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights if weights else None,
                          initial_labels=initial, **kw)
    G = _graph_on_gpu(g, tuning, on_device, weights)
    init = None if initial is None else (_dev(initial) if on_device else initial)
    res = G.run("det", initial_labels=init, flag_mode=flag_mode, **kw)
    labels = res.labels.cpu().numpy() if on_device else res.labels
    assert res.iterations == ref.iterations
    for s_gpu, s_ref in zip(res.stats, ref.stats):
        for key in ("iteration", "pick_less", "changed", "processed", "edges_scanned"):
            assert s_gpu[key] == s_ref[key], (key, s_gpu, s_ref)
    mism = np.nonzero(labels != ref.labels)[0]
    assert mism.size == 0, f"{mism.size} labels differ, first at {mism[:5]}"
    G.close()
    return ref


def _golden_cases():
    with open(GOLDEN) as f:
        return json.load(f)["lpa_cases"]


def _golden_graph(spec):
    k = spec["kind"]
    if k == "disjoint_cliques":
        return graphgen.disjoint_cliques(spec["r"], spec["s"])
    if k == "complete_bipartite":
        return graphgen.complete_bipartite(spec["n"])
    return graphgen.from_edges(spec["n"], [tuple(e) for e in spec["edges"]])


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
def test_det_hand_derived_cases(case):
    g = _golden_graph(case["graph"])
    G = _graph_on_gpu(g)
    res = G.run("det", pl_period=case["pl_period"], tolerance=case.get("tolerance", 0.05),
                cc_period=case.get("cc_period", 0))
    assert res.iterations == case["iterations"]
    assert res.labels.cpu().tolist() == case["labels"]
    for key in ("changed", "processed", "edges_scanned"):
        if key in case:
            assert [s[key] for s in res.stats] == case[key]


def test_det_planted_partition_10k():
    ref = assert_det_parity(graphgen.planted_partition_10k(1))
    assert ref.iterations >= 3


@pytest.mark.parametrize("n,p,wmax", [(3000, 0.01, 8), (2000, 0.2, 8), (600, 0.9, 3),
                                      (5000, 0.002, 1)])
def test_det_random_graphs(n, p, wmax):
    assert_det_parity(graphgen.random_graph(n, p, seed=n + int(p * 1000), wmax=wmax))


def test_det_every_class_small_thresholds():
    # thresholds shrunk so that a small graph exercises the 4- and 16-lane
    # groups, both wave tables, the workgroup tables and the multi-slice path
    t = _tuning(**SMALL_TUNING)
    g = graphgen.random_graph(1500, 0.25, seed=5, wmax=8)
    G = _graph_on_gpu(g, t)
    cls = G.classes()
    assert cls["hub"] > 0
    G.close()
    assert_det_parity(g, tuning=t)
    r = graphgen.rmat_graph(12, 7, "int8")
    assert_det_parity(r, tuning=t)


@pytest.mark.parametrize("xcd_local", [0, 1, 2, 3])
def test_det_hub_merge_paths(xcd_local):
    # hub buckets merged on one XCD with L2-local atomics, or device-wide
    # only; hub slices taken in target-window groups per XCD, or round-robin
    t = _tuning(**SMALL_TUNING, xcd_local=xcd_local)
    assert_det_parity(graphgen.random_graph(1500, 0.25, seed=5, wmax=8), tuning=t)
    assert_det_parity(graphgen.rmat_graph(13, 8, "int8"), tuning=t)
    t2 = _tuning(block=1024, hub_chunk=256, xcd_local=xcd_local)
    assert_det_parity(graphgen.rmat_graph(16, 16, "int8"), tuning=t2)


def test_det_hub_slice_with_more_labels_than_its_slot_list():
    # a hub of 20,000 leaves whose initial labels are all distinct: its first
    # 8,192-entry slice holds 8,192 labels, more than the slice kernel's list
    # of claimed slots keeps, so that slice reads back its whole table; the
    # leaves are paired up so that they keep moving after the first sweep
    rng = np.random.default_rng(11)
    n = 20001
    edges = [(0, i) for i in range(1, n)] + [(i, i + 1) for i in range(1, n - 1, 2)]
    g = graphgen.from_edges(n, edges)
    init = rng.permutation(n).astype(np.int32)
    assert_det_parity(g, initial=init)
    assert_det_parity(g, tuning=_tuning(xcd_local=0), initial=init)


@pytest.mark.parametrize("cap", [1, 7, 63])
def test_det_hub_spill_path(cap):
    # bucket tables capped far below the labels of a bucket: most labels
    # spill into the hubs' global tables, which must give the same result
    t = _tuning(**SMALL_TUNING, hub_table_cap=cap)
    assert_det_parity(graphgen.random_graph(1500, 0.25, seed=5, wmax=8), tuning=t)
    assert_det_parity(graphgen.rmat_graph(13, 8, "int8"), tuning=t)
    t2 = _tuning(block=1024, hub_chunk=256, hub_table_cap=cap, xcd_local=0)
    assert_det_parity(graphgen.rmat_graph(16, 16, "int8"), tuning=t2)


def _shuffle_rows(g, seed):
    """The same graph with every row's entries in random order."""
    rng = np.random.default_rng(seed)
    off = g.offsets.astype(np.int64)
    row = np.repeat(np.arange(g.num_vertices), np.diff(off))
    order = np.lexsort((rng.random(g.num_edges), row))
    return graphgen.Graph(g.offsets, g.targets[order].copy(), g.weights[order].copy())


def test_det_unsorted_rows_and_repeated_entries():
    # rows that are not strictly increasing take the table path in the first
    # sweep too; repeated entries add their weights
    t = _tuning(**SMALL_TUNING)
    g = graphgen.rmat_graph(13, 8, "int8")
    assert_det_parity(_shuffle_rows(g, 1))
    assert_det_parity(_shuffle_rows(g, 2), tuning=t)
    edges = [(i, (i * 7 + 3) % 300) for i in range(300)] * 3 + [(i, i + 1) for i in range(299)]
    assert_det_parity(graphgen.from_edges(300, edges))
    assert_det_parity(graphgen.from_edges(300, edges), tuning=t)


def test_det_rmat_default_tuning():
    g = graphgen.rmat_graph(15, 15, "int8")
    G = _graph_on_gpu(g)
    cls = G.classes()
    G.close()
    assert cls["small4"] > 0 and cls["wave"] > 0 and cls["block"] > 0
    assert_det_parity(g)


def test_det_int64_offsets_and_host_arrays():
    g = graphgen.rmat_graph(13, 3, "int8")
    g64 = graphgen.Graph(g.offsets.astype(np.int64), g.targets, g.weights)
    assert_det_parity(g64, tuning=_tuning(**SMALL_TUNING))
    assert_det_parity(g64, on_device=False)
    assert_det_parity(g, on_device=False, tuning=_tuning(**SMALL_TUNING))


def test_det_unit_weights_null_pointer():
    g = graphgen.planted_partition_10k(2)
    assert_det_parity(g, weights=False)


@pytest.mark.parametrize("bt,load,pdiv", [(256, 2, 16), (512, 1, 16), (1024, 4, 16),
                                           (0, 1, 1), (0, 4, 4096)])
def test_det_block_shapes_table_loads_and_flag_policy(bt, load, pdiv):
    # the autotuner's axes: threads of the workgroup classes, the table
    # capacity rule (load up to 1, 1/2, 1/4) and the push/pull crossover
    # leave every label and counter unchanged
    for g, tun in ((graphgen.rmat_graph(16, 16, "int8"), {}),
                   (graphgen.random_graph(1500, 0.25, 5, wmax=8), SMALL_TUNING)):
        assert_det_parity(g, _tuning(block_threads=bt, table_load=load, pull_divisor=pdiv,
                                     **tun))


def test_det_options():
    g = graphgen.rmat_graph(12, 9, "int8")
    t = _tuning(**SMALL_TUNING)
    assert_det_parity(g, tuning=t, pl_period=0)
    assert_det_parity(g, tuning=t, pl_period=0, prune=False)
    assert_det_parity(g, tuning=t, pl_period=3, prune=False, max_iterations=7)
    assert_det_parity(g, tuning=t, tolerance=0.0, max_iterations=13)
    rng = np.random.default_rng(3)
    init = rng.integers(0, g.num_vertices, size=g.num_vertices).astype(np.int32)
    assert_det_parity(g, tuning=t, initial=init)
    assert_det_parity(g, tuning=t, initial=init, on_device=False)


@pytest.mark.parametrize("flag_mode", [lpa.FLAGS_PUSH, lpa.FLAGS_PULL])
def test_det_flag_modes(flag_mode):
    # neighbour flags pushed by changed vertices or pulled by every vertex:
    # the same flags, hence the same run, on a symmetric graph
    assert_det_parity(graphgen.planted_partition_10k(1), flag_mode=flag_mode)
    assert_det_parity(graphgen.rmat_graph(14, 3, "int8"), flag_mode=flag_mode)
    assert_det_parity(graphgen.rmat_graph(12, 6, "int8"), tuning=_tuning(**SMALL_TUNING),
                      flag_mode=flag_mode)
    assert_det_parity(graphgen.from_edges(5, [(0, 1), (1, 1), (2, 3)]), flag_mode=flag_mode,
                      pl_period=0)


def test_edge_cases():
    # empty graph
    G = lpa.LpaGraph(_dev(np.zeros(1, np.int32)), _dev(np.zeros(0, np.int32)))
    res = G.run("det")
    assert res.iterations == 0
    assert G.modularity(res.labels) == 0.0
    # vertices without edges, and self-loops only
    for g in (graphgen.from_edges(5, []), graphgen.from_edges(4, [(1, 1), (2, 2)])):
        assert_det_parity(g)
        assert_det_parity(g, pl_period=0)


def test_modularity_matches_oracle():
    rng = np.random.default_rng(9)
    for g in (graphgen.planted_partition_10k(1), graphgen.rmat_graph(14, 4, "int8"),
              graphgen.ring_of_cliques(30, 5)):
        G = _graph_on_gpu(g)
        res = G.run("det")
        labs = [res.labels.cpu().numpy(), np.arange(g.num_vertices, dtype=np.int32),
                np.zeros(g.num_vertices, dtype=np.int32),
                rng.integers(0, 50, size=g.num_vertices).astype(np.int32)]
        for lab in labs:
            want = oracle.modularity(g.offsets, g.targets, g.weights, lab)
            got_dev = G.modularity(_dev(lab))
            got_host = G.modularity(lab)
            assert got_dev == pytest.approx(want, rel=1e-9, abs=1e-12)
            assert got_host == pytest.approx(want, rel=1e-9, abs=1e-12)
        G.close()
    g = graphgen.ring_of_cliques(30, 5)
    G = _graph_on_gpu(g)
    lab = (np.arange(150) // 5).astype(np.int32)
    assert G.modularity(lab) == pytest.approx(20 / 22 - 1 / 30, abs=1e-12)


def _async_invariant(g, tuning=None, seed_runs=2):
    G = _graph_on_gpu(g, tuning)
    for r in range(seed_runs):
        res = G.run("async", pl_period=0, flag_mode=(lpa.FLAGS_PUSH, lpa.FLAGS_PULL)[r % 2])
        lab = res.labels.cpu().numpy()
        flags = G.flags().astype(bool)
        ok = oracle.local_optimal(g.offsets, g.targets, g.weights, lab)
        bad = np.nonzero(~ok & ~flags)[0]
        assert bad.size == 0, f"{bad.size} unflagged vertices hold a non-maximal label"
        for s in res.stats:
            assert 0 <= s["changed"] <= s["processed"] <= g.num_vertices
    G.close()


def test_async_local_optimality_invariant():
    _async_invariant(graphgen.planted_partition_10k(1), seed_runs=4)
    _async_invariant(graphgen.rmat_graph(14, 5, "int8"))
    _async_invariant(graphgen.rmat_graph(12, 6, "int8"), _tuning(**SMALL_TUNING))


def test_async_modularity_band():
    for g, t in ((graphgen.planted_partition_10k(1), None),
                 (graphgen.rmat_graph(15, 8, "int8"), None),
                 (graphgen.rmat_graph(13, 2, "int8"), _tuning(**SMALL_TUNING))):
        ref = oracle.lpa_sync(g.offsets, g.targets, g.weights)
        q_ref = oracle.modularity(g.offsets, g.targets, g.weights, ref.labels)
        G = _graph_on_gpu(g, t)
        res = G.run("async")
        q = oracle.modularity(g.offsets, g.targets, g.weights, res.labels.cpu().numpy())
        assert abs(q - q_ref) <= 0.01, (q, q_ref)
        assert G.modularity(res.labels) == pytest.approx(q, rel=1e-9, abs=1e-12)
        G.close()


def test_invalid_inputs_rejected():
    g = graphgen.from_edges(4, [(0, 1), (1, 2)])
    bad_t = g.targets.copy()
    bad_t[0] = 7
    with pytest.raises(lpa.LpaError):
        lpa.LpaGraph(_dev(g.offsets), _dev(bad_t), _dev(g.weights))
    bad_w = g.weights.copy()
    bad_w[1] = -1.0
    with pytest.raises(lpa.LpaError):
        lpa.LpaGraph(_dev(g.offsets), _dev(g.targets), _dev(bad_w))
    bad_w[1] = -0.0
    with pytest.raises(lpa.LpaError):
        lpa.LpaGraph(_dev(g.offsets), _dev(g.targets), _dev(bad_w))
    bad_o = g.offsets.copy()
    bad_o[2] = 0
    with pytest.raises(lpa.LpaError):
        lpa.LpaGraph(_dev(bad_o), _dev(g.targets), _dev(g.weights))
    for bad in (-1, 4):
        t = lpa.default_tuning()
        t.xcd_local = bad
        with pytest.raises(lpa.LpaError):
            lpa.LpaGraph(_dev(g.offsets), _dev(g.targets), _dev(g.weights), tuning=t)
    G = _graph_on_gpu(g)
    with pytest.raises(lpa.LpaError):
        G.run("det", initial_labels=_dev(np.array([0, 1, 2, 9], np.int32)))
    with pytest.raises(lpa.LpaError):
        G.modularity(np.array([0, -1, 2, 3], np.int32))
    with pytest.raises(lpa.LpaError):
        G.run(mode=7)
    res = G.run("det")  # still usable after rejected calls
    assert res.labels.cpu().tolist() == [0, 0, 0, 3]
    G.close()


def test_det_rmat_scale22_full_size():
    # full-size R-MAT scale 22 with integer weights 1..8 (exact fp32 sums)
    g = graphgen.rmat_graph(22, 22, "int8")
    assert int(g.weights.max()) * int(g.degrees().max()) < 2 ** 24
    assert_det_parity(g)


def test_async_rmat_scale22_full_size():
    # the second configuration in asynchronous mode at its full size, both
    # launch modes: with Pick-Less off every vertex left unflagged holds a
    # label of maximum weight; with Pick-Less every 4th iteration (the
    # configuration's) an unflagged vertex off the maximum must be one whose
    # maximum-weight labels are all larger than its own (a Pick-Less refusal
    # since its last evaluation), and modularity lies within 0.01 of the
    # oracle's deterministic run
    g = graphgen.rmat_graph(22, 22, "int8")
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    q_ref = oracle.modularity(g.offsets, g.targets, g.weights, ref.labels)
    G = _graph_on_gpu(g)
    for launch in (lpa.LAUNCH_EAGER, lpa.LAUNCH_GRAPH):
        for pl in (0, 4):
            res = G.run("async", pl_period=pl, launch=launch)
            lab = res.labels.cpu().numpy()
            flags = G.flags().astype(bool)
            ok = oracle.local_optimal(g.offsets, g.targets, g.weights, lab)
            bad = np.nonzero(~ok & ~flags)[0]
            if pl == 0:
                assert bad.size == 0, f"{bad.size} unflagged vertices off the maximum"
            else:
                refused = oracle.pl_refusable(g.offsets, g.targets, g.weights, lab, bad)
                assert refused.all(), f"{int((~refused).sum())} unflagged vertices off the maximum"
                q = oracle.modularity(g.offsets, g.targets, g.weights, lab)
                assert abs(q - q_ref) <= 0.01, (q, q_ref)
                assert G.modularity(res.labels) == pytest.approx(q, rel=1e-9, abs=1e-12)
            assert 1 <= res.iterations <= 20
            for st in res.stats:
                assert 0 <= st["changed"] <= st["processed"] <= g.num_vertices
    G.close()


def test_profile_books_each_kernel():
    # every class kernel once per iteration; the table-free first sweep
    # under its own names, once per run
    g = graphgen.rmat_graph(12, 6, "int8")
    G = _graph_on_gpu(g, _tuning(**SMALL_TUNING))
    cls = G.classes()
    G.profile_reset()
    res = G.run("det", profile=True)
    prof = {p["name"]: p for p in G.profile()}
    it = res.iterations
    assert it >= 3
    assert prof["frontier"]["launches"] == it
    assert prof["hub_direct"]["launches"] == 1
    assert prof["hub_part"]["launches"] == it - 1
    if cls["small4"]:
        assert prof["direct_small4"]["launches"] == 1
        assert prof["sweep_small4"]["launches"] == it - 1
    for name in ("hub_direct", "hub_part", "direct_small16", "sweep_small16"):
        p = prof[name]
        assert p["total_ms"] > 0 and p["bytes"] > 0 and p["edges"] > 0, p
    G.close()


def test_label_read_rate():
    g = graphgen.rmat_graph(14, 5, "int8")
    for relabel in (0, 1):
        G = _graph_on_gpu(g, _tuning(relabel=relabel))
        r = G.label_read_rate(2)
        assert r > 1e8, r
        # the probe leaves no trace on later runs
        ref = oracle.lpa_sync(g.offsets, g.targets, g.weights)
        assert np.array_equal(G.run("det").labels.cpu().numpy(), ref.labels)
        with pytest.raises(lpa.LpaError):
            G.label_read_rate(0)
        G.close()
    E = _graph_on_gpu(graphgen.from_edges(3, []))
    assert E.label_read_rate(1) == 0.0
    E.close()


@pytest.mark.parametrize("relabel", [0, 1])
def test_final_flags_are_the_neighbours_of_the_last_changes(relabel):
    # the stop iteration's flags are set on demand by lpa_get_flags; they must
    # be exactly the neighbours of the vertices that iteration changed
    g = graphgen.rmat_graph(13, 8, "int8")
    G = _graph_on_gpu(g, _tuning(relabel=relabel, **SMALL_TUNING))
    full = G.run("det")
    flags = G.flags().astype(bool)
    # a second call returns the same flags
    np.testing.assert_array_equal(G.flags().astype(bool), flags)
    k = full.iterations
    assert k >= 2
    before = G.run("det", max_iterations=k - 1).labels.cpu().numpy()
    after = full.labels.cpu().numpy()
    changed = before != after
    assert changed.sum() == full.stats[-1]["changed"]
    rows = np.repeat(np.arange(g.num_vertices), np.diff(g.offsets))
    want = np.zeros(g.num_vertices, dtype=bool)
    np.logical_or.at(want, rows, changed[g.targets])
    np.testing.assert_array_equal(flags, want)
    G.close()


def test_all_ones_weights_read_as_unit_weights():
    # an explicit array of 1.0f gives the NULL-weight run (same labels and
    # counters, no weight bytes in the profile); one other weight does not
    g = graphgen.rmat_graph(13, 8, "unit")
    assert g.weights is not None and np.all(g.weights == 1.0)
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    A = _graph_on_gpu(g)
    B = _graph_on_gpu(g, weights=False)
    for G in (A, B):
        G.profile_reset()
        res = G.run("det", profile=True)
        assert res.iterations == ref.iterations
        np.testing.assert_array_equal(res.labels.cpu().numpy(), ref.labels)
    pa = {p["name"]: p["bytes"] for p in A.profile()}
    pb = {p["name"]: p["bytes"] for p in B.profile()}
    assert pa == pb
    A.close()
    B.close()
    # one undirected edge of weight 2 (both directions)
    w = g.weights.copy()
    rows = np.repeat(np.arange(g.num_vertices), np.diff(g.offsets))
    e = int(np.nonzero(rows != g.targets)[0][0])
    u, v = int(rows[e]), int(g.targets[e])
    back = int(g.offsets[v] + np.nonzero(g.targets[g.offsets[v]:g.offsets[v + 1]] == u)[0][0])
    w[e] = w[back] = 2.0
    g2 = graphgen.Graph(g.offsets, g.targets, w, "one-heavy-edge")
    assert_det_parity(g2)


@pytest.mark.parametrize("probe", [0, 1, 2, 3])
def test_det_probe_sequences(probe):
    # every probe sequence of Sec. 4.2 gives the same tables, hence the
    # oracle's labels and counters, through every class and the hub paths
    t = _tuning(**SMALL_TUNING, probe=probe)
    assert_det_parity(graphgen.random_graph(1500, 0.25, seed=5, wmax=8), tuning=t)
    assert_det_parity(graphgen.rmat_graph(13, 8, "int8"), tuning=t)
    t2 = _tuning(block=1024, hub_chunk=256, hub_table_cap=63, probe=probe, max_retries=4)
    assert_det_parity(graphgen.rmat_graph(14, 16, "int8"), tuning=t2)
    assert_det_parity(graphgen.planted_partition_10k(1), tuning=_tuning(probe=probe))


@pytest.mark.parametrize("relabel", [0, 1])
def test_det_low_degree_lattice(relabel):
    # road-like lattice, mean degree 2.1: mostly the one-lane-per-row class,
    # many tiny communities, degree-0 vertices
    g = graphgen.lowdeg_graph(300, seed=7)
    ref = assert_det_parity(g, tuning=_tuning(relabel=relabel))
    assert ref.iterations >= 5
    _async_invariant(g, _tuning(relabel=relabel))



@pytest.mark.parametrize("relabel", [0, 1])
@pytest.mark.parametrize("pl,cc", [(0, 1), (0, 2), (4, 2), (4, 3), (2, 1)])
def test_det_cross_check(pl, cc, relabel):
    # Cross-Check (Sec. 4.1) alone and in the hybrids with Pick-Less: labels
    # and counters equal the oracle's id-order reading, in both vertex orders
    t = _tuning(relabel=relabel, **SMALL_TUNING)
    for g in (graphgen.random_graph(1500, 0.25, seed=5, wmax=8),
              graphgen.rmat_graph(13, 8, "int8"),
              graphgen.planted_partition_10k(1),
              graphgen.complete_bipartite(40)):
        assert_det_parity(g, tuning=t, pl_period=pl, cc_period=cc)


def test_cross_check_breaks_swaps_and_rejects_unsupported_runs():
    g = graphgen.complete_bipartite(50)
    G = _graph_on_gpu(g)
    plain = G.run("det", pl_period=0)
    assert plain.iterations == 20          # swaps until the cap
    cc = G.run("det", pl_period=0, cc_period=1)
    assert cc.iterations < 20
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=0, cc_period=1)
    np.testing.assert_array_equal(cc.labels.cpu().numpy(), ref.labels)
    a = G.run("async", pl_period=0, cc_period=2)
    assert 1 <= a.iterations <= 20
    for kw in (dict(cc_period=-1), dict(cc_period=1, launch=lpa.LAUNCH_GRAPH)):
        with pytest.raises(lpa.LpaError):
            G.run("det", **kw)
    G.close()

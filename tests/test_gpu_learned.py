"""GPU parity of learned skipping and training traces (liblpa.so through the C
ABI) against the learned-skip oracle (oracle/learned_oracle.c).

Deterministic mode with integer weights is compared exactly: labels, every
per-iteration counter, the skipping history and the state records.  The skip
decision is a floating-point comparison of a logit with a threshold; the
predictors used here are built so that every logit lies at least 0.1 from the
threshold (checked through the oracle's smallest margin), far beyond the
1e-5-scale difference between the MFMA evaluation and the fp64 oracle, so the
two sides must take the same decisions.  Traces are compared as sets of
(iteration, vertex) samples with their features and targets.  Asynchronous
learned runs are judged by the invariants of the plain asynchronous mode.
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
N_H = 64


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _tuning(**kw):
    t = lpa.default_tuning()
    for k, v in kw.items():
        setattr(t, k, v)
    return t


def _gpu_graph(g, tuning=None):
    return lpa.LpaGraph(_dev(g.offsets), _dev(g.targets), _dev(g.weights), tuning=tuning)


def _params(feature_weights: dict, scale: float, bias: float) -> np.ndarray:
    """z = scale * relu(sum_k a_k f_k) + bias, through one unit of each layer
    (exact in bf16 when the a_k, scale are)."""
    p = {k: np.zeros(v, dtype=np.float32) for k, v in mlp.PARAM_SHAPES.items()}
    for k, a in feature_weights.items():
        p["W1"][k, 0] = a
    p["W2"][0, 0] = 1.0
    p["W3"][0, 0] = scale
    p["b3"][0] = bias
    return mlp.flatten(p)


# changed in l-1 or l-2 -> keep; neither -> predicted unchanged (logits -3, 3, 9)
P_HISTORY = _params({5: 1.0, 6: 1.0}, 6.0, -3.0)
# best-own gain of the last evaluation above 7.5/255 of the weight -> keep
P_GAIN = _params({4: 1.0}, 256.0, -7.53)
P_ALWAYS = _params({}, 0.0, -50.0)
P_NEVER = _params({}, 0.0, 50.0)


def _graphs():
    return [
        ("sbm10k", graphgen.planted_partition_10k(1), None),
        ("random_w8", graphgen.random_graph(3000, 0.01, seed=3010, wmax=8), None),
        ("rmat12_small", graphgen.rmat_graph(12, 6, "int8"), SMALL_TUNING),
        ("random_hubs", graphgen.random_graph(3000, 0.033, seed=5, wmax=8), SMALL_TUNING),
    ]


def _max_pred_degree(tuning, predict_large=False):
    # rows of the workgroup classes (wave+1 .. block entries) are predicted
    # only with predict_large; longer rows never
    t = tuning or {}
    return t.get("block", 8192) if predict_large else t.get("wave", 512)


def _min_pred_degree(tuning, predict_small=False):
    # rows of the register classes (at most small16 entries) are predicted
    # only with predict_small
    return 1 if predict_small else (tuning or {}).get("small16", 16) + 1


def _learned_pair(g, tuning, params, *, threshold=0.5, fn_bound=0.02, guard=4, pl_period=4,
                  launch=lpa.LAUNCH_EAGER, mode="det", predict_small=False,
                  predict_large=False, first=2):
    zt = float(np.float32(np.log(threshold / (1 - threshold))))
    ref = oracle.lpa_learned(g.offsets, g.targets, g.weights, params=params, z_theta=zt,
                             pl_period=pl_period, guard=guard, fn_bound=fn_bound,
                             max_pred_degree=_max_pred_degree(tuning, predict_large),
                             min_pred_degree=_min_pred_degree(tuning, predict_small),
                             pred_start=first)
    G = _gpu_graph(g, None if tuning is None else _tuning(**tuning))
    pr = lpa.Predictor(params=params)
    G.set_predictor(pr, threshold=threshold, fn_bound=fn_bound, guard_period=guard,
                    predict_small=predict_small, predict_large=predict_large,
                    first_predicted=first)
    res = G.run(mode, learned=True, pl_period=pl_period, launch=launch)
    return ref, G, pr, res


def _assert_same(ref, G, res):
    assert res.iterations == ref.iterations
    np.testing.assert_array_equal(res.labels.cpu().numpy(), ref.labels)
    for a, b in zip(res.stats, ref.stats):
        for k in ("iteration", "pick_less", "changed", "processed", "edges_scanned", "skipped"):
            assert a[k] == b[k], (k, a, b)
    hist = G.learned_history()
    assert len(hist) == ref.iterations
    for a, b in zip(hist, ref.stats):
        assert (a["skipping"], a["fallback"], a["skipped"], a["predicted"],
                a["false_negatives"]) == (b["skipping"], b["fallback"], b["skipped"],
                                          b["predicted"], b["false_neg"]), (a, b)
    np.testing.assert_array_equal(G.records(), ref.records)


@pytest.mark.parametrize("name,g,tuning", _graphs(), ids=[x[0] for x in _graphs()])
@pytest.mark.parametrize("pname", ["history", "gain"])
@pytest.mark.parametrize("small,large,first", [(False, False, 2), (True, True, 1),
                                               (False, True, 3)])
def test_learned_det_matches_oracle(name, g, tuning, pname, small, large, first):
    params = P_HISTORY if pname == "history" else P_GAIN
    ref, G, pr, res = _learned_pair(g, tuning, params, fn_bound=1.0, predict_small=small,
                                    predict_large=large, first=first)
    deg = np.diff(g.offsets)
    eligible = (deg >= _min_pred_degree(tuning, small)) & (deg <= _max_pred_degree(tuning, large))
    if eligible.sum() > 100:
        assert ref.min_margin > 0.1
        assert any(s["skipped"] > 0 for s in ref.stats)
    _assert_same(ref, G, res)
    G.close()
    pr.close()


@pytest.mark.parametrize("pl_period,guard", [(0, 4), (4, 3), (4, 0)])
def test_learned_det_schedules(pl_period, guard):
    g = graphgen.planted_partition_10k(1)
    ref, G, pr, res = _learned_pair(g, None, P_HISTORY, fn_bound=0.02, guard=guard,
                                    pl_period=pl_period)
    assert ref.min_margin > 0.1
    _assert_same(ref, G, res)
    G.close()
    pr.close()


def test_always_unchanged_falls_back():
    g = graphgen.planted_partition_10k(1)
    ref, G, pr, res = _learned_pair(g, None, P_ALWAYS, fn_bound=0.02, pl_period=0)
    assert any(s["fallback"] for s in ref.stats)
    _assert_same(ref, G, res)
    # and without a fallback bound the skipping alternates to the plain
    # result (every row predicted, so that a skipping iteration does nothing)
    ref2, G2, pr2, res2 = _learned_pair(g, None, P_ALWAYS, fn_bound=1.0, pl_period=0,
                                        predict_small=True, predict_large=True)
    _assert_same(ref2, G2, res2)
    plain = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=0)
    np.testing.assert_array_equal(res2.labels.cpu().numpy(), plain.labels)
    for x in (G, G2, pr, pr2):
        x.close()


def test_never_unchanged_is_the_plain_run():
    g = graphgen.random_graph(3000, 0.01, seed=3010, wmax=8)
    ref, G, pr, res = _learned_pair(g, None, P_NEVER)
    plain = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    assert res.iterations == plain.iterations
    np.testing.assert_array_equal(res.labels.cpu().numpy(), plain.labels)
    _assert_same(ref, G, res)
    G.close()
    pr.close()


def test_learned_graph_launch_matches_eager():
    g = graphgen.planted_partition_10k(1)
    ref, G, pr, res = _learned_pair(g, None, P_HISTORY, launch=lpa.LAUNCH_GRAPH)
    assert res.iterations == ref.iterations
    np.testing.assert_array_equal(res.labels.cpu().numpy(), ref.labels)
    for _ in range(2):   # replays of the captured iteration
        again = G.run("det", learned=True, launch=lpa.LAUNCH_GRAPH)
        np.testing.assert_array_equal(again.labels.cpu().numpy(), ref.labels)
        eager = G.run("det", learned=True)
        np.testing.assert_array_equal(eager.labels.cpu().numpy(), ref.labels)
    G.close()
    pr.close()


@pytest.mark.parametrize("name,g,tuning", _graphs()[:3], ids=[x[0] for x in _graphs()[:3]])
def test_trace_matches_oracle(name, g, tuning):
    ref = oracle.lpa_learned(g.offsets, g.targets, g.weights, sample_rate=1.0,
                             trace_cap=4_000_000, max_pred_degree=_max_pred_degree(tuning),
                             min_pred_degree=_min_pred_degree(tuning), pred_start=2)
    G = _gpu_graph(g, None if tuning is None else _tuning(**tuning))
    X, y, v, it, drawn = G.trace(sample_rate=1.0, cap=4_000_000)
    assert drawn == ref.trace_total == X.shape[0]
    order = np.lexsort((v, it))
    t = ref.trace
    np.testing.assert_array_equal(it[order], t["l"])
    np.testing.assert_array_equal(v[order], t["v"])
    np.testing.assert_array_equal(X[order], t["X"])
    np.testing.assert_array_equal(y[order], t["y"])
    np.testing.assert_array_equal(G.records(), ref.records)
    G.close()


def test_trace_sampling_cap_and_device_buffers():
    g = graphgen.planted_partition_10k(1)
    ref = oracle.lpa_learned(g.offsets, g.targets, g.weights, sample_rate=0.3, seed=77,
                             trace_cap=1_000_000, min_pred_degree=_min_pred_degree(None),
                             max_pred_degree=_max_pred_degree(None), pred_start=2)
    G = _gpu_graph(g)
    X, y, v, it, drawn = G.trace(sample_rate=0.3, seed=77, cap=1_000_000,
                                 device=torch.device("cuda"))
    assert drawn == ref.trace_total
    order = np.lexsort((v.cpu().numpy(), it.cpu().numpy()))
    np.testing.assert_array_equal(v.cpu().numpy()[order], ref.trace["v"])
    np.testing.assert_array_equal(X.cpu().numpy()[order], ref.trace["X"])
    np.testing.assert_array_equal(y.cpu().numpy()[order], ref.trace["y"])
    # capped: the kept samples are drawn samples, the count is the total
    Xc, yc, vc, itc, dc = G.trace(sample_rate=0.3, seed=77, cap=100)
    assert dc == drawn and Xc.shape[0] == 100
    keys = set(zip(ref.trace["l"].tolist(), ref.trace["v"].tolist()))
    assert set(zip(itc.tolist(), vc.tolist())) <= keys
    G.close()


def _async_invariant_learned(g, tuning=None, params=P_HISTORY):
    G = _gpu_graph(g, None if tuning is None else _tuning(**tuning))
    pr = lpa.Predictor(params=params)
    G.set_predictor(pr, threshold=0.5, fn_bound=1.0)
    res = G.run("async", learned=True, pl_period=0)
    lab = res.labels.cpu().numpy()
    flags = G.flags().astype(bool)
    ok = oracle.local_optimal(g.offsets, g.targets, g.weights, lab)
    bad = np.nonzero(~ok & ~flags)[0]
    assert bad.size == 0, f"{bad.size} unflagged vertices hold a non-maximal label"
    assert res.stats[-1]["skipped"] == 0 or res.iterations == 20
    G.close()
    pr.close()
    return res


def test_learned_async_invariants_and_modularity():
    _async_invariant_learned(graphgen.planted_partition_10k(1))
    _async_invariant_learned(graphgen.rmat_graph(12, 6, "int8"), SMALL_TUNING)
    # (On graphs whose vertex ids are not ordered by community, such as the
    # LFR-like ones, the asynchronous mode with ties to the smallest label
    # floods small labels in the first Pick-Less sweep, learned or not; the
    # band against the synchronous oracle holds on id-ordered graphs.)
    for g in (graphgen.planted_partition_10k(1),):
        ref = oracle.lpa_sync(g.offsets, g.targets, g.weights)
        q_ref = oracle.modularity(g.offsets, g.targets, g.weights, ref.labels)
        G = _gpu_graph(g)
        pr = lpa.Predictor(params=P_HISTORY)
        G.set_predictor(pr, threshold=0.5)
        res = G.run("async", learned=True)
        q = oracle.modularity(g.offsets, g.targets, g.weights, res.labels.cpu().numpy())
        # asynchronous order may land higher than the synchronous oracle; it
        # may lose at most 0.01
        assert q_ref - 0.01 <= q <= q_ref + 0.05, (q, q_ref)
        G.close()
        pr.close()


def test_learned_argument_errors():
    g = graphgen.planted_partition_10k(1)
    G = _gpu_graph(g)
    with pytest.raises(lpa.LpaError) as e:
        G.run("det", learned=True)
    assert e.value.status == 4   # LPA_ERR_STATE: no predictor attached
    pr = lpa.Predictor(seed=1)
    for bad in (dict(threshold=0.0), dict(threshold=1.0), dict(fn_bound=-1.0),
                dict(guard_period=-1)):
        with pytest.raises(lpa.LpaError):
            G.set_predictor(pr, **bad)
    G.set_predictor(pr)
    G.set_predictor(None)
    with pytest.raises(lpa.LpaError):
        G.run("det", learned=True)
    with pytest.raises(lpa.LpaError):
        G.trace(sample_rate=1.5)
    G.close()
    graphs = [graphgen.random_graph(50, 0.1, seed=s, wmax=3) for s in range(3)]
    packed, v_off = graphgen.pack_graphs(graphs)
    B = lpa.LpaBatch(v_off, _dev(packed.offsets), _dev(packed.targets), _dev(packed.weights))
    with pytest.raises(lpa.LpaError) as e:
        B.set_predictor(pr)
    assert e.value.status == 5   # LPA_ERR_UNSUPPORTED
    B.close()
    pr.close()


def test_stop_after_a_skip_iteration_matches_oracle():
    K, L = 30, 20
    edges = [(c, K + c * L + i) for c in range(K) for i in range(L)]
    g = graphgen.from_edges(K + K * L, edges)
    ref, G, pr, res = _learned_pair(g, None, P_ALWAYS, fn_bound=1.0, first=1)
    assert ref.iterations == 2 and ref.stats[1]["skipping"] == 1
    _assert_same(ref, G, res)
    G.close()
    pr.close()


def _shuffled(g, seed):
    rng = np.random.default_rng(seed)
    tgt, w = g.targets.copy(), g.weights.copy()
    for v in range(g.num_vertices):
        a, b = g.offsets[v], g.offsets[v + 1]
        p = rng.permutation(b - a) + a
        tgt[a:b], w[a:b] = tgt[p], w[p]
    return graphgen.Graph(g.offsets.copy(), tgt, w, g.name + "-shuffled")


@pytest.mark.parametrize("shuffle", [False, True])
def test_learned_first_sweep_records_both_paths(shuffle):
    # sorted rows: the records of the first sweep come from the table-free
    # kernels; shuffled rows: from the table kernels -- both equal the oracle
    g = graphgen.rmat_graph(12, 6, "int8")
    if shuffle:
        g = _shuffled(g, 3)
    ref, G, pr, res = _learned_pair(g, SMALL_TUNING, P_GAIN, fn_bound=1.0)
    _assert_same(ref, G, res)
    G.close()
    pr.close()

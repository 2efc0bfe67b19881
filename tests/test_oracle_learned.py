"""Pins for the learned-predictor oracle (oracle/learned_oracle.c).  No GPU.

The learned variant is a project addition, so the pins come from its own
definitions and from the plain oracle, which the paper pins:

 * with no predictor, or one that never predicts "unchanged", the run is the
   plain synchronous run of Algorithm 1, statistic by statistic;
 * with a predictor that always predicts "unchanged" and no fallback, every
   skipping iteration does nothing and the plain iterations reproduce the
   plain run in order (Pick-Less off); with the fallback bound the run turns
   plain after the first guard;
 * records after one and two iterations against a brute-force evaluation of
   their definitions (exact rational floors, integer arithmetic);
 * the log quantiser, the feature decoding and the sampling draw against hand
   values and published SplitMix64 outputs;
 * the C network against the numpy network oracle (oracle/mlp.py);
 * traces with sample rate 1 against the run's own statistics.
"""
from fractions import Fraction

import numpy as np
import pytest

import graphgen
import oracle
from oracle import mlp

N_PARAMS = 5057


def _graphs():
    return [
        ("sbm10k", graphgen.planted_partition_10k(1)),
        ("random_w8", graphgen.random_graph(300, 0.03, seed=4, wmax=8)),
        ("rings", graphgen.ring_of_cliques(12, 5)),
        ("random_w3", graphgen.random_graph(500, 0.01, seed=9, wmax=3)),
    ]


def _const_params(b3: float) -> np.ndarray:
    p = np.zeros(N_PARAMS, dtype=np.float32)
    p[-1] = b3
    return p


@pytest.mark.parametrize("name,g", _graphs(), ids=[n for n, _ in _graphs()])
@pytest.mark.parametrize("rho,prune", [(4, True), (0, True), (4, False)])
def test_plain_schedule_is_the_plain_run(name, g, rho, prune):
    want = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=rho, prune=prune)
    for params in (None, _const_params(50.0)):
        got = oracle.lpa_learned(g.offsets, g.targets, g.weights, params=params,
                                 pl_period=rho, prune=prune)
        assert got.iterations == want.iterations
        assert np.array_equal(got.labels, want.labels)
        for a, b in zip(got.stats, want.stats):
            for k in ("pick_less", "changed", "processed", "edges_scanned"):
                assert a[k] == b[k], (k, a["iteration"])
            assert a["skipped"] == 0 and a["predicted"] == 0
            assert a["skipping"] == 0 or params is not None
        if params is not None and got.iterations > 1:
            assert got.min_margin == pytest.approx(50.0)


@pytest.mark.parametrize("name,g", _graphs()[:2], ids=[n for n, _ in _graphs()[:2]])
@pytest.mark.parametrize("tol", [0.05, 0.3])
def test_always_unchanged_without_fallback(name, g, tol):
    want = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=0, tolerance=tol)
    assert want.iterations < 20
    got = oracle.lpa_learned(g.offsets, g.targets, g.weights, params=_const_params(-50.0),
                             pl_period=0, guard=4, fn_bound=1.0, max_iterations=40,
                             tolerance=tol)
    plain = [s for s in got.stats if not s["skipping"]]
    skips = [s for s in got.stats if s["skipping"]]
    for a, b in zip(plain, want.stats):
        for k in ("changed", "processed", "edges_scanned"):
            assert a[k] == b[k]
    k = len(plain)
    assert got.iterations == k + len(skips) and len(skips) <= k
    # a skip follows a plain iteration that changed at least 2 tol N labels
    for s in skips:
        assert got.stats[s["iteration"] - 1]["changed"] >= 2 * tol * g.num_vertices
    if got.stats[-1]["skipping"]:
        # stopped on a skip iteration: its skipped vertices (the plain run's
        # next frontier) were fewer than tolerance * N, so the plain run's
        # next iteration is its last; the labels are those before it
        assert got.stats[-1]["skipped"] < tol * g.num_vertices
        assert k == want.iterations - 1
        before = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=0,
                                 max_iterations=k, tolerance=tol)
        assert np.array_equal(got.labels, before.labels)
    else:
        assert k == want.iterations
        assert np.array_equal(got.labels, want.labels)
    for s in skips:
        # every flagged vertex with a neighbour is skipped and nothing moves
        assert s["changed"] == 0 and s["processed"] == 0
        assert s["skipped"] == got.stats[s["iteration"] + 1]["processed"]
    # every plain iteration after the first predicts all its vertices
    for s in plain[1:]:
        assert s["predicted"] == s["processed"] and s["false_neg"] == s["changed"]


def test_always_unchanged_falls_back_after_the_first_guard():
    g = graphgen.planted_partition_10k(1)
    want = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=0)
    got = oracle.lpa_learned(g.offsets, g.targets, g.weights, params=_const_params(-50.0),
                             pl_period=0, guard=4, fn_bound=0.02)
    s = got.stats
    assert s[1]["skipping"] == 1 and s[1]["processed"] == 0
    assert s[2]["skipping"] == 0 and s[2]["false_neg"] == s[2]["changed"] > 0
    assert s[2]["fallback"] == 1
    assert all(x["skipping"] == 0 for x in s[2:])
    assert got.iterations == want.iterations + 1
    for a, b in zip(s[2:], want.stats[1:]):
        assert (a["changed"], a["processed"]) == (b["changed"], b["processed"])
    assert np.array_equal(got.labels, want.labels)


# ---- records against their definitions -------------------------------------------
def _lq(u: int) -> int:
    e = u.bit_length() - 1
    m = (u >> (e - 3)) & 7 if e >= 3 else (u << (3 - e)) & 7
    return min(255, 8 * e + m)


def _q(x: Fraction, K: Fraction) -> int:
    return 0 if K == 0 else min(255, int((255 * x) // K))


def _brute_records(g, labels, prev_rec, l, processed_mask, moved):
    """Records after evaluating the vertices of processed_mask in iteration l
    with the iteration-start labels `labels` (integer weights)."""
    rec = prev_rec.copy()
    off, tgt = g.offsets.astype(np.int64), g.targets
    w = g.weights
    for i in np.nonzero(processed_mask)[0]:
        d = int(off[i + 1] - off[i])
        if d == 0:
            continue
        sums = {}
        for e in range(off[i], off[i + 1]):
            j = int(tgt[e])
            if j == i:
                continue
            sums[int(labels[j])] = sums.get(int(labels[j]), 0) + Fraction(float(w[e]))
        K = sum(sums.values(), Fraction(0))
        own = sums.get(int(labels[i]), Fraction(0))
        if sums:
            best = min(sums, key=lambda c: (-sums[c], c))
            bw = sums[best]
            second = max([v for c, v in sums.items() if c != best], default=Fraction(0))
        else:
            bw = second = Fraction(0)
        r = rec[i]
        shift = 8 if r[7] == 255 else l - int(r[7])
        h = ((int(r[6]) & 0x7F) << shift if shift < 8 else 0) | int(moved[i])
        r[:] = [_q(own, K), _q(bw - second, K), _q(bw - own, K), (255 * len(sums)) // d,
                _lq(d + 1), _lq(int(K) + 1), h & 0x7F, min(l, 254)]
    return rec


@pytest.mark.parametrize("seed", [4, 5])
def test_records_match_brute_force(seed):
    g = graphgen.random_graph(120, 0.08, seed=seed, wmax=8)
    n = g.num_vertices
    init = np.zeros((n, 8), dtype=np.uint8)
    init[:, 7] = 255
    # iteration 0: every vertex, labels = ids
    one = oracle.lpa_learned(g.offsets, g.targets, g.weights, max_iterations=1)
    s0 = oracle.lpa_sync(g.offsets, g.targets, g.weights, max_iterations=1)
    moved0 = s0.labels != np.arange(n)
    want0 = _brute_records(g, np.arange(n), init, 0, np.ones(n, bool), moved0)
    assert np.array_equal(one.records, want0)
    # iteration 1: the flagged vertices (neighbours of movers), labels of s0
    two = oracle.lpa_learned(g.offsets, g.targets, g.weights, max_iterations=2)
    s1 = oracle.lpa_sync(g.offsets, g.targets, g.weights, max_iterations=2)
    off = g.offsets.astype(np.int64)
    flagged = np.zeros(n, bool)
    for i in np.nonzero(moved0)[0]:
        flagged[g.targets[off[i]:off[i + 1]]] = True
    moved1 = s1.labels != s0.labels
    want1 = _brute_records(g, s0.labels, want0, 1, flagged, moved1)
    assert np.array_equal(two.records, want1)
    assert two.stats[1]["processed"] == int(flagged.sum())


def test_log_quantiser():
    hand = {1: 0, 2: 8, 3: 12, 4: 16, 5: 18, 7: 22, 8: 24, 9: 25, 15: 31, 16: 32,
            17: 32, 18: 33, 1000: 79, 2 ** 31: 248, 2 ** 32 - 1: 255, 2 ** 40: 255}
    for u, q in hand.items():
        assert oracle.log_quant(u, 1.0)[0] == q == _lq(u)
    rng = np.random.default_rng(0)
    for u in list(range(1, 3000)) + [int(x) for x in rng.integers(1, 2 ** 24, 2000)]:
        qi, qf = oracle.log_quant(u, float(u))
        assert qi == _lq(u) == qf, u
    # non-integers: 8 * exponent + the top three mantissa bits
    assert oracle.log_quant(1, 1.5)[1] == 4
    assert oracle.log_quant(1, 2.99)[1] == 8 + 3     # 2.99 = 2 * 1.495
    assert oracle.log_quant(1, 3.99)[1] == 8 + 7     # 3.99 = 2 * 1.995


def test_feature_decoding():
    rec = np.array([51, 102, 0, 255, 64, 72, 0b0000101, 5], dtype=np.uint8)
    f = oracle.record_features(rec, 7, 20, 4)
    # age 2: iteration 6 -> bit -1 (never), 5 -> bit 0, 4 -> bit 1
    want = np.array([1.0, 1.125, 0.2, 0.4, 0.0, 0.0, 1.0, 0.0, 0.35, 0.0, 0.1, 1.0],
                    dtype=np.float32)
    np.testing.assert_array_equal(f, want)
    f8 = oracle.record_features(rec, 8, 20, 4)
    assert f8[9] == 1.0 and f8[5:8].tolist() == [0.0, 0.0, 1.0]
    never = np.array([0, 0, 0, 0, 0, 0, 0, 255], dtype=np.uint8)
    fn = oracle.record_features(never, 3, 20, 0)
    assert fn[5:8].tolist() == [0, 0, 0] and fn[10] == 1.0 and fn[9] == 0.0
    # ages beyond the history window read as unchanged
    old = np.array([0, 0, 0, 0, 0, 0, 0x7F, 0], dtype=np.uint8)
    fo = oracle.record_features(old, 10, 20, 4)
    assert fo[5:8].tolist() == [0, 0, 0] and fo[10] == np.float32(0.5)


def test_sample_draw_is_splitmix64():
    # published SplitMix64 outputs: state 0 -> 0xE220A8397B1DCDAF,
    # 0x6E789E6AA1B965F4, ...; state 1234567 -> 6457827717110365317, ...
    two53 = float(2 ** 53)
    assert oracle.sample_draw(0, 0, 0) == (0xE220A8397B1DCDAF >> 11) / two53
    assert oracle.sample_draw(0, 0, 1) == (0x6E789E6AA1B965F4 >> 11) / two53
    assert oracle.sample_draw(0, 0, 2) == (0x06C45D188009454F >> 11) / two53
    assert oracle.sample_draw(1234567, 0, 0) == (6457827717110365317 >> 11) / two53
    assert oracle.sample_draw(1234567, 0, 3) == (4593380528125082431 >> 11) / two53
    # the iteration enters the counter above bit 32
    assert oracle.sample_draw(0, 1, 0) == oracle.sample_draw(0x9E3779B97F4A7C15 * (1 << 32)
                                                             % 2 ** 64, 0, 0)


def test_network_matches_numpy_oracle():
    rng = np.random.default_rng(3)
    p = mlp.init_params(7)
    for k in ("b1", "b2", "b3"):
        p[k] = (rng.standard_normal(p[k].shape) * 0.2).astype(np.float32)
    flat = mlp.flatten(p)
    X = (rng.standard_normal((64, 12)) * 1.5).astype(np.float32)
    z, _ = mlp.forward(p, X, bf16_h1=True)
    for i in range(X.shape[0]):
        assert oracle.mlp_logit(flat, X[i]) == pytest.approx(z[i], rel=1e-12, abs=1e-12)
    # and it is not the unrounded network
    z_plain, _ = mlp.forward(p, X)
    assert np.max(np.abs(z_plain - z)) > 1e-6


def test_trace_with_full_sampling():
    g = graphgen.random_graph(400, 0.02, seed=2, wmax=4)
    r = oracle.lpa_learned(g.offsets, g.targets, g.weights, sample_rate=1.0, trace_cap=100000)
    deg = np.diff(g.offsets.astype(np.int64))
    tr = r.trace
    assert r.trace_total == tr["X"].shape[0]
    for s in r.stats[1:]:
        sel = tr["l"] == s["iteration"]
        n_isolated = 0  # no degree-0 vertex is flagged after iteration 0
        assert sel.sum() == s["processed"] - n_isolated
        assert tr["y"][sel].sum() == s["changed"]
        np.testing.assert_array_equal(tr["X"][sel, 8],
                                      np.float32(s["iteration"]) / np.float32(20))
    assert (deg[tr["v"]] >= 1).all()
    # capped trace keeps the first samples and reports the total
    c = oracle.lpa_learned(g.offsets, g.targets, g.weights, sample_rate=1.0, trace_cap=10)
    assert c.trace["X"].shape[0] == 10 and c.trace_total == r.trace_total
    np.testing.assert_array_equal(c.trace["X"], tr["X"][:10])
    # partial sampling keeps exactly the vertices whose draw is below the rate
    h = oracle.lpa_learned(g.offsets, g.targets, g.weights, sample_rate=0.25, seed=11,
                           trace_cap=100000)
    keep = np.array([oracle.sample_draw(11, int(l), int(v)) < 0.25
                     for l, v in zip(tr["l"], tr["v"])])
    np.testing.assert_array_equal(h.trace["v"], tr["v"][keep])
    np.testing.assert_array_equal(h.trace["y"], tr["y"][keep])


def test_stop_after_a_skip_iteration():
    # 30 stars, centre ids 0..29 (the smallest), 20 leaves each: the Pick-Less
    # iteration 0 moves every leaf to its centre's label and flags only the
    # 30 centres; the next iteration skips them all (30 < 0.05 N) and the
    # bound changed + skipped < tolerance N ends the run there -- the plain
    # run ends at the same iteration, its centres keeping their labels
    K, L = 30, 20
    edges = [(c, K + c * L + i) for c in range(K) for i in range(L)]
    g = graphgen.from_edges(K + K * L, edges)
    want = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    got = oracle.lpa_learned(g.offsets, g.targets, g.weights, params=_const_params(-50.0),
                             fn_bound=1.0)
    assert want.iterations == 2 and want.stats[1]["changed"] == 0
    assert got.iterations == 2
    s = got.stats[1]
    assert (s["skipping"], s["skipped"], s["processed"], s["changed"]) == (1, K, 0, 0)
    assert np.array_equal(got.labels, want.labels)


@pytest.mark.parametrize("name,g", _graphs(), ids=[n for n, _ in _graphs()])
def test_rows_below_the_predicted_length_are_always_processed(name, g):
    # min_pred_degree k: rows shorter than k are never predicted, skipped or
    # recorded; with an always-"unchanged" predictor and no fallback a
    # skipping iteration skips exactly the flagged rows of >= k entries, and
    # with k above every row length the run is the plain run
    deg = np.diff(g.offsets)
    k = int(np.median(deg[deg > 0])) + 1
    got = oracle.lpa_learned(g.offsets, g.targets, g.weights, params=_const_params(-50.0),
                             pl_period=0, guard=4, fn_bound=1.0, max_iterations=40,
                             min_pred_degree=k)
    short = deg < k
    assert (got.records[short, 7] == 255).all()
    assert (got.records[short, :7] == 0).all()
    for s in got.stats:
        if s["iteration"] >= 1 and s["skipping"]:
            assert s["skipped"] == s["predicted"]
        assert s["predicted"] + s["processed"] >= s["skipped"]
    plain = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=4)
    none = oracle.lpa_learned(g.offsets, g.targets, g.weights, params=_const_params(-50.0),
                              pl_period=4, guard=4, fn_bound=1.0,
                              min_pred_degree=int(deg.max()) + 1)
    assert none.iterations == plain.iterations
    assert np.array_equal(none.labels, plain.labels)
    for a, b in zip(none.stats, plain.stats):
        for key in ("changed", "processed", "edges_scanned"):
            assert a[key] == b[key]
        assert a["skipped"] == 0 and a["predicted"] == 0
    with pytest.raises(ValueError):
        oracle.lpa_learned(g.offsets, g.targets, g.weights, min_pred_degree=0)


def test_predictions_records_and_traces_start_at_pred_start():
    # pred_start k: no prediction (or skip) before iteration k, no record
    # written before iteration k - 1, no trace sample before iteration k
    g = graphgen.planted_partition_10k(1)
    P = _const_params(-50.0)
    k = 3
    r = oracle.lpa_learned(g.offsets, g.targets, g.weights, params=P, pl_period=0, guard=4,
                           fn_bound=1.0, pred_start=k, sample_rate=1.0, trace_cap=4_000_000)
    for s in r.stats[:k]:
        assert s["predicted"] == 0 and s["skipped"] == 0 and not s["skipping"]
    assert any(s["predicted"] > 0 for s in r.stats[k:])
    assert (r.trace["l"] >= k).all() and r.trace["l"].size > 0
    early = oracle.lpa_learned(g.offsets, g.targets, g.weights, params=P, pl_period=0,
                               guard=4, fn_bound=1.0, pred_start=k, max_iterations=k - 1)
    assert (early.records[:, 7] == 255).all()
    at = oracle.lpa_learned(g.offsets, g.targets, g.weights, params=P, pl_period=0,
                            guard=4, fn_bound=1.0, pred_start=k, max_iterations=k)
    ev = at.records[:, 7] != 255
    assert ev.any() and (at.records[ev, 7] == k - 1).all()
    # the first k iterations are those of the plain run
    plain = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=0, max_iterations=k)
    assert np.array_equal(at.labels, plain.labels)
    with pytest.raises(ValueError):
        oracle.lpa_learned(g.offsets, g.targets, g.weights, pred_start=0)

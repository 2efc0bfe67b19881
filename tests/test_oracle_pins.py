"""Pins for the CPU oracle: facts fixed by the paper and by mathematics, not by
the oracle itself.  No GPU needed.

 * hand-derived runs of Algorithm 1 on tiny graphs (tests/golden/closed_forms.json)
 * closed-form modularity (Eq. 1) of clique partitions and special partitions
 * Eq. 1 community form == pair form on random tiny graphs
 * one synchronous sweep == dense brute force of Eq. 3 on every graph with
   up to 5 vertices (and random 6-7 vertex graphs), with and without Pick-Less
 * invariants: pruning changes nothing when Pick-Less is off; Pick-Less
   iterations never raise a label; stats agree with the label history
"""
import itertools
import json
import os

import numpy as np
import pytest

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def _graph(spec):
    k = spec["kind"]
    if k == "disjoint_cliques":
        return graphgen.disjoint_cliques(spec["r"], spec["s"])
    if k == "ring_of_cliques":
        return graphgen.ring_of_cliques(spec["r"], spec["s"])
    if k == "complete_bipartite":
        return graphgen.complete_bipartite(spec["n"])
    if k == "edges":
        return graphgen.from_edges(spec["n"], [tuple(e) for e in spec["edges"]])
    raise ValueError(k)


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("case", _golden()["lpa_cases"], ids=lambda c: c["name"])
def test_hand_derived_lpa_runs(case):
    g = _graph(case["graph"])
    r = oracle.lpa_sync(g.offsets, g.targets, g.weights,
                        tolerance=case.get("tolerance", 0.05),
                        pl_period=case["pl_period"], cc_period=case.get("cc_period", 0))
    assert r.iterations == case["iterations"]
    assert r.labels.tolist() == case["labels"]
    for key in ("changed", "processed", "edges_scanned"):
        if key in case:
            assert [s[key] for s in r.stats] == case[key], key
    if "modularity" in case:
        q = oracle.modularity(g.offsets, g.targets, g.weights, r.labels)
        assert q == pytest.approx(case["modularity"], abs=1e-12)


def _partition(g, spec, kind):
    n = g.num_vertices
    if kind == "cliques":
        return np.arange(n, dtype=np.int32) // spec["s"] * spec["s"]
    if kind == "singletons":
        return np.arange(n, dtype=np.int32)
    if kind == "one":
        return np.zeros(n, dtype=np.int32)
    raise ValueError(kind)


@pytest.mark.parametrize("case", _golden()["modularity_cases"], ids=lambda c: c["name"])
def test_modularity_closed_forms(case):
    g = _graph(case["graph"])
    lab = _partition(g, case["graph"], case["partition"])
    q = oracle.modularity(g.offsets, g.targets, g.weights, lab)
    assert q == pytest.approx(case["q"], abs=1e-12)
    qp = oracle.modularity_pairs(g.offsets, g.targets, g.weights, lab)
    assert qp == pytest.approx(case["q"], abs=1e-12)


def test_clique_closed_form_many_sizes():
    # r disjoint K_s under Pick-Less every 4: two iterations, minimum id per
    # clique, r(s-1) moves in iteration 0, Q = 1 - 1/r.
    for r in (1, 2, 5):
        for s in (3, 4, 7):
            g = graphgen.disjoint_cliques(r, s)
            res = oracle.lpa_sync(g.offsets, g.targets, g.weights)
            assert res.iterations == 2
            assert [x["changed"] for x in res.stats] == [r * (s - 1), 0]
            assert res.labels.tolist() == [(v // s) * s for v in range(r * s)]
            q = oracle.modularity(g.offsets, g.targets, g.weights, res.labels)
            assert q == pytest.approx(1.0 - 1.0 / r, abs=1e-12)


def test_bipartite_closed_form_many_sizes():
    for n in (2, 3, 5, 8):
        g = graphgen.complete_bipartite(n)
        res = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=4)
        assert res.iterations == 3
        assert [x["changed"] for x in res.stats] == [n, n - 1, 0]
        assert res.labels.tolist() == [0] * (2 * n)
        res0 = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=0)
        assert res0.iterations == 20
        assert all(x["changed"] == 2 * n for x in res0.stats)
        assert res0.labels.tolist() == [0] * n + [n] * n


def _ring_clique_q(r, s):
    return s * (s - 1) / (s * (s - 1) + 2) - 1.0 / r


def test_ring_of_cliques_modularity_formula():
    for r in (3, 4, 10, 30):
        for s in (3, 5, 6):
            g = graphgen.ring_of_cliques(r, s)
            lab = np.arange(r * s, dtype=np.int32) // s
            q = oracle.modularity(g.offsets, g.targets, g.weights, lab)
            assert q == pytest.approx(_ring_clique_q(r, s), abs=1e-12)


def _random_tiny(n, p, rng, wmax=3, self_loops=False):
    edges, ws = [], []
    for u in range(n):
        for v in range(u + 1, n):
            if rng.random() < p:
                edges.append((u, v))
                ws.append(float(rng.integers(1, wmax + 1)))
        if self_loops and rng.random() < 0.3:
            edges.append((u, u))
            ws.append(float(rng.integers(1, wmax + 1)))
    return graphgen.from_edges(n, edges, ws)


def test_modularity_forms_agree_random():
    rng = np.random.default_rng(7)
    for _ in range(200):
        n = int(rng.integers(1, 12))
        g = _random_tiny(n, 0.4, rng, self_loops=True)
        lab = rng.integers(0, n, size=n).astype(np.int32)
        q1 = oracle.modularity(g.offsets, g.targets, g.weights, lab)
        q2 = oracle.modularity_pairs(g.offsets, g.targets, g.weights, lab)
        assert q1 == pytest.approx(q2, abs=1e-12)
        if g.num_edges:
            assert -0.5 - 1e-12 <= q1 <= 1.0 + 1e-12


def _dense(g):
    n = g.num_vertices
    W = np.zeros((n, n))
    off = g.offsets.astype(np.int64)
    for i in range(n):
        for e in range(off[i], off[i + 1]):
            W[i, g.targets[e]] += g.weights[e]
    return W


def _brute_step(W, C, pick_less):
    """One synchronous sweep by enumerating every candidate label: for each
    vertex, sum the weight towards each label in [0, n) over neighbours j != i
    (dense matrix), take the largest sum, smallest label on ties."""
    n = W.shape[0]
    out = C.copy()
    for i in range(n):
        has_nb = any(W[i, j] > 0 for j in range(n) if j != i)
        if not has_nb:
            continue
        best_c, best_s = None, -1.0
        for c in range(n):
            s = sum(W[i, j] for j in range(n) if j != i and C[j] == c)
            present = any(W[i, j] > 0 and C[j] == c for j in range(n) if j != i)
            if present and s > best_s:
                best_c, best_s = c, s
        if best_c != C[i] and (not pick_less or best_c < C[i]):
            out[i] = best_c
    return out


def _graphs_upto(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield [pairs[k] for k in range(len(pairs)) if mask >> k & 1]


def test_one_sweep_equals_brute_force_exhaustive():
    rng = np.random.default_rng(11)
    count = 0
    for n in range(1, 6):
        for edges in _graphs_upto(n):
            ws = [float(rng.integers(1, 4)) for _ in edges]
            g = graphgen.from_edges(n, edges, ws)
            W = _dense(g)
            C0 = rng.integers(0, n, size=n).astype(np.int32)
            for pl in (0, 1):
                res = oracle.lpa_sync(g.offsets, g.targets, g.weights, max_iterations=1,
                                      pl_period=pl, initial_labels=C0)
                want = _brute_step(W, C0, pick_less=(pl == 1))
                assert res.labels.tolist() == want.tolist(), (n, edges, ws, C0, pl)
                assert res.stats[0]["changed"] == int((want != C0).sum())
            count += 1
    assert count == 1 + 2 + 8 + 64 + 1024


def test_one_sweep_equals_brute_force_random_larger():
    rng = np.random.default_rng(12)
    for _ in range(300):
        n = int(rng.integers(6, 9))
        g = _random_tiny(n, float(rng.uniform(0.2, 0.8)), rng, wmax=4, self_loops=True)
        W = _dense(g)
        C0 = rng.integers(0, n, size=n).astype(np.int32)
        for pl in (0, 1):
            res = oracle.lpa_sync(g.offsets, g.targets, g.weights, max_iterations=1,
                                  pl_period=pl, initial_labels=C0)
            assert res.labels.tolist() == _brute_step(W, C0, pl == 1).tolist()


def test_multi_sweep_equals_repeated_brute_force():
    # Without pruning, k sweeps of the oracle = k brute-force sweeps, with
    # Pick-Less exactly on sweeps 0, 4, 8, ... (counting from 0).
    rng = np.random.default_rng(13)
    for _ in range(60):
        n = int(rng.integers(3, 9))
        g = _random_tiny(n, 0.5, rng, wmax=3)
        W = _dense(g)
        C = np.arange(n, dtype=np.int32)
        res = oracle.lpa_sync(g.offsets, g.targets, g.weights, max_iterations=9,
                              pl_period=4, prune=False, tolerance=-1.0)
        assert res.iterations == 9
        for l in range(9):
            C = _brute_step(W, C, pick_less=(l % 4 == 0))
            assert res.stats[l]["pick_less"] == int(l % 4 == 0)
        assert res.labels.tolist() == C.tolist()


def _planted():
    return graphgen.planted_partition_10k(1)


def test_pruning_is_exact_without_pick_less():
    # A vertex none of whose neighbours changed has the same neighbourhood as
    # when it last chose, so skipping it changes nothing (Sec. 4 item 4).
    graphs = [_planted(), graphgen.random_graph(500, 0.02, 3, wmax=8),
              graphgen.rmat_graph(10, 4, "int8")]
    for g in graphs:
        a = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=0, prune=True)
        b = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=0, prune=False)
        assert a.iterations == b.iterations
        assert np.array_equal(a.labels, b.labels)
        assert [s["changed"] for s in a.stats] == [s["changed"] for s in b.stats]
        assert all(x["processed"] <= y["processed"] for x, y in zip(a.stats, b.stats))


def test_stats_and_pick_less_invariants():
    g = graphgen.rmat_graph(11, 5, "int8")
    n = g.num_vertices
    deg = g.degrees()
    prev = np.arange(n, dtype=np.int32)
    full = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    F = np.ones(n, dtype=bool)
    for k in range(1, full.iterations + 1):
        r = oracle.lpa_sync(g.offsets, g.targets, g.weights, max_iterations=k, tolerance=-1.0)
        s = r.stats[k - 1]
        assert s == full.stats[k - 1]
        changed = r.labels != prev
        assert s["changed"] == int(changed.sum())
        assert s["processed"] == int(F.sum())
        assert s["edges_scanned"] == int(deg[F].sum())
        assert not np.any(changed & ~F)  # only processed vertices move
        if s["pick_less"]:
            assert np.all(r.labels[changed] < prev[changed])
        # next frontier: neighbours of changed vertices
        nf = np.zeros(n, dtype=bool)
        off = g.offsets.astype(np.int64)
        for i in np.nonzero(changed)[0]:
            nf[g.targets[off[i]:off[i + 1]]] = True
        F = nf
        prev = r.labels
    assert full.stats[0]["processed"] == n


def test_labels_are_neighbour_labels_and_runs_deterministic():
    g = _planted()
    a = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    b = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    assert np.array_equal(a.labels, b.labels) and a.stats == b.stats
    assert 0.5 < oracle.modularity(g.offsets, g.targets, g.weights, a.labels) < 0.8


def test_local_optimal_checker():
    g = graphgen.disjoint_cliques(2, 4)
    good = np.array([0, 0, 0, 0, 4, 4, 4, 4], dtype=np.int32)
    assert oracle.local_optimal(g.offsets, g.targets, g.weights, good).all()
    bad = good.copy()
    bad[1] = 4
    ok = oracle.local_optimal(g.offsets, g.targets, g.weights, bad)
    assert not ok[1] and ok[0]


def test_empty_graph():
    off = np.zeros(1, dtype=np.int32)
    r = oracle.lpa_sync(off, np.zeros(0, np.int32), np.zeros(0, np.float32))
    assert r.iterations == 0 and r.labels.size == 0


def test_philox_known_answers():
    # Known-answer vectors published with the Random123 library.
    assert graphgen.philox4x32_10([0, 0, 0, 0], [0, 0]).tolist() == \
        [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]
    assert graphgen.philox4x32_10([0xffffffff] * 4, [0xffffffff] * 2).tolist() == \
        [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]
    assert graphgen.philox4x32_10([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344],
                                  [0xa4093822, 0x299f31d0]).tolist() == \
        [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]


def test_generators_shapes():
    g = _planted()
    assert g.num_vertices == 10000
    d = g.degrees()
    assert 19.0 < d.mean() < 21.0
    off = g.offsets.astype(np.int64)
    for i in range(0, 10000, 97):
        row = g.targets[off[i]:off[i + 1]]
        assert np.all(np.diff(row) > 0) and i not in row
    # symmetry
    src = np.repeat(np.arange(10000), d)
    fwd = set(zip(src.tolist(), g.targets.tolist()))
    assert all((v, u) in fwd for (u, v) in list(fwd)[:5000])
    r = graphgen.rmat_graph(12, 1, "int8")
    assert r.weights.min() >= 1 and r.weights.max() <= 8
    r2 = graphgen.rmat_graph(12, 1, "int8")
    assert np.array_equal(r.targets, r2.targets) and np.array_equal(r.weights, r2.weights)


def test_cross_check_properties():
    # Sec. 4.1 Cross-Check: with the period 0 it is the plain run; a run with
    # it never changes more vertices in an iteration than the changes it
    # starts from; on the swap-prone inputs (single edge, path, K3,3) it
    # converges where the plain run swaps until the cap
    rng = np.random.default_rng(41)
    for trial in range(60):
        n = int(rng.integers(2, 40))
        g = graphgen.random_graph(n, float(rng.uniform(0.05, 0.5)), seed=trial, wmax=3)
        a = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=4)
        b = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=4, cc_period=0)
        assert np.array_equal(a.labels, b.labels) and a.stats == b.stats
        # one Cross-Check iteration from the same labels: its kept changes are
        # a subset of the plain iteration's changes
        start = rng.integers(0, n, n).astype(np.int32)
        p1 = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=0, max_iterations=1,
                             initial_labels=start, tolerance=-1.0)
        c1 = oracle.lpa_sync(g.offsets, g.targets, g.weights, pl_period=0, max_iterations=1,
                             initial_labels=start, tolerance=-1.0, cc_period=1)
        kept = c1.labels != start
        assert np.all(c1.labels[kept] == p1.labels[kept])
        assert c1.stats[0]["changed"] == int(kept.sum()) <= p1.stats[0]["changed"]
        # the first kept change (lowest id) saw a leader holding its label,
        # and every revert restored the starting label
        moved = p1.labels != start
        assert np.all(c1.labels[moved & ~kept] == start[moved & ~kept])
        if kept.any():
            i = int(np.nonzero(kept)[0][0])
            c = int(c1.labels[i])
            # vertex c is either below i (final) or above (its plain move)
            lab_c = c1.labels[c] if c < i else p1.labels[c]
            assert lab_c == c


def test_pl_refusable_hand_cases_and_pick_less_sweeps():
    # a star 0 - {1, 2, 3}: the centre's neighbour labels 5, 5, 7 sum to
    # {5: 2, 7: 1}; its maximum (5) lies above 0 and below 6
    g = graphgen.from_edges(4, [(0, 1), (0, 2), (0, 3)])
    assert oracle.pl_refusable(g.offsets, g.targets, g.weights,
                               np.array([0, 5, 5, 7], np.int32), [0]).tolist() == [True]
    assert oracle.pl_refusable(g.offsets, g.targets, g.weights,
                               np.array([6, 5, 5, 7], np.int32), [0]).tolist() == [False]
    # tied maxima {3, 9}: refusable only when both lie above the own label
    g = graphgen.from_edges(3, [(0, 1), (0, 2)])
    for own, want in ((2, True), (5, False), (10, False)):
        lab = np.array([own, 3, 9], np.int32)
        assert oracle.pl_refusable(g.offsets, g.targets, g.weights, lab, [0]).tolist() == [want]
    # against Algorithm 1: in one Pick-Less sweep a vertex off the maximum
    # keeps its label exactly when it is refusable
    rng = np.random.default_rng(7)
    for t in range(40):
        g = graphgen.random_graph(30, 0.2, 100 + t, wmax=4)
        lab = rng.integers(0, 30, 30).astype(np.int32)
        one = oracle.lpa_sync(g.offsets, g.targets, g.weights, tolerance=0.0, max_iterations=1,
                              pl_period=1, initial_labels=lab).labels
        ok = oracle.local_optimal(g.offsets, g.targets, g.weights, lab)
        off_max = np.nonzero(~ok)[0]
        ref = oracle.pl_refusable(g.offsets, g.targets, g.weights, lab, off_max)
        assert np.array_equal(ref, one[off_max] == lab[off_max]), t


def test_cpu_async_baseline_results():
    # the multi-core CPU baseline (not the oracle): disjoint cliques end with
    # one label per clique, Q = 1 - 1/r; on the planted partition every label
    # names a vertex, the run stops within the cap and finds the planted
    # structure (its in-place order, 1024 vertices per thread and step in id
    # order, ends near Q 0.69 where the synchronous oracle reaches 0.75)
    for r_, s_ in ((6, 5), (20, 4)):
        g = graphgen.disjoint_cliques(r_, s_)
        res = oracle.cpu_lpa_async(g.offsets, g.targets, g.weights)
        q = oracle.modularity(g.offsets, g.targets, g.weights, res.labels)
        assert q == pytest.approx(1 - 1 / r_, abs=1e-12)
        assert res.iterations <= 20 and res.threads >= 1
    g = _planted()
    res = oracle.cpu_lpa_async(g.offsets, g.targets, g.weights)
    assert ((res.labels >= 0) & (res.labels < g.num_vertices)).all()
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    q = oracle.modularity(g.offsets, g.targets, g.weights, res.labels)
    assert q >= 0.6 and q <= oracle.modularity(g.offsets, g.targets, g.weights, ref.labels) + 0.05
    assert 1 <= res.iterations <= 20

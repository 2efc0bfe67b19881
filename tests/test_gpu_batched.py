"""GPU parity of batched runs and of graph-captured iterations.

Batched, deterministic mode: for every graph of the batch, labels minus the
graph's vertex offset, the iteration count and the changed count of its last
iteration equal a solo run of the oracle on that graph.  Graph launch: the
same run as eager launch, replayed several times with eager work between."""
import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2411_11468_amd import lpa  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _mixed_graphs():
    gs = [graphgen.disjoint_cliques(3, 4), graphgen.complete_bipartite(3),
          graphgen.from_edges(1, []), graphgen.from_edges(2, [(0, 1)]),
          graphgen.from_edges(4, [(1, 1), (2, 3)]),
          graphgen.planted_partition_10k(3), graphgen.random_graph(700, 0.3, 9, wmax=8),
          graphgen.rmat_graph(12, 4, "int8"), graphgen.from_edges(3, [])]
    return gs


def _solo(g, **kw):
    return oracle.lpa_sync(g.offsets, g.targets, g.weights, **kw)


def _check_batch(graphs, tuning=None, launch=lpa.LAUNCH_GRAPH, **kw):
    packed, v_off = graphgen.pack_graphs(graphs)
    B = lpa.LpaBatch(v_off, _dev(packed.offsets), _dev(packed.targets), _dev(packed.weights),
                     tuning=tuning)
    res = B.run_batched("det", launch=launch, **kw)
    lab = res.labels.cpu().numpy()
    for q, g in enumerate(graphs):
        ref = _solo(g, **kw)
        got = lab[v_off[q]:v_off[q + 1]] - v_off[q]
        assert np.array_equal(got, ref.labels), q
        assert res.iters_per_graph[q] == ref.iterations, (q, res.iters_per_graph[q], ref.iterations)
        want_last = ref.stats[-1]["changed"] if ref.stats else 0
        assert res.changed_last[q] == want_last, q
    assert res.iterations == max(1, int(res.iters_per_graph.max()))
    B.close()


@pytest.mark.parametrize("launch", [lpa.LAUNCH_EAGER, lpa.LAUNCH_GRAPH])
def test_batched_equals_solo_runs(launch):
    _check_batch(_mixed_graphs(), launch=launch)


def test_batched_options_and_classes():
    t = lpa.default_tuning()
    t.small4, t.small16, t.wave, t.block, t.hub_chunk = 2, 8, 40, 100, 64
    _check_batch(_mixed_graphs()[5:], tuning=t)
    _check_batch(_mixed_graphs(), pl_period=0)
    _check_batch(_mixed_graphs(), pl_period=3, max_iterations=7)


def test_batched_generated_planted_partitions():
    g, v_off = graphgen.planted_partition_batch(48, 11, n_range=(64, 3000))
    graphs = []
    for q in range(48):
        a, b = v_off[q], v_off[q + 1]
        o = g.offsets[a:b + 1] - g.offsets[a]
        t = g.targets[g.offsets[a]:g.offsets[b]] - a
        graphs.append(graphgen.Graph(o.astype(np.int64), t.astype(np.int32),
                                     g.weights[g.offsets[a]:g.offsets[b]]))
    _check_batch(graphs)


def test_batched_rejects_cross_graph_edges():
    packed, v_off = graphgen.pack_graphs([graphgen.from_edges(2, [(0, 1)]),
                                          graphgen.from_edges(2, [(0, 1)])])
    t = packed.targets.copy()
    t[0] = 3  # vertex 0 (graph 0) -> vertex 3 (graph 1)
    with pytest.raises(lpa.LpaError):
        lpa.LpaBatch(v_off, _dev(packed.offsets), _dev(t), _dev(packed.weights))
    with pytest.raises(lpa.LpaError):
        lpa.LpaBatch(np.array([0, 1, 3]), _dev(packed.offsets), _dev(packed.targets))


@pytest.mark.parametrize("mode", ["det", "async"])
def test_graph_launch_replays_match_eager(mode):
    g = graphgen.rmat_graph(14, 21, "int8")
    G = lpa.LpaGraph(_dev(g.offsets), _dev(g.targets), _dev(g.weights))
    eager = G.run(mode, launch=lpa.LAUNCH_EAGER)
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    q_ref = oracle.modularity(g.offsets, g.targets, g.weights, ref.labels)
    if mode == "det":
        assert np.array_equal(eager.labels.cpu().numpy(), ref.labels)
    for rep in range(3):
        res = G.run(mode, launch=lpa.LAUNCH_GRAPH)
        if mode == "det":
            assert res.iterations == eager.iterations
            assert np.array_equal(res.labels.cpu().numpy(), eager.labels.cpu().numpy()), rep
            for a, b in zip(res.stats, eager.stats):
                for k in ("iteration", "pick_less", "changed", "processed", "edges_scanned"):
                    assert a[k] == b[k], (rep, k)
        else:
            # each replay: Pick-Less refusals aside (labels above the
            # vertex's own), every unflagged vertex holds a label of maximum
            # weight, and modularity lies within 0.01 of the oracle's
            flags = G.flags().astype(bool)
            lab = res.labels.cpu().numpy()
            assert 1 <= res.iterations <= 20
            ok = oracle.local_optimal(g.offsets, g.targets, g.weights, lab)
            bad = np.nonzero(~ok & ~flags)[0]
            assert oracle.pl_refusable(g.offsets, g.targets, g.weights, lab, bad).all(), (rep, bad[:5])
            q = oracle.modularity(g.offsets, g.targets, g.weights, lab)
            assert abs(q - q_ref) <= 0.01, (rep, q, q_ref)
            assert G.modularity(res.labels) == pytest.approx(q, rel=1e-9, abs=1e-12)
        # eager work between replays
        e2 = G.run(mode, launch=lpa.LAUNCH_EAGER, pl_period=0, max_iterations=3)
        assert e2.iterations <= 3
    G.close()


@pytest.fixture(scope="module")
def batch8k():
    # the batched configuration at its full size: 8,192 planted partitions
    # (vertex counts log-uniform in [256, 65536], seed 5), the benchmark's
    # batch and handle
    g, v_off = graphgen.planted_partition_batch(8192, 5)
    B = lpa.LpaBatch(v_off, _dev(g.offsets), _dev(g.targets), _dev(g.weights))
    sizes = np.diff(v_off)
    rng = np.random.default_rng(5)
    pick = np.unique(np.concatenate([rng.choice(len(sizes), 256, replace=False),
                                     np.argsort(sizes, kind="stable")[-8:]]))
    refs = {}
    for q in pick:
        a, b = int(v_off[q]), int(v_off[q + 1])
        ea, eb = int(g.offsets[a]), int(g.offsets[b])
        refs[int(q)] = oracle.lpa_sync(g.offsets[a:b + 1] - ea, g.targets[ea:eb] - a,
                                       g.weights[ea:eb])
    yield g, v_off, B, refs
    B.close()


@pytest.mark.parametrize("launch", [lpa.LAUNCH_EAGER, lpa.LAUNCH_GRAPH])
def test_batched_full_size_sampled_graphs_equal_oracle(batch8k, launch):
    # one deterministic batched run over all 8,192 graphs; 256 graphs drawn
    # at random and the 8 largest equal their solo oracle runs (labels,
    # iteration count, last iteration's changed count)
    g, v_off, B, refs = batch8k
    res = B.run_batched("det", launch=launch)
    lab = res.labels.cpu().numpy()
    assert int(np.diff(v_off).max()) > 60000
    for q, ref in refs.items():
        got = lab[v_off[q]:v_off[q + 1]] - v_off[q]
        mism = np.nonzero(got != ref.labels)[0]
        assert mism.size == 0, (q, mism.size, mism[:5])
        assert res.iters_per_graph[q] == ref.iterations, (q, res.iters_per_graph[q], ref.iterations)
        assert res.changed_last[q] == ref.stats[-1]["changed"], q
    assert res.iterations == int(res.iters_per_graph.max())

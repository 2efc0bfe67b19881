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


def _queue_graphs():
    # rows of at most 512 entries (the work queue's limit): rows of 1..64
    # entries for the 16-lane groups, up to 465 for the wave path
    gs = _mixed_graphs()
    gs[7] = graphgen.rmat_graph(10, 4, "int8")
    return gs


def _queue_tuning(chunk=64, group=64, queue=1):
    t = lpa.default_tuning()
    t.batch_queue, t.queue_chunk, t.queue_group = queue, chunk, group
    return t


@pytest.mark.parametrize("launch", [lpa.LAUNCH_EAGER, lpa.LAUNCH_GRAPH])
@pytest.mark.parametrize("chunk,group", [(64, 64), (256, 16), (1024, 32)])
def test_batched_work_queue_equals_solo_runs(launch, chunk, group):
    # the persistent work-queue kernel: graphs of several chunks, rows on
    # both the 16-lane and the wave path
    _check_batch(_queue_graphs(), tuning=_queue_tuning(chunk, group), launch=launch)


def test_batched_work_queue_options():
    t = _queue_tuning()
    _check_batch(_queue_graphs(), tuning=t, pl_period=0)
    _check_batch(_queue_graphs(), tuning=t, pl_period=3, max_iterations=7)
    _check_batch(_queue_graphs(), tuning=t, max_iterations=1)
    # prune = 0 takes the class kernels on the same handle
    _check_batch(_queue_graphs(), tuning=t, prune=False)
    g, v_off = graphgen.planted_partition_batch(48, 11, n_range=(64, 3000))
    graphs = [_sub(g, v_off, q) for q in range(48)]
    _check_batch(graphs, tuning=_queue_tuning(128, 48))


def test_batched_work_queue_rejects_long_rows_and_auto_choice():
    packed, v_off = graphgen.pack_graphs(_mixed_graphs())  # a row of 1331 entries
    with pytest.raises(lpa.LpaError):
        lpa.LpaBatch(v_off, _dev(packed.offsets), _dev(packed.targets), _dev(packed.weights),
                     tuning=_queue_tuning())
    # automatic: that batch stays on the class kernels, whose flags are readable
    B = lpa.LpaBatch(v_off, _dev(packed.offsets), _dev(packed.targets), _dev(packed.weights))
    B.run_batched("det")
    assert B.flags().shape == (packed.num_vertices,)
    B.close()


@pytest.mark.parametrize("chunk", [64, 512])
def test_batched_work_queue_final_flags(chunk):
    # after a deterministic work-queue run every graph's flags are those its
    # last iteration set: the rows of the vertices it changed (Algorithm 1)
    graphs = _queue_graphs()
    packed, v_off = graphgen.pack_graphs(graphs)
    B = lpa.LpaBatch(v_off, _dev(packed.offsets), _dev(packed.targets), _dev(packed.weights),
                     tuning=_queue_tuning(chunk))
    res = B.run_batched("det")
    flags = B.flags().astype(bool)
    for q, g in enumerate(graphs):
        k = int(res.iters_per_graph[q])
        want = np.zeros(g.num_vertices, dtype=bool)
        if k > 0:
            a = oracle.lpa_sync(g.offsets, g.targets, g.weights, max_iterations=k - 1).labels \
                if k > 1 else np.arange(g.num_vertices, dtype=np.int32)
            b = oracle.lpa_sync(g.offsets, g.targets, g.weights, max_iterations=k).labels
            for i in np.nonzero(a != b)[0]:
                want[g.targets[g.offsets[i]:g.offsets[i + 1]]] = True
        got = flags[v_off[q]:v_off[q + 1]]
        assert np.array_equal(got, want), (q, int((got != want).sum()))
    B.close()


def test_batched_work_queue_async_invariants():
    # asynchronous work-queue runs, judged as asynchronous runs are: every
    # vertex left unflagged holds a label of maximum weight unless Pick-Less
    # refused its move (all maximal labels above its own), labels stay in
    # their graph, and modularity is no more than 0.01 below the oracle's
    # synchronous result.  The band is one-sided: the queue takes a chunk's
    # vertices in order with labels updated in place, which on planted
    # partitions ends 0.01-0.02 above the synchronous oracle
    g, v_off = graphgen.planted_partition_batch(64, 12, n_range=(256, 4000))
    graphs = [_sub(g, v_off, q) for q in range(64)]
    ref = np.concatenate([oracle.lpa_sync(x.offsets, x.targets, x.weights).labels + v_off[q]
                          for q, x in enumerate(graphs)])
    q_ref = oracle.modularity(g.offsets, g.targets, g.weights, ref)
    for launch in (lpa.LAUNCH_EAGER, lpa.LAUNCH_GRAPH):
        B = lpa.LpaBatch(v_off, _dev(g.offsets), _dev(g.targets), _dev(g.weights),
                         tuning=_queue_tuning(256))
        res = B.run_batched("async", launch=launch)
        lab = res.labels.cpu().numpy()
        for q in range(64):
            part = lab[v_off[q]:v_off[q + 1]]
            assert ((part >= v_off[q]) & (part < v_off[q + 1])).all(), q
        assert (res.iters_per_graph >= 1).all() and (res.iters_per_graph <= 20).all()
        flags = B.flags().astype(bool)
        ok = oracle.local_optimal(g.offsets, g.targets, g.weights, lab)
        bad = np.nonzero(~ok & ~flags)[0]
        assert oracle.pl_refusable(g.offsets, g.targets, g.weights, lab, bad).all(), bad[:5]
        q = oracle.modularity(g.offsets, g.targets, g.weights, lab)
        assert q >= q_ref - 0.01, (q, q_ref)
        assert B.modularity(res.labels) == pytest.approx(q, rel=1e-9, abs=1e-12)
        B.close()


def test_batched_options_and_classes():
    t = lpa.default_tuning()
    t.small4, t.small16, t.wave, t.block, t.hub_chunk = 2, 8, 40, 100, 64
    _check_batch(_mixed_graphs()[5:], tuning=t)
    _check_batch(_mixed_graphs(), pl_period=0)
    _check_batch(_mixed_graphs(), pl_period=3, max_iterations=7)


def _sub(g, v_off, q):
    """Graph q of a packed batch, in its own numbering."""
    a, b = v_off[q], v_off[q + 1]
    o = g.offsets[a:b + 1] - g.offsets[a]
    t = g.targets[g.offsets[a]:g.offsets[b]] - a
    return graphgen.Graph(o.astype(np.int64), t.astype(np.int32),
                          g.weights[g.offsets[a]:g.offsets[b]])


def test_batched_generated_planted_partitions():
    g, v_off = graphgen.planted_partition_batch(48, 11, n_range=(64, 3000))
    _check_batch([_sub(g, v_off, q) for q in range(48)], tuning=_queue_tuning(queue=0))


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
    # batch; one handle per schedule (work queue, class kernels)
    g, v_off = graphgen.planted_partition_batch(8192, 5)
    d = (_dev(g.offsets), _dev(g.targets), _dev(g.weights))
    B = {sched: lpa.LpaBatch(v_off, *d, tuning=_queue_tuning(512, 64, queue))
         for sched, queue in (("queue", 1), ("classes", 0))}
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
    for b in B.values():
        b.close()


@pytest.mark.parametrize("sched", ["queue", "classes"])
@pytest.mark.parametrize("launch", [lpa.LAUNCH_EAGER, lpa.LAUNCH_GRAPH])
def test_batched_full_size_sampled_graphs_equal_oracle(batch8k, launch, sched):
    # one deterministic batched run over all 8,192 graphs; 256 graphs drawn
    # at random and the 8 largest equal their solo oracle runs (labels,
    # iteration count, last iteration's changed count)
    g, v_off, B, refs = batch8k
    res = B[sched].run_batched("det", launch=launch)
    lab = res.labels.cpu().numpy()
    assert int(np.diff(v_off).max()) > 60000
    for q, ref in refs.items():
        got = lab[v_off[q]:v_off[q + 1]] - v_off[q]
        mism = np.nonzero(got != ref.labels)[0]
        assert mism.size == 0, (q, mism.size, mism[:5])
        assert res.iters_per_graph[q] == ref.iterations, (q, res.iters_per_graph[q], ref.iterations)
        assert res.changed_last[q] == ref.stats[-1]["changed"], q
    assert res.iterations == int(res.iters_per_graph.max())

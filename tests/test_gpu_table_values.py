"""GPU: the table-value precision ablation (Sec. 4.4; lpa_tuning.table_values
32 and 64) against the oracle.

Both widths run the same kernel set (a wave or a workgroup per row with an
LDS table, global-memory tables for longer rows), so:
  - on integer weights every sum is exact in either width and a
    deterministic run equals the oracle (labels, iteration count, counters);
  - on fp32 weights of at least 2^-7 every weight is a multiple of 2^-30, so
    fp64 sums below 2^22 are exact in any order: the 64-bit variant equals the
    fp64 oracle on arbitrary real weights as well;
  - a row where fp32 rounding decides the arg-max shows the difference: the
    64-bit tables take the oracle's label, the 32-bit ones (and the main
    path) the label that rounding ties.
"""
import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2411_11468_amd import lpa  # noqa: E402

SMALL_TUNING = dict(small4=2, small16=8, wave=40, block=100, hub_chunk=64)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _graph(g, tv, **tun):
    t = lpa.default_tuning()
    t.table_values = tv
    for k, v in tun.items():
        setattr(t, k, v)
    return lpa.LpaGraph(_dev(g.offsets), _dev(g.targets),
                        None if g.weights is None else _dev(g.weights), tuning=t)


def _labels(res):
    return res.labels.cpu().numpy()


def _assert_matches(ref, res):
    assert res.iterations == ref.iterations
    for a, b in zip(res.stats, ref.stats):
        for k in ("iteration", "pick_less", "changed", "processed", "edges_scanned"):
            assert a[k] == b[k], (k, a, b)
    lab = _labels(res)
    mism = np.nonzero(lab != ref.labels)[0]
    assert mism.size == 0, f"{mism.size} labels differ, first at {mism[:5]}"


def _real_weights(g):
    """Symmetric fp32 weights in [0.01, 1) with full 24-bit mantissas, from a
    hash of the unordered pair."""
    n = g.num_vertices
    rows = np.repeat(np.arange(n, dtype=np.uint64), np.diff(g.offsets.astype(np.int64)))
    cols = g.targets.astype(np.uint64)
    lo, hi = np.minimum(rows, cols), np.maximum(rows, cols)
    z = (lo * np.uint64(0x9E3779B97F4A7C15) + hi * np.uint64(0xBF58476D1CE4E5B9)) & \
        np.uint64(0xFFFFFFFFFFFFFFFF)
    z ^= z >> np.uint64(31)
    z = (z * np.uint64(0x94D049BB133111EB)) & np.uint64(0xFFFFFFFFFFFFFFFF)
    z ^= z >> np.uint64(29)
    frac = (z >> np.uint64(40)).astype(np.float64) / float(1 << 24)
    return (0.01 + 0.99 * frac).astype(np.float32)


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


@pytest.mark.parametrize("tv", [32, 64])
@pytest.mark.parametrize("name,g,tun", _cases(), ids=[c[0] for c in _cases()])
def test_det_parity_integer_weights(name, g, tun, tv):
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    G = _graph(g, tv, **tun)
    _assert_matches(ref, G.run("det"))
    _assert_matches(ref, G.run("det", launch=lpa.LAUNCH_GRAPH))
    G.close()


@pytest.mark.parametrize("tv", [32, 64])
def test_det_parity_internal_order_and_probes(tv):
    g = graphgen.rmat_graph(14, 6, "int8")
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    for probe in (0, 1, 3):
        G = _graph(g, tv, relabel=1, probe=probe, **SMALL_TUNING)
        _assert_matches(ref, G.run("det"))
        G.close()


@pytest.mark.parametrize("name,g,tun", [
    ("random", graphgen.random_graph(3000, 0.01, seed=77), {}),
    ("random_hubs", graphgen.random_graph(1500, 0.25, seed=6), SMALL_TUNING),
    ("rmat13", graphgen.rmat_graph(13, 9, "unit"), SMALL_TUNING),
], ids=["random", "random_hubs", "rmat13"])
def test_fp64_values_equal_the_oracle_on_real_weights(name, g, tun):
    w = _real_weights(g)
    rows = np.repeat(np.arange(g.num_vertices), np.diff(g.offsets.astype(np.int64)))
    wsum = np.bincount(rows, weights=w.astype(np.float64), minlength=g.num_vertices)
    assert wsum.max() < 2.0 ** 22 and w.min() >= 2.0 ** -7
    ref = oracle.lpa_sync(g.offsets, g.targets, w)
    G = _graph(graphgen.Graph(g.offsets, g.targets, w), 64, **tun)
    _assert_matches(ref, G.run("det"))
    G.close()


def test_fp32_rounding_decides_the_label():
    # vertex 0: label 1 through one edge of weight 2^24, label 5 through two
    # edges of weights 2^24 and 1.  The sums 2^24 and 2^24 + 1 are distinct in
    # fp64; fp32 rounds the second to 2^24 and the tie goes to the smaller
    # label.
    big = float(2 ** 24)
    g = graphgen.from_edges(6, [(0, 1), (0, 2), (0, 3), (4, 5)], weights=[big, big, 1.0, 1.0])
    init = np.array([0, 1, 5, 5, 4, 5], dtype=np.int32)
    kw = dict(tolerance=0.0, max_iterations=1, pl_period=0)
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights, initial_labels=init, **kw)
    assert ref.labels[0] == 5
    got = {}
    for tv in (0, 32, 64):
        G = _graph(g, tv)
        got[tv] = _labels(G.run("det", initial_labels=_dev(init), **kw))
        G.close()
    np.testing.assert_array_equal(got[64], ref.labels)
    assert got[32][0] == 1 and got[0][0] == 1
    np.testing.assert_array_equal(got[32][1:], ref.labels[1:])
    np.testing.assert_array_equal(got[0], got[32])


@pytest.mark.parametrize("tv", [32, 64])
def test_async_invariant_and_modularity(tv):
    for g, tun in ((graphgen.rmat_graph(14, 5, "int8"), {}),
                   (graphgen.rmat_graph(12, 6, "int8"), SMALL_TUNING)):
        G = _graph(g, tv, **tun)
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
        G.close()


def test_unsupported_and_invalid():
    g = graphgen.planted_partition_10k(1)
    with pytest.raises(lpa.LpaError):
        _graph(g, 16)
    G = _graph(g, 64)
    pr = lpa.Predictor()
    G.set_predictor(pr, threshold=0.5)
    with pytest.raises(lpa.LpaError):
        G.run("det", learned=True)
    with pytest.raises(lpa.LpaError):
        G.trace(sample_rate=0.1, seed=1, cap=1000)
    # the handle still runs plain
    ref = oracle.lpa_sync(g.offsets, g.targets, g.weights)
    _assert_matches(ref, G.run("det"))
    G.close()
    pr.close()
    packed, v_off = graphgen.pack_graphs([g, graphgen.disjoint_cliques(3, 4)])
    t = lpa.default_tuning()
    t.table_values = 64
    with pytest.raises(lpa.LpaError):
        lpa.LpaBatch(v_off, _dev(packed.offsets), _dev(packed.targets), _dev(packed.weights),
                     tuning=t)

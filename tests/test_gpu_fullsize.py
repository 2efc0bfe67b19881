"""GPU parity at the benchmark's full size: R-MAT scale 26 (67,108,864
vertices, 2,103,831,556 CSR entries, int64 offsets, an fp32 weight array of
1.0f), the handle and run options bench.py times.

The oracle cannot run Algorithm 1 over the whole graph in test time, so it
decides sampled vertices one by one:
  - deterministic mode, every iteration k of the run: the labels after k - 1
    iterations (a run capped there; the vertex ids for k = 1) and the flags
    that select iteration k's vertices go into one oracle iteration over the
    sampled rows (the other rows empty, so they keep their labels); every
    sampled vertex's label after k iterations must equal the oracle's, and
    iteration k's processed and changed counts must equal the flag and label
    differences over all vertices.  Iteration 1 is the table-free first
    sweep; the later ones run the table kernels, hub slices and bucket
    reductions;
  - asynchronous mode: every sampled vertex that is not flagged at exit
    holds a label of maximum weight (the oracle's local-optimality check on
    the sampled rows).
Samples: 100,000 vertices drawn uniformly plus 64 of the largest rows.
"""
import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2411_11468_amd import lpa  # noqa: E402

SCALE = 26
SAMPLES = 100_000


@pytest.fixture(scope="module")
def big():
    g = graphgen.rmat_graph(SCALE, SCALE, "unit", np.int64)
    dev = torch.device("cuda:0")
    d_off = torch.from_numpy(g.offsets).to(dev)
    d_tgt = torch.from_numpy(g.targets).to(dev)
    d_w = torch.from_numpy(g.weights).to(dev)
    G = lpa.LpaGraph(d_off, d_tgt, d_w)
    rng = np.random.default_rng(2026)
    n = g.num_vertices
    deg = np.diff(g.offsets)
    hubs = np.argsort(deg)[-64:]
    sample = np.unique(np.concatenate([rng.integers(0, n, SAMPLES), hubs])).astype(np.int64)
    yield g, G, sample
    G.close()


def _sampled_rows(g, sample):
    """The CSR with only the sampled rows kept (the others empty)."""
    n = g.num_vertices
    deg = np.diff(g.offsets)
    counts = np.zeros(n, dtype=np.int64)
    counts[sample] = deg[sample]
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    starts = g.offsets[sample]
    lens = deg[sample]
    idx = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens) + \
        np.arange(int(lens.sum()), dtype=np.int64)
    return off, np.ascontiguousarray(g.targets[idx])


def test_det_every_iteration_sampled(big):
    g, G, sample = big
    n = g.num_vertices
    full = G.run("det", profile=True)
    K = full.iterations
    assert K >= 2
    off, tgt = _sampled_rows(g, sample)
    prev = np.arange(n, dtype=np.int32)
    flags = np.ones(n, dtype=bool)
    for k in range(1, K + 1):
        nxt = None
        if k == K:
            cur = full.labels.cpu().numpy()
        else:
            cur = G.run("det", max_iterations=k).labels.cpu().numpy()
            nxt = G.flags().astype(bool)      # the vertices iteration k + 1 processes
        st = full.stats[k - 1]
        assert st["processed"] == int(flags.sum()), k
        assert st["changed"] == int((cur != prev).sum()), k
        pl = 1 if (k - 1) % 4 == 0 else 0     # Pick-Less period 4, from iteration 0
        one = oracle.lpa_sync(off, tgt, None, tolerance=0.0, max_iterations=1, pl_period=pl,
                              initial_labels=prev).labels
        want = np.where(flags[sample], one[sample], prev[sample])
        mism = np.nonzero(cur[sample] != want)[0]
        assert mism.size == 0, \
            f"iteration {k}: {mism.size} sampled labels differ, first at {sample[mism[:5]]}"
        prev, flags = cur, nxt


def test_async_invariant_sampled(big):
    g, G, sample = big
    res = G.run("async", profile=True)
    assert res.iterations >= 2
    lab = res.labels.cpu().numpy()
    flags = G.flags().astype(bool)
    off, tgt = _sampled_rows(g, sample)
    ok = oracle.local_optimal(off, tgt, None, lab)
    bad = sample[~ok[sample] & ~flags[sample]]
    assert bad.size == 0, f"{bad.size} sampled unflagged vertices hold a non-maximal label"
    for s in res.stats:
        assert 0 <= s["changed"] <= s["processed"] <= g.num_vertices

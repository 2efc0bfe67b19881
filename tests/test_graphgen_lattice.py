"""The road-like lattice generator (graphgen.lattice): structure only."""
import numpy as np

import graphgen


def test_lattice_is_a_symmetric_sorted_subgrid():
    rows, cols, keep = 60, 75, 0.525
    off, tgt = graphgen.lattice(rows, cols, keep, seed=3)
    n = rows * cols
    assert off.shape == (n + 1,) and off[0] == 0 and off[-1] == tgt.shape[0]
    src = np.repeat(np.arange(n), np.diff(off))
    # only lattice neighbours, rows strictly increasing, no self-loops
    d = tgt.astype(np.int64) - src
    assert np.all(np.isin(d, [-cols, -1, 1, cols]))
    assert np.all((d != 1) | (src % cols != cols - 1))      # no wrap to the next row
    assert np.all((d != -1) | (src % cols != 0))
    for v in range(n):
        row = tgt[off[v]:off[v + 1]]
        assert np.all(np.diff(row) > 0)
    # symmetric
    fwd = set(zip(src.tolist(), tgt.tolist()))
    assert all((b, a) in fwd for a, b in fwd)
    # about keep of the 2*rows*cols - rows - cols lattice edges
    edges = tgt.shape[0] // 2
    total = 2 * rows * cols - rows - cols
    assert abs(edges / total - keep) < 0.03


def test_lattice_extremes_and_seeds():
    off, tgt = graphgen.lattice(7, 9, 1.0, seed=1)
    assert tgt.shape[0] == 2 * (2 * 7 * 9 - 7 - 9)
    off, tgt = graphgen.lattice(7, 9, 0.0, seed=1)
    assert tgt.shape[0] == 0 and np.all(off == 0)
    a = graphgen.lattice(40, 40, 0.5, seed=11)
    b = graphgen.lattice(40, 40, 0.5, seed=11)
    c = graphgen.lattice(40, 40, 0.5, seed=12)
    assert np.array_equal(a[1], b[1]) and not np.array_equal(a[1], c[1])
    g = graphgen.lowdeg_graph(64, seed=2)
    assert g.num_vertices == 64 * 64 and np.all(g.weights == 1.0)
    assert 1.8 < g.num_edges / g.num_vertices < 2.4

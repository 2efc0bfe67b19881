"""GPU: lpa_modularity_noalloc, the modularity entry point that allocates no
device memory (its scratch is a fixed array in the library), against
lpa_modularity on the same handles and labels, through the C ABI.

Two calls in a row, the second on a smaller graph, so that the second finds
the first's sums in the shared scratch and must clear them; host and device
labels; the size limit and the label check.
"""
import numpy as np
import pytest

import graphgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2411_11468_amd import lpa  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _handle(g):
    return lpa.LpaGraph(_dev(g.offsets), _dev(g.targets), _dev(g.weights))


def test_noalloc_modularity_equals_lpa_modularity_twice_then_smaller():
    big = graphgen.rmat_graph(16, 3, "int8")
    small = graphgen.planted_partition_10k(2)
    rng = np.random.default_rng(11)
    for g in (big, small):  # the second call: a smaller graph on the same scratch
        G = _handle(g)
        res = G.run("det")
        labs = [res.labels, _dev(np.arange(g.num_vertices, dtype=np.int32)),
                rng.integers(0, 40, size=g.num_vertices).astype(np.int32)]
        for lab in labs:
            want = lpa.lpa_modularity(G.handle, lab)
            got = lpa.lpa_modularity_noalloc(G.handle, lab)
            assert got == pytest.approx(want, rel=1e-9, abs=1e-12), (g.name, got, want)
        G.close()


def test_noalloc_modularity_limits_and_errors():
    g = graphgen.ring_of_cliques(30, 5)
    G = _handle(g)
    lab = (np.arange(150) // 5).astype(np.int32)
    assert lpa.lpa_modularity_noalloc(G.handle, lab) == pytest.approx(20 / 22 - 1 / 30, abs=1e-12)
    with pytest.raises(lpa.LpaError):
        lpa.lpa_modularity_noalloc(G.handle, np.full(150, 150, np.int32))
    G.close()
    n = lpa.MODULARITY_NOALLOC_MAX_VERTICES + 1
    H = lpa.LpaGraph(_dev(np.r_[np.zeros(n - 1, np.int64), [1, 2]]),
                     _dev(np.array([n - 1, n - 2], np.int32)), None)
    with pytest.raises(lpa.LpaError):
        lpa.lpa_modularity_noalloc(H.handle, _dev(np.arange(n, dtype=np.int32)))
    H.close()

"""What the trained change predictor gains over the run without it (GPU).

The predictor shipped in paper_2411_11468_amd/predictor_lfr.npz was trained
by the library's own kernels on traces of 64 LFR-like graphs (seeds
1000-1063, 10^6 vertices).  On a held-out graph it must cut the label-scan
work (CSR entries scanned) of a deterministic run while keeping modularity
within 0.5% and the iteration count of the plain run, and its time to
termination (median of graph-launched runs) is reported beside the plain
run's and may not be more than 10% longer.  A tiny end-to-end pipeline
(traces -> training -> threshold) checks the training path.
"""
import os

import numpy as np
import pytest

import graphgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2411_11468_amd import learned, lpa  # noqa: E402

PARAMS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "paper_2411_11468_amd", "predictor_lfr.npz")


def _scanned(res):
    return sum(s["edges_scanned"] for s in res.stats)


def test_trained_predictor_cuts_scan_work_on_heldout_graph():
    pred, info = learned.load(PARAMS)
    g = learned.lfr(200_000, 2003)
    G = learned.gpu_graph(g)
    G.set_predictor(pred, threshold=info["threshold"])
    plain = G.run("det")
    learn = G.run("det", learned=True)
    qp, ql = G.modularity(plain.labels), G.modularity(learn.labels)
    sp, sl = _scanned(plain), _scanned(learn)
    hist = G.learned_history()
    print(f"plain {plain.iterations} it, {sp} entries, Q {qp:.4f}; learned "
          f"{learn.iterations} it, {sl} entries, Q {ql:.4f}, skipped "
          f"{sum(h['skipped'] for h in hist)}")
    assert learn.iterations <= plain.iterations + 1
    assert sl <= 0.95 * sp
    assert (qp - ql) / qp <= 0.005
    # time to termination on a held-out graph of the training size
    g1 = learned.lfr(1_000_000, 2003)
    G1 = learned.gpu_graph(g1)
    G1.set_predictor(pred, threshold=info["threshold"])
    _, tp = learned.timed_run(G1, "det", False, 5, lpa.LAUNCH_GRAPH)
    _, tl = learned.timed_run(G1, "det", True, 5, lpa.LAUNCH_GRAPH)
    print(f"10^6 vertices: plain {1e3 * tp:.3f} ms, learned {1e3 * tl:.3f} ms, "
          f"speedup {tp / tl:.3f}")
    assert tl <= 1.10 * tp
    G1.close()
    # an untrained network at the same threshold: the guard sweeps catch
    # its mistakes (fallback) or it skips far less usefully
    rnd = lpa.Predictor(seed=3)
    G.set_predictor(rnd, threshold=info["threshold"])
    r2 = G.run("det", learned=True)
    q2 = G.modularity(r2.labels)
    assert (qp - q2) / qp <= 0.05
    G.close()
    pred.close()
    rnd.close()


def test_training_pipeline_small():
    pred, info = learned.train(n=20_000, graphs=2, mode="det", rate=0.5, epochs=3, batch=1024,
                               lr=3e-3, seed=5, fn_target=0.02)
    assert info["samples"] > 10_000
    assert info["losses"][-1] < info["losses"][0]
    assert 0.0 < info["threshold"] <= 0.5
    assert info["val_fn_share"] <= 0.03
    pred.close()

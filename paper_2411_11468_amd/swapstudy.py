"""Community-swap mitigation study (Sec. 4.1, Fig. 1): runtime and modularity
of Pick-Less every 1..4 iterations (PL1..PL4), Cross-Check every 1..4
iterations (CC1..CC4) and their 16 hybrids (H p,q: PL every p and CC every
q), each against PL4, the method's choice.

  python -m paper_2411_11468_amd.swapstudy --graph rmat22 --mode async

Runs use eager launches (Cross-Check resolves its reverts in host-driven
rounds); times are medians of --reps runs after one warm-up.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def variants():
    out = [(f"PL{p}", p, 0) for p in (1, 2, 3, 4)]
    out += [(f"CC{q}", 0, q) for q in (1, 2, 3, 4)]
    out += [(f"H{p},{q}", p, q) for p in (1, 2, 3, 4) for q in (1, 2, 3, 4)]
    return out


def make(name: str):
    import graphgen
    if name == "rmat22":
        return graphgen.rmat_graph(22, 22, "int8")
    if name == "lfr1m":
        g, _ = graphgen.lfr_graph(1_000_000, 2000)
        return g
    if name == "lowdeg":
        return graphgen.lowdeg_graph(4096, 7)
    raise ValueError(name)


def study(graph: str, mode: str, reps: int) -> dict:
    import torch
    from . import lpa
    g = make(graph)
    dev = torch.device("cuda")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    G = lpa.LpaGraph(d(g.offsets), d(g.targets), d(g.weights))
    lab = torch.empty(g.num_vertices, dtype=torch.int32, device=dev)
    rows = []
    for name, p, q in variants():
        G.run(mode, out=lab, pl_period=p, cc_period=q)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = G.run(mode, out=lab, pl_period=p, cc_period=q)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        rows.append(dict(variant=name, pl_period=p, cc_period=q, iterations=res.iterations,
                         ms=1e3 * float(np.median(ts)), modularity=G.modularity(lab)))
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    G.close()
    base = next(r for r in rows if r["variant"] == "PL4")
    for r in rows:
        r["rel_runtime"] = r["ms"] / base["ms"]
        r["rel_modularity"] = r["modularity"] / base["modularity"] if base["modularity"] else None
    return dict(graph=graph, vertices=g.num_vertices, edges=g.num_edges, mode=mode, rows=rows)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--graph", default="rmat22", choices=["rmat22", "lfr1m", "lowdeg"])
    ap.add_argument("--mode", default="async", choices=["async", "det"])
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    print(json.dumps(study(args.graph, args.mode, args.reps)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

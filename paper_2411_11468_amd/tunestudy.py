"""Autotuner study: lpa_autotune on one workload, then the tuned and the
default tuning timed again side by side (fresh handles, captured iterations,
the same graph and options).

  python -m paper_2411_11468_amd.tunestudy --workload batch8k --budget-s 120

Workloads (seeded, synthetic; the same generators as bench.py):
  batch8k   8,192 planted partitions packed in one CSR (deterministic)
  lowdeg26  road-like lattice 8192 x 8192, mean degree 2.1 (asynchronous)
  rmat22    R-MAT scale 22, integer weights 1..8 (asynchronous)
  lfr1m     LFR-like graph of 10^6 vertices, seed 2000 (asynchronous)
Prints one JSON line: the chosen tuning, the search report and both times.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import lpa
from .autotune import tuning_to_dict


def _graph(name: str):
    import graphgen
    if name == "batch8k":
        g, v_off = graphgen.planted_partition_batch(8192, 5)
        return g, v_off, lpa.MODE_DETERMINISTIC
    if name == "lowdeg26":
        return graphgen.lowdeg_graph(8192, 7), None, lpa.MODE_ASYNC
    if name == "rmat22":
        return graphgen.rmat_graph(22, 22, "int8"), None, lpa.MODE_ASYNC
    if name == "lfr1m":
        g, _ = graphgen.lfr_graph(1_000_000, 2000)
        return g, None, lpa.MODE_ASYNC
    raise ValueError(name)


def _time(dev, v_off, mode, tuning, reps: int) -> float:
    import torch
    off, tgt, w = dev
    if v_off is None:
        G = lpa.LpaGraph(off, tgt, w, tuning=tuning, validate=False)
        run = lambda out: G.run(mode, out=out, launch=lpa.LAUNCH_GRAPH)  # noqa: E731
    else:
        G = lpa.LpaBatch(v_off, off, tgt, w, tuning=tuning, validate=False)
        run = lambda out: G.run_batched(mode, out=out, launch=lpa.LAUNCH_GRAPH)  # noqa: E731
    out = torch.empty(off.shape[0] - 1, dtype=torch.int32, device=off.device)
    run(out)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        run(out)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    G.close()
    return float(np.median(ts)) * 1e3


def main(argv=None) -> int:
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="batch8k",
                    choices=["batch8k", "lowdeg26", "rmat22", "lfr1m"])
    ap.add_argument("--budget-s", type=float, default=120.0)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    g, v_off, mode = _graph(args.workload)
    dev = tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda()
                for a in (g.offsets, g.targets, g.weights))
    t0 = time.perf_counter()
    best, rep = lpa.lpa_autotune(*dev, v_off=v_off, mode=mode, budget_ms=1e3 * args.budget_s)
    print(f"[tune] {args.workload}: search {time.perf_counter() - t0:.1f}s, {rep}",
          file=sys.stderr, flush=True)
    ms_default = _time(dev, v_off, mode, lpa.default_tuning(), args.reps)
    ms_tuned = _time(dev, v_off, mode, best, args.reps)
    print(json.dumps({"workload": args.workload, "mode": "det" if mode == 0 else "async",
                      "tuning": tuning_to_dict(best), "report": rep,
                      "default_ms": ms_default, "tuned_ms": ms_tuned,
                      "speedup": ms_default / ms_tuned}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

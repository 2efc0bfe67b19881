"""Training and evaluation of the change predictor (learned skipping).

All work runs in liblpa.so on the GPU: traces come from lpa_trace, the
network is trained by the library's forward/backward/Adam kernels
(lpa_predictor_train), and runs are timed with lpa_run.  The graphs are the
LFR-like planted partitions of graphgen (power-law degrees, exponent 2.5,
mean 20; power-law community sizes, exponent 2, in [20, 5000]; mixing mu
drawn per seed from U[0.1, 0.5]).

  python -m paper_2411_11468_amd.learned train --graphs 64 --n 1000000 \
      --out paper_2411_11468_amd/predictor_lfr.npz
  python -m paper_2411_11468_amd.learned evaluate --params paper_2411_11468_amd/predictor_lfr.npz

The comparison of a learned run with the plain run uses time to termination
on the same graph: |E| * iterations(plain) / t, so that cheaper iterations in
larger number earn nothing.
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

TRAIN_SEEDS = range(1000, 1064)
HELDOUT_SEEDS = range(2000, 2016)


def log(msg: str) -> None:
    print(f"[learned] {msg}", file=sys.stderr, flush=True)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_graph(g, tuning=None):
    from . import lpa
    return lpa.LpaGraph(_dev(g.offsets), _dev(g.targets), _dev(g.weights), tuning=tuning)


def lfr(n: int, seed: int):
    import graphgen
    g, _ = graphgen.lfr_graph(n, seed)
    return g


def collect_traces(n: int, seeds, mode: str, rate: float, cap_per_graph: int):
    """Sampled (features, changed) pairs of plain runs, as torch tensors on
    the GPU."""
    import torch
    from . import lpa
    Xs, ys = [], []
    m = lpa.MODE_DETERMINISTIC if mode == "det" else lpa.MODE_ASYNC
    for s in seeds:
        t0 = time.perf_counter()
        g = lfr(n, s)
        G = gpu_graph(g)
        X, y, v, it, drawn = G.trace(sample_rate=rate, seed=s, cap=cap_per_graph, mode=m,
                                     device=torch.device("cuda"))
        Xs.append(X.clone())
        ys.append(y.clone())
        G.close()
        log(f"trace seed {s}: mu {g.mu:.3f}, {int(y.shape[0])} samples "
            f"({float(y.float().mean()):.3f} changed), {time.perf_counter() - t0:.1f}s")
    return torch.cat(Xs), torch.cat(ys)


def choose_threshold(pred, X, y, fn_target: float) -> float:
    """Largest probability threshold whose predicted-unchanged set has a
    false-negative share (changed among predicted unchanged) <= fn_target on
    the samples (X, y)."""
    p = pred.predict(X).cpu().numpy().astype(np.float64)
    yy = y.cpu().numpy() > 0.5
    order = np.argsort(p)
    cum_fn = np.cumsum(yy[order])
    k = np.arange(1, len(p) + 1)
    ok = cum_fn <= fn_target * k
    if not ok.any():
        return 1e-4
    last = np.nonzero(ok)[0].max()
    th = float(p[order[last]])
    return min(max(th, 1e-4), 0.5)


def train(n: int, graphs: int, mode: str, rate: float, epochs: int, batch: int, lr: float,
          seed: int, fn_target: float):
    import torch
    from . import lpa
    seeds = list(TRAIN_SEEDS)[:graphs]
    X, y = collect_traces(n, seeds, mode, rate, cap_per_graph=4_000_000)
    pos = float(y.mean())
    log(f"{X.shape[0]} samples, {pos:.3f} positive")
    # hold out a tenth for the threshold
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(X.shape[0], generator=g).cuda()
    nv = max(1, X.shape[0] // 10)
    Xv, yv = X[perm[:nv]], y[perm[:nv]]
    Xt, yt = X[perm[nv:]], y[perm[nv:]]
    pred = lpa.Predictor(seed=seed)
    pos_weight = float((1.0 - pos) / max(pos, 1e-6))
    t0 = time.perf_counter()
    losses = []
    for ep in range(epochs):
        losses.append(pred.train(Xt, yt, epochs=1, batch=batch, lr=lr, pos_weight=pos_weight,
                                 seed=seed + ep))
        log(f"epoch {ep}: loss {losses[-1]:.4f}")
    train_s = time.perf_counter() - t0
    th = choose_threshold(pred, Xv, yv, fn_target)
    pv = pred.predict(Xv).cpu().numpy()
    yvn = yv.cpu().numpy() > 0.5
    skip = pv < th
    info = dict(samples=int(X.shape[0]), positive=pos, pos_weight=pos_weight, epochs=epochs,
                batch=batch, lr=lr, losses=losses, train_s=train_s, threshold=th,
                val_skip_share=float(skip.mean()),
                val_fn_share=float(yvn[skip].mean()) if skip.any() else 0.0,
                mode=mode, n=n, graphs=graphs, rate=rate)
    return pred, info


def timed_run(G, mode: str, learned: bool, reps: int, launch):
    import torch
    res = G.run(mode, learned=learned, launch=launch)      # warm-up
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = G.run(mode, learned=learned, launch=launch)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return res, float(np.median(ts))


def evaluate(pred, threshold: float, graphs, mode: str, reps: int = 5, guard: int = 4,
             fn_bound: float = 0.02):
    """Plain vs learned time to termination and modularity per graph."""
    from . import lpa
    out = []
    for name, g in graphs:
        G = gpu_graph(g)
        G.set_predictor(pred, threshold=threshold, fn_bound=fn_bound, guard_period=guard)
        launch = lpa.LAUNCH_GRAPH
        rp, tp = timed_run(G, mode, False, reps, launch)
        rl, tl = timed_run(G, mode, True, reps, launch)
        qp = G.modularity(rp.labels)
        ql = G.modularity(rl.labels)
        # scanned edges of both (eager, for the counters)
        sp = G.run(mode, learned=False)
        sl = G.run(mode, learned=True)
        hist = G.learned_history()
        m = g.num_edges
        out.append(dict(
            graph=name, vertices=g.num_vertices, edges=m, mode=mode,
            plain_iters=rp.iterations, learned_iters=rl.iterations,
            plain_ms=1e3 * tp, learned_ms=1e3 * tl,
            plain_edges_per_s=m * rp.iterations / tp,
            learned_edges_per_s_plain_iters=m * rp.iterations / tl,
            speedup=tp / tl,
            plain_q=qp, learned_q=ql, dq_rel=(qp - ql) / abs(qp) if qp else 0.0,
            plain_scanned=int(sum(s["edges_scanned"] for s in sp.stats)),
            learned_scanned=int(sum(s["edges_scanned"] for s in sl.stats)),
            skipped=int(sum(h["skipped"] for h in hist)),
            fallback=bool(hist and hist[-1]["fallback"])))
        log(json.dumps(out[-1]))
        G.close()
    return out


def save(path: str, pred, info: dict) -> None:
    np.savez(path, params=pred.params(), info=json.dumps(info))


def load(path: str):
    from . import lpa
    z = np.load(path, allow_pickle=False)
    info = json.loads(str(z["info"]))
    return lpa.Predictor(params=z["params"]), info


def table_md(res: dict, command: str) -> str:
    """Markdown table of a learned-vs-plain evaluation (the JSON line of
    bench.py --workload lfr1m, or of the evaluate command)."""
    runs = res["runs"]
    th = res.get("config", {}).get("threshold", res.get("threshold"))
    mode = runs[0]["mode"] if runs else "?"
    sp = res.get("speedup_geomean", res.get("geomean_speedup"))
    out = [f"# Learned skipping vs plain ({'deterministic' if mode == 'det' else 'asynchronous'}"
           " mode)", "", f"Command: `{command}`", "",
           f"Threshold {th}; times are medians of graph-launched runs to termination on one "
           "MI355X.", "",
           "| graph | vertices | CSR entries | iterations plain / learned | ms plain | "
           "ms learned | speedup | Q plain | Q learned | scanned plain | scanned learned | "
           "skipped | fallback |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in runs:
        out.append(f"| {r['graph']} | {r['vertices']} | {r['edges']} | {r['plain_iters']} / "
                   f"{r['learned_iters']} | {r['plain_ms']:.3f} | {r['learned_ms']:.3f} | "
                   f"{r['speedup']:.3f} | {r['plain_q']:.4f} | {r['learned_q']:.4f} | "
                   f"{r['plain_scanned']} | {r['learned_scanned']} | {r['skipped']} | "
                   f"{r['fallback']} |")
    out += ["", f"Geometric-mean speedup {sp:.3f}; worst relative modularity loss "
                f"{res['worst_dq_rel']:.4f}."]
    return "\n".join(out) + "\n"


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--graphs", type=int, default=64)
    t.add_argument("--n", type=int, default=1_000_000)
    t.add_argument("--mode", default="det", choices=["det", "async"])
    t.add_argument("--rate", type=float, default=0.05)
    t.add_argument("--epochs", type=int, default=4)
    t.add_argument("--batch", type=int, default=4096)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--seed", type=int, default=7)
    t.add_argument("--fn-target", type=float, default=0.01)
    t.add_argument("--out", required=True)
    e = sub.add_parser("evaluate")
    e.add_argument("--params", required=True)
    e.add_argument("--n", type=int, default=1_000_000)
    e.add_argument("--heldout", type=int, default=4)
    e.add_argument("--rmat", type=int, default=24, help="R-MAT scale (0: none)")
    e.add_argument("--mode", default=None, choices=["det", "async"])
    e.add_argument("--threshold", type=float, default=None)
    e.add_argument("--seeds", default=None,
                   help="comma-separated LFR seeds instead of the first --heldout held-out ones")
    e.add_argument("--out", default=None)
    tb = sub.add_parser("table")
    tb.add_argument("json")
    tb.add_argument("--command", required=True)
    tb.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "table":
        with open(args.json) as f:
            res = json.loads(f.read().strip().splitlines()[-1])
        with open(args.out, "w") as f:
            f.write(table_md(res, args.command))
        return 0
    if args.cmd == "train":
        pred, info = train(args.n, args.graphs, args.mode, args.rate, args.epochs, args.batch,
                           args.lr, args.seed, args.fn_target)
        save(args.out, pred, info)
        log(f"saved {args.out}: {json.dumps({k: v for k, v in info.items() if k != 'losses'})}")
        return 0
    import graphgen
    pred, info = load(args.params)
    mode = args.mode or info["mode"]
    th = args.threshold if args.threshold is not None else info["threshold"]
    seeds = ([int(x) for x in args.seeds.split(",")] if args.seeds
             else list(HELDOUT_SEEDS)[:args.heldout])
    graphs = [(f"lfr{args.n}-s{s}", lfr(args.n, s)) for s in seeds]
    if args.rmat:
        graphs.append((f"rmat{args.rmat}", graphgen.rmat_graph(args.rmat, args.rmat, "unit")))
    res = evaluate(pred, th, graphs, mode)
    summary = dict(threshold=th, mode=mode, runs=res,
                   geomean_speedup=float(np.exp(np.mean([np.log(r["speedup"]) for r in res]))),
                   worst_dq_rel=float(max(r["dq_rel"] for r in res)))
    print(json.dumps(summary), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(summary, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())

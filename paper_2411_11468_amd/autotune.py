"""Autotuned lpa_tuning with a cache keyed by the graph's degree histogram.

The search itself is lpa_autotune in liblpa.so (successive halving in stages:
the batched schedule, class thresholds and slice sizes, workgroup sizes,
table capacities and the flag policy; each candidate timed on complete
runs).  Graphs
whose degree distributions agree to two significant digits per power-of-two
bin (and in vertex / entry counts) share a cache entry.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import lpa

TUNING_FIELDS = ("small4", "small16", "wave", "block", "hub_chunk", "max_retries", "xcd_local",
                 "hub_table_cap", "relabel", "probe", "table_values", "batch_queue",
                 "queue_chunk", "queue_group", "sort_rows", "block_threads", "table_load",
                 "pull_divisor", "memory_limit_kib")


def _round2(x: int) -> int:
    """x rounded to two significant digits."""
    if x < 100:
        return int(x)
    e = len(str(int(x))) - 2
    return int(round(x / 10 ** e)) * 10 ** e


def degree_signature(offsets, num_graphs: int = 0) -> str:
    off = np.asarray(offsets, dtype=np.int64)
    deg = np.diff(off)
    b = np.zeros(deg.shape, dtype=np.int64)
    nz = deg > 0
    b[nz] = np.floor(np.log2(deg[nz])).astype(np.int64) + 1
    hist = np.bincount(b, minlength=34)
    key = [_round2(int(h)) for h in hist] + [_round2(int(deg.shape[0])), _round2(int(off[-1])),
                                             int(num_graphs)]
    return hashlib.sha1(json.dumps(key).encode()).hexdigest()[:16]


def tuning_to_dict(t) -> dict:
    return {f: int(getattr(t, f)) for f in TUNING_FIELDS}


def tuning_from_dict(d: dict):
    t = lpa.default_tuning()
    for f in TUNING_FIELDS:
        if f in d:  # entries written before a field existed keep its default
            setattr(t, f, int(d[f]))
    return t


def tuned(offsets, targets, weights=None, *, v_off=None, mode: int = lpa.MODE_ASYNC,
          budget_ms: float = 60_000.0, cache_path: str | None = None, tuner=None):
    """lpa_tuning for this graph: from the cache when its signature is there,
    else searched with lpa_autotune (tuner: a stand-in with the same
    signature, for tests) and stored.  Returns (tuning, info dict)."""
    offs = offsets.cpu().numpy() if hasattr(offsets, "cpu") else offsets
    sig = degree_signature(offs, 0 if v_off is None else len(v_off) - 1)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    key = f"{sig}-mode{int(mode)}"
    if key in cache:
        return tuning_from_dict(cache[key]["tuning"]), dict(cache[key], cached=True)
    run = tuner or lpa.lpa_autotune
    t, rep = run(offsets, targets, weights, v_off=v_off, mode=mode, budget_ms=budget_ms)
    entry = {"tuning": tuning_to_dict(t), "report": rep}
    if cache_path:
        cache[key] = entry
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return t, dict(entry, cached=False)

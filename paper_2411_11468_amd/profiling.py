"""Summaries of rocprofv3 output for the label-propagation kernels.

  python -m paper_2411_11468_amd.profiling stats <kernel_stats.csv> --command CMD --out F.md
      per-kernel call count, total and average duration (kernel-trace --stats)
  python -m paper_2411_11468_amd.profiling traffic --fetch <counter_collection.csv>
      --write <counter_collection.csv> --copy-bytes B --command CMD --out F.json
      per-kernel FETCH_SIZE and WRITE_SIZE per dispatch (KiB), each scaled by
      the ratio the same counter shows for a plain device copy of B bytes
      (the largest copy kernel in the same files), and the hash of the kernel
      sources the counters were taken with.

The traffic summary is read by bench.py, which reports it only while the
kernel sources still hash to the recorded value.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

# rocprofv3 kernel names -> the names used by lpa_profile
_NAME_RULES = [
    (r"k_sweep_small<[^,]+, 4>", "sweep_small4"),
    (r"k_sweep_small<[^,]+, 16>", "sweep_small16"),
    (r"k_sweep_wave<[^,]+, 127,", "sweep_wave127"),
    (r"k_sweep_wave<[^,]+, 1023,", "sweep_wave1023"),
    (r"k_sweep_block<[^,]+, 2047,", "sweep_block2047"),
    (r"k_sweep_block<[^,]+, 4095,", "sweep_block4095"),
    (r"k_sweep_block<[^,]+, 8191,", "sweep_block8191"),
    (r"k_sweep_block<[^,]+, 16383,", "sweep_block16383"),
    (r"k_hub_acc<[^>]*true>", "hub_acc"),
    (r"k_hub_acc<[^>]*false>", "hub_acc_rest"),
    (r"k_hub_fin<", "hub_fin"),
    (r"k_hub_plan<", "hub_plan"),
    (r"k_frontier", "frontier"),
    (r"k_apply", "apply"),
    (r"k_pull_flags<", "pull_flags"),
    (r"k_pull_hubs<", "pull_hubs"),
    (r"k_push_lists<", "push_flags"),
    (r"k_push_hubs<", "push_hubs"),
    (r"k_flag_decide", "flag_decide"),
    (r"k_batch_step", "batch_step"),
    (r"k_iter_end", "iter_end"),
    (r"k_mod_edges<", "mod_edges"),
    (r"k_mod_sq", "mod_sq"),
]


def short_name(kernel: str) -> str:
    for pat, name in _NAME_RULES:
        if re.search(pat, kernel):
            return name
    return kernel.split("(")[0][:60]


def source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(CSRC, "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_stats_md(csv_path: str, command: str) -> str:
    rows = list(csv.DictReader(open(csv_path)))
    out = ["# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
           f"Kernel sources: {source_hash()}", "",
           "| kernel | short name | calls | total ms | average us | % |",
           "|---|---|---|---|---|---|"]
    for r in rows:
        name = r.get("Name") or r.get("KERNEL_NAME") or ""
        calls = int(float(r.get("Calls", 0)))
        tot = float(r.get("TotalDurationNs", 0)) / 1e6
        avg = float(r.get("AverageNs", 0)) / 1e3
        pct = float(r.get("Percentage", 0))
        out.append(f"| `{name[:90]}` | {short_name(name)} | {calls} | {tot:.3f} | {avg:.1f} | {pct:.2f} |")
    return "\n".join(out) + "\n"


def _counter_means(csv_path: str, counter: str) -> dict:
    """Average counter value per dispatch for every kernel name."""
    acc = defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        if r.get("Counter_Name") != counter:
            continue
        acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def traffic_json(fetch_csv: str, write_csv: str, copy_bytes: float, command: str) -> dict:
    fetch = _counter_means(fetch_csv, "FETCH_SIZE")
    write = _counter_means(write_csv, "WRITE_SIZE")
    copies = [k for k in fetch if "copy" in k.lower()]
    if not copies:
        raise SystemExit("no copy kernel in the FETCH_SIZE run")
    ck = max(copies, key=lambda k: fetch[k])
    kib = copy_bytes / 1024.0
    f_scale = kib / fetch[ck]
    w_scale = kib / write.get(ck, fetch[ck]) if write.get(ck) else 1.0
    kernels = {}
    for k in fetch:
        s = short_name(k)
        kernels.setdefault(s, {"fetch_kib": 0.0, "write_kib": 0.0, "n": 0})
        kernels[s]["fetch_kib"] += fetch[k]
        kernels[s]["write_kib"] += write.get(k, 0.0)
        kernels[s]["n"] += 1
    for s, v in kernels.items():
        v["fetch_kib"] /= v["n"]
        v["write_kib"] /= v["n"]
        v["bytes_per_dispatch"] = 1024.0 * (v["fetch_kib"] * f_scale + v["write_kib"] * w_scale)
        del v["n"]
    return {"command": command, "sources": source_hash(), "copy_kernel": ck,
            "copy_bytes": copy_bytes, "fetch_scale": f_scale, "write_scale": w_scale,
            "kernels": kernels}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--command", required=True)
    a.add_argument("--out", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--copy-bytes", type=float, required=True)
    b.add_argument("--command", required=True)
    b.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        with open(args.out, "w") as f:
            f.write(kernel_stats_md(args.csv, args.command))
    else:
        with open(args.out, "w") as f:
            json.dump(traffic_json(args.fetch, args.write, args.copy_bytes, args.command), f,
                      indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Summaries of rocprofv3 output for the label-propagation kernels.

  python -m paper_2411_11468_amd.profiling stats <kernel_stats.csv> --command CMD --out F.md
      per-kernel call count, total and average duration (kernel-trace --stats)
  python -m paper_2411_11468_amd.profiling traffic --fetch <counter_collection.csv>
      --write <counter_collection.csv> --copy-bytes B --command CMD --out F.json
      per-kernel FETCH_SIZE and WRITE_SIZE per dispatch (KiB, averaged over the
      kernel's dispatches), each scaled by the ratio the same counter shows
      for plain device copies of B bytes (the largest copy dispatches in the
      same files), and the hash of the kernel sources the counters were
      taken with.

  python -m paper_2411_11468_amd.profiling counters <counter_collection.csv>...
      --command CMD --out F.md
      per-kernel mean per dispatch of every counter in the given files (one
      file per --pmc pass), e.g. the L2 hits, misses and HBM read requests

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
    (r"k_sweep_small<[^,]+, 4[,>]", "sweep_small4"),
    (r"k_sweep_small<[^,]+, 16[,>]", "sweep_small16"),
    (r"k_sweep_small16x2<", "sweep_small16"),
    (r"k_sweep_group<[^,]+, 127,", "sweep_wave127"),
    (r"k_sweep_wave_pipe<[^,]+, 1023,", "sweep_wave1023"),
    (r"k_sweep_block(_pipe)?<[^,]+, 2047,", "sweep_block2047"),
    (r"k_sweep_block(_pipe)?<[^,]+, 4095,", "sweep_block4095"),
    (r"k_sweep_block(_pipe)?<[^,]+, 8191,", "sweep_block8191"),
    (r"k_sweep_block(_pipe)?<[^,]+, 16383,", "sweep_block16383"),
    # the table-free first sweep: one instantiation per lane-group width
    # (1 for degrees up to 4; 4 for 5..16; 8 for 17..64; 16 for 65..512;
    # 64 for 513..2048; 256 above), so lpa_profile's direct_wave1023 is
    # "direct_g16", its block2047 + block4095 "direct_g64" and its
    # block8191 + block16383 "direct_g256"
    (r"k_sweep_direct2?<[^,]+, 1,", "direct_small4"),
    (r"k_sweep_direct2?<[^,]+, 4,", "direct_small16"),
    (r"k_sweep_direct2?<[^,]+, 8,", "direct_wave127"),
    (r"k_sweep_direct2?<[^,]+, 16,", "direct_g16"),
    (r"k_sweep_direct2?<[^,]+, 64,", "direct_g64"),
    (r"k_sweep_direct2?<[^,]+, 256,", "direct_g256"),
    (r"k_sweep_lane4<", "sweep_small4"),
    # the table-value ablation kernels (sweep_tv.hip)
    (r"k_tv_wave<|k_tv_block<", "tv_sweep"),
    (r"k_tv_hub_acc<", "tv_hub_acc"),
    (r"k_tv_hub_(max|arg|pack)", "tv_hub_select"),
    (r"k_hub_direct<", "hub_direct"),
    (r"k_rl_|k_scan_chunks|k_scan_add", "relabel_build"),
    (r"k_unpermute<", "unpermute"),
    (r"k_hub_part<", "hub_part"),
    (r"k_hub_reduce<", "hub_reduce"),
    (r"k_hub_spill<", "hub_spill"),
    (r"k_hub_fin<", "hub_fin"),
    (r"k_hub_plan<", "hub_plan"),
    (r"k_frontier_learned", "frontier_learned"),
    (r"k_frontier", "frontier"),
    (r"k_trace_label", "trace_label"),
    (r"k_mlp_infer", "mlp_infer"),
    (r"k_mlp_grad", "mlp_grad"),
    (r"k_adam", "adam"),
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
    # anything else: the bare function name without its namespace,
    # template arguments or the k_ prefix
    base = re.sub(r"<.*", "", kernel.replace("(anonymous namespace)::", "").split("(")[0])
    return re.sub(r"^(void )?(lpa::)?(k_)?", "", base)[:60]


def source_hash() -> str:
    """Hash of the device code (the .hip kernels and the headers they
    include); host-only .cpp files do not change what a kernel does."""
    h = hashlib.sha256()
    files = glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h"))
    for f in sorted(files):
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


def _counter_rows(csv_path: str, counter: str) -> list:
    """(kernel name, value) per dispatch; rocprofv3 writes one row per
    dispatch and counter, values in KiB for FETCH_SIZE / WRITE_SIZE."""
    return [(r["Kernel_Name"], float(r["Counter_Value"]))
            for r in csv.DictReader(open(csv_path)) if r.get("Counter_Name") == counter]


def _copy_rows(csv_path: str, counter: str) -> list:
    """(dispatch id, grid size, value) of the copy kernels, in dispatch order."""
    rows = [(int(r["Dispatch_Id"]), int(r.get("Grid_Size") or 0), float(r["Counter_Value"]))
            for r in csv.DictReader(open(csv_path))
            if r.get("Counter_Name") == counter and "copy" in r["Kernel_Name"].lower()]
    return sorted(rows)


def _calibration(copies: list, copy_kib: float) -> tuple:
    """Scale that maps the counter of the reference copies (copy_kib KiB
    each) onto their true size.  bench.py --calibrate-copy runs them last:
    one untimed and three timed copies of the same size, so they are the
    trailing copy dispatches of the run with the last one's grid size (an
    upload earlier in the run may be a larger copy kernel)."""
    if not copies:
        raise SystemExit("no copy kernel in the counter run")
    grid = copies[-1][1]
    tail = []
    for d, gsz, v in reversed(copies):
        if gsz != grid or len(tail) == 3:
            break
        tail.append(v)
    mean = sum(tail) / len(tail)
    return copy_kib / mean, len(tail)


def _means_by_kernel(rows: list) -> dict:
    acc = defaultdict(list)
    for k, v in rows:
        acc[short_name(k)].append(v)
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def traffic_json(fetch_csv: str, write_csv: str, copy_bytes: float, command: str) -> dict:
    frows = _counter_rows(fetch_csv, "FETCH_SIZE")
    wrows = _counter_rows(write_csv, "WRITE_SIZE")
    kib = copy_bytes / 1024.0
    f_scale, nf = _calibration(_copy_rows(fetch_csv, "FETCH_SIZE"), kib)
    w_scale, nw = _calibration(_copy_rows(write_csv, "WRITE_SIZE"), kib)
    fm, wm = _means_by_kernel(frows), _means_by_kernel(wrows)
    kernels = {}
    for s, (f, n) in fm.items():
        w = wm.get(s, (0.0, 0))[0]
        kernels[s] = {"dispatches": n, "fetch_kib": f, "write_kib": w,
                      "bytes_per_dispatch": 1024.0 * (f * f_scale + w * w_scale)}
    return {"command": command, "sources": source_hash(), "copy_bytes": copy_bytes,
            "copy_dispatches": [nf, nw], "fetch_scale": f_scale, "write_scale": w_scale,
            "kernels": kernels}


def counters_md(paths: list, command: str) -> str:
    vals = defaultdict(lambda: defaultdict(list))   # kernel -> counter -> values
    names = []
    for p in paths:
        for r in csv.DictReader(open(p)):
            c = r.get("Counter_Name")
            if not c:
                continue
            if c not in names:
                names.append(c)
            vals[short_name(r["Kernel_Name"])][c].append(float(r["Counter_Value"]))
    out = ["# rocprofv3 counters per dispatch", "", f"Command: `{command}`", "",
           f"Kernel sources: {source_hash()}", "",
           "Mean per dispatch over the kernel's dispatches.", "",
           "| kernel | dispatches | " + " | ".join(names) + " |",
           "|---|---|" + "---|" * len(names)]
    for k in sorted(vals, key=lambda k: -max(sum(v) for v in vals[k].values())):
        n = max(len(v) for v in vals[k].values())
        cells = [f"{sum(vals[k][c]) / len(vals[k][c]):.4g}" if vals[k][c] else "" for c in names]
        out.append(f"| {k} | {n} | " + " | ".join(cells) + " |")
    return "\n".join(out) + "\n"


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
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+")
    c.add_argument("--command", required=True)
    c.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "counters":
        with open(args.out, "w") as f:
            f.write(counters_md(args.csv, args.command))
    elif args.cmd == "stats":
        with open(args.out, "w") as f:
            f.write(kernel_stats_md(args.csv, args.command))
    else:
        with open(args.out, "w") as f:
            json.dump(traffic_json(args.fetch, args.write, args.copy_bytes, args.command), f,
                      indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Summary of a rocprofv3 kernel trace of the benchmark, as markdown.

    rocprofv3 --kernel-trace --stats --output-format csv -d DIR -- python bench.py
    python -m paper_2211_01185_amd.trace_summary --trace DIR --bench-json FILE

Prints the kernel statistics of the whole command and the contact-force
kernel's launch durations over the main measurement's two regions: the timed
steps of the first bed and the same steps replayed on a second bed (where the
benchmark reads its per-launch HIP events).  A bed of the main measurement is
recognised by its creation-time evaluation (force_kick<float, false, false,
L, false>: no rolling friction) at the main bed's grid size followed by step
launches of the single-bed kernel: the measurement's two beds run exactly
warm-up + timed steps (the autotuner's trials run two more coupling periods,
the settling run thousands of steps, the smoothing run fewer).
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re

import numpy as np

FORCE_BLOCK = 128


def _one(d, suffix):
    files = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if len(files) != 1:
        raise SystemExit(f"{d}: expected one *{suffix}, found {len(files)}")
    with open(files[0]) as fh:
        return list(csv.DictReader(fh))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--bench-json", required=True)
    ap.add_argument("--top", type=int, default=12)
    args = ap.parse_args(argv)
    with open(args.bench_json) as fh:
        bench = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    lanes = int(bench["config"]["tuned"]["lanes"])
    n = int(bench["config"]["particles"])
    warmup, steps = int(bench["warmup"]), int(bench["steps"])
    grid = -(-n * lanes // FORCE_BLOCK) * FORCE_BLOCK

    stats = _one(args.trace, "kernel_stats.csv")
    print("| kernel | calls | avg us | min us | max us | share % |")
    print("|---|---|---|---|---|---|")
    for r in stats[:args.top]:
        name = r["Name"] if len(r["Name"]) <= 72 else r["Name"][:69] + "..."
        print(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
              f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")

    rows = _one(args.trace, "kernel_trace.csv")
    key = "Kernel_Name" if "Kernel_Name" in rows[0] else "Name"
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    prime_re = re.compile(rf"cfddem::force_kick<float, false, false, {lanes}, false>")
    step_re = re.compile(rf"cfddem::force_kick<float, true, (true|false), {lanes}, false>")
    beds, cur = [], None
    for r in rows:
        if int(r.get("Grid_Size", r.get("Grid_Size_X", 0)) or 0) != grid:
            continue
        if prime_re.search(r[key]):
            cur = []
            beds.append(cur)
        elif cur is not None and step_re.search(r[key]):
            cur.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    full = [b for b in beds if len(b) == warmup + steps]
    if len(full) != 2:
        raise SystemExit(f"found {len(full)} beds with exactly {warmup + steps} step launches at grid {grid}")
    print()
    print(f"Contact-force kernel `force_kick<float, true, *, {lanes}>` over the main measurement "
          f"({steps} launches after {warmup} warm-up steps; grid {grid}):")
    print()
    for name, b in (("timed region (first bed)", full[0]), ("replayed region (second bed)", full[1])):
        x = np.array(b[warmup:warmup + steps])
        med = float(np.median(x))
        print(f"- {name}: mean {x.mean():.2f} us, median {med:.2f} us, p90 {np.percentile(x, 90):.2f} us, "
              f"max {x.max():.2f} us; {int((x > 2 * med).sum())} launches above twice the median "
              f"(steps that run a broad search)")
    print(f"- bench.py's HIP events over the replayed region (same run, under the profiler): "
          f"{bench['roofline']['avg_launch_us']:.2f} us per launch")


if __name__ == "__main__":
    main()

"""Summary of a rocprofv3 kernel trace of the benchmark, as markdown.

    rocprofv3 --kernel-trace --stats --output-format csv -d DIR -- python bench.py
    python -m paper_2211_01185_amd.trace_summary --trace DIR --bench-json FILE

Prints the kernel statistics of the whole command and the contact-force
kernel's launch durations over the main bed's timed region and over the
roofline window's two runs (the second is where the benchmark reads its
per-launch HIP events).  With --bed spouted: the kernels
of the spouted-bed measurement's timed bed instead (the last two beds created
at that bed's grid are the timed one and its replay; the tuner's trial beds
come before them).  A bed of the main measurement is
recognised by its creation-time evaluation (force_kick<float, false, false,
L, false>: no rolling friction) at the main bed's grid size followed by step
launches of the single-bed kernel; the timed bed runs exactly warm-up + timed
steps and the window's beds the window's steps (the autotuner's trials run two
more coupling periods, the settling run thousands of steps, the smoothing run
fewer).  With --bed batched: the kernels of the batched ensemble's run (from
the first to the last contact-force launch at the ensemble's grid, which the
benchmark reports; the tuner's trials run fewer beds, so smaller grids), per
launch and per ensemble step, and the contact-force kernel's fraction of the
HBM peak at the ensemble's algorithmic bytes per step.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re

import numpy as np



def _force_block():
    """Threads per block of the contact-force kernels, from the device header."""
    hdr = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "device.h")
    with open(hdr) as f:
        return int(re.search(r"constexpr int kForceBlock = (\d+);", f.read()).group(1))


FORCE_BLOCK = _force_block()


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
    ap.add_argument("--bed", choices=("main", "spouted", "batched"), default="main")
    args = ap.parse_args(argv)
    with open(args.bench_json) as fh:
        bench = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    if args.bed == "spouted":
        return spouted(args, bench)
    if args.bed == "batched":
        return batched(args, bench)
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
    # beds in creation order: the tuner's trials (two coupling periods longer
    # than the window), the timed region (warmup + steps launches), then the
    # roofline window's run and its replay (WINDOW launches each)
    window = bench["roofline"]["window"]
    ww, ws = int(window["warmup"]), int(window["steps"])
    timed = [b for b in beds if len(b) == warmup + steps]
    win = [b for b in beds if len(b) == ww + ws]
    if warmup + steps == ww + ws:
        win = win[1:]  # the timed region itself comes first
    if not timed or len(win) < 2:
        raise SystemExit(f"found {len(timed)} timed beds and {len(win)} window beds at grid {grid}")
    print()
    print(f"Contact-force kernel `force_kick<float, true, *, {lanes}>` of the main bed (grid {grid}):")
    print()
    for name, b, w0, k in (("timed region", timed[0], warmup, steps),
                           ("roofline window, run", win[0], ww, ws),
                           ("roofline window, replay with per-launch events", win[1], ww, ws)):
        x = np.array(b[w0:w0 + k])
        med = float(np.median(x))
        print(f"- {name} ({k} launches after {w0} warm-up steps): mean {x.mean():.2f} us, median {med:.2f} us, "
              f"p90 {np.percentile(x, 90):.2f} us, max {x.max():.2f} us; {int((x > 2 * med).sum())} launches "
              f"above twice the median (steps that run a broad search)")
    print(f"- bench.py's HIP events over the window's replay (same run, under the profiler): "
          f"{bench['roofline']['avg_launch_us']:.2f} us per launch")


def spouted(args, bench):
    sp = bench["spouted"]
    lanes = int(sp["tuned"]["lanes"])
    n = int(sp["particles"])
    warmup, steps = int(sp["warmup"]), int(sp["steps"])
    grid = -(-n * lanes // FORCE_BLOCK) * FORCE_BLOCK
    rows = _one(args.trace, "kernel_trace.csv")
    key = "Kernel_Name" if "Kernel_Name" in rows[0] else "Name"
    gkey = "Grid_Size" if "Grid_Size" in rows[0] else "Grid_Size_X"
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    prime_re = re.compile(rf"cfddem::force_kick<float, false, false, {lanes}, false>")
    step_re = re.compile(rf"cfddem::force_kick<float, true, (true|false), {lanes}, false>")
    starts = [i for i, r in enumerate(rows) if int(r[gkey] or 0) == grid and prime_re.search(r[key])]
    starts.append(len(rows))
    # the timed bed: the first bed at this grid that runs exactly warm-up +
    # timed step launches (the tuner's trials run two coupling periods more,
    # the replay comes after it and the oracle comparison's bed one step)
    timed = [(b, e) for b, e in zip(starts, starts[1:])
             if sum(1 for r in rows[b:e] if int(r[gkey] or 0) == grid and step_re.search(r[key])) == warmup + steps]
    if not timed:
        raise SystemExit(f"no bed at grid {grid} with {warmup + steps} step launches")
    region = rows[timed[0][0]:timed[0][1]]
    tot = {}
    for r in region:
        name = r[key]
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        c, t = tot.get(name, (0, 0.0))
        tot[name] = (c + 1, t + d)
    busy = sum(t for _, t in tot.values())
    span = (int(region[-1]["End_Timestamp"]) - int(region[0]["Start_Timestamp"])) / 1e3
    print(f"Spouted bed ({n} spheres, tuned {sp['tuned']}): kernels of the timed bed, from its creation "
          f"through {warmup} warm-up and {steps} timed steps; {busy / 1e3:.2f} ms of kernel time in a "
          f"{span / 1e3:.2f} ms span")
    print()
    print("| kernel | calls | avg us | total ms | share % |")
    print("|---|---|---|---|---|")
    for name, (c, t) in sorted(tot.items(), key=lambda kv: -kv[1][1])[:args.top]:
        short = name if len(name) <= 72 else name[:69] + "..."
        print(f"| `{short}` | {c} | {t / c:.2f} | {t / 1e3:.3f} | {100.0 * t / busy:.2f} |")
    print()
    print(f"- bench.py in the same run (under the profiler): {sp['ms_per_step']:.4f} ms per step, "
          f"force kernel {sp['force_kernel']['avg_launch_us']:.2f} us per launch (HIP events, replay)")


def batched(args, bench, hbm_peak_gbs=8000.0):
    bt = bench["batched"]
    gf = int(bt["grid_threads"]["force_kick_batch"])
    n, cpe = int(bt["particles"]), 10
    rows = _one(args.trace, "kernel_trace.csv")
    key = "Kernel_Name" if "Kernel_Name" in rows[0] else "Name"
    gkey = "Grid_Size" if "Grid_Size" in rows[0] else "Grid_Size_X"
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    force = [i for i, r in enumerate(rows) if int(r[gkey] or 0) == gf and "force_kick_batch" in r[key]]
    if not force:
        raise SystemExit(f"no force_kick_batch launch at grid {gf}")
    region = rows[force[0]:force[-1] + 1]
    steps = len(force)  # one contact-force launch per bed group and step (beds without rolling friction)
    tot = {}
    for r in region:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        tot.setdefault(r[key], []).append(d)
    busy = sum(sum(v) for v in tot.values())
    print(f"Batched ensemble ({bt['beds']} beds, {n} spheres, tuned {bt['autotune']['config']}): kernels from the "
          f"first to the last contact-force launch at the ensemble's grid ({gf} threads), {steps} DEM steps "
          f"(warm-up chunks included); {busy / steps:.1f} us of kernel time per ensemble step")
    print()
    print("| kernel | calls | mean us | median us | per step us | per particle-step ns |")
    print("|---|---|---|---|---|---|")
    for name, v in sorted(tot.items(), key=lambda kv: -sum(kv[1]))[:args.top]:
        short = name if len(name) <= 72 else name[:69] + "..."
        x = np.array(v)
        print(f"| `{short}` | {len(x)} | {x.mean():.1f} | {np.median(x):.1f} | {x.sum() / steps:.1f} | "
              f"{1e3 * x.sum() / steps / n:.4f} |")
    fk = np.array([(int(rows[i]["End_Timestamp"]) - int(rows[i]["Start_Timestamp"])) / 1e3 for i in force])
    alg = float(bt["algorithmic_bytes_per_step"])
    gbs = alg / (fk.mean() * 1e-6) / 1e9
    print()
    print(f"- `force_kick_batch` at the ensemble's grid: {len(fk)} launches, mean {fk.mean():.1f} us, median "
          f"{np.median(fk):.1f} us; {alg / 1e6:.1f} MB algorithmic per step (184 B per particle, 56 B per "
          f"contact, {bt['contacts_end']} contacts) gives {gbs:.0f} GB/s, {100 * gbs / hbm_peak_gbs:.1f} % of "
          f"the {hbm_peak_gbs:.0f} GB/s HBM peak")
    print(f"- bench.py in the same run (under the profiler): {bt['ms_per_step']:.4f} ms per ensemble step, "
          f"{bt['value']:.4g} particle-steps/s; coupling every {cpe} steps")


if __name__ == "__main__":
    main()

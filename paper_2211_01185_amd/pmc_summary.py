"""HBM traffic of the contact-force kernel from rocprofv3 counter runs.

Inputs: one `rocprofv3 --pmc FETCH_SIZE` and one `--pmc WRITE_SIZE` run of
the benchmark's main measurement (its JSON line saved to a file), and the same
two counters over the plain device copy of calib.py.  The force-kernel
dispatches of the roofline window's replay are selected (the last FP32 bed the
run created at the main bed's launch shape, after its creation-time
evaluation, skipping the window's warm-up steps), each counter is scaled
by true copy bytes / counted copy bytes, and the mean per dispatch is written
as the JSON entry the benchmark reports as roofline.traffic.  The entry is
keyed by the hash of the kernel source and by its launch shape (lanes per
particle, precision); it records the whole configuration it was taken at
(skin, re-sort interval), which the benchmark reports beside it.

    python -m paper_2211_01185_amd.pmc_summary --fetch D1 --write D2 \\
        --cal-fetch D3 --cal-write D4 --bench-json F1 --bench-json-write F2 --out JSON

(F1, F2: the benchmark's output in the two counter runs; both must have run
the same configuration, e.g. by passing bench.py --bed-config.)
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

COPY_KIB = 256 * 1024  # calib.py: 256 MiB read and written per dispatch
KERNEL_SOURCES = [os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", f)
                  for f in ("dem_kernels.hip", "device.h")]


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if len(files) != 1:
        raise SystemExit(f"{d}: expected one counter_collection.csv, found {len(files)}")
    with open(files[0]) as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def _scale(d, counter):
    vals = [float(r["Counter_Value"]) for r in _rows(d)
            if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]]
    big = [v for v in vals if v > 0.25 * COPY_KIB]  # the 256 MiB copies, not torch's small fills
    if not big:
        raise SystemExit(f"{d}: no copy dispatches with {counter}")
    return COPY_KIB / (sum(big) / len(big)), len(big)


def _region(d, counter, lanes, warmup, steps):
    """Counter values of the force-kernel step launches of the last bed the
    run created (the replayed region), after its warm-up."""
    step_re = re.compile(rf"force_kick<float, true, (true|false), {lanes}, false>")
    prime_re = re.compile(rf"force_kick<float, false, false, {lanes}, false>")
    rows = [r for r in _rows(d) if r["Counter_Name"] == counter]
    last_prime = max(i for i, r in enumerate(rows) if prime_re.search(r["Kernel_Name"]))
    launches = [r for r in rows[last_prime + 1:] if step_re.search(r["Kernel_Name"])]
    sel = launches[warmup:warmup + steps]
    if len(sel) != steps:
        raise SystemExit(f"{d}: {len(sel)} step launches after warm-up, expected {steps}")
    return [float(r["Counter_Value"]) for r in sel]


def main(argv=None):
    ap = argparse.ArgumentParser()
    for k in ("fetch", "write", "cal_fetch", "cal_write", "bench_json", "bench_json_write", "out"):
        ap.add_argument("--" + k.replace("_", "-"), required=True)
    args = ap.parse_args(argv)

    def bench_line(path):
        with open(path) as fh:
            return json.loads([ln for ln in fh if ln.startswith("{")][-1])

    bench = bench_line(args.bench_json)
    tuned = bench["config"]["tuned"]
    cfg = {k: tuned[k] for k in ("skin", "resort_every", "lanes")}
    other = bench_line(args.bench_json_write)["config"]["tuned"]
    if {k: other[k] for k in cfg} != cfg:
        raise SystemExit("the two counter runs used different configurations")
    window = bench["roofline"]["window"]
    warmup, steps = int(window["warmup"]), int(window["steps"])
    cfg["precision"] = "fp32"
    fs, nf = _scale(args.cal_fetch, "FETCH_SIZE")
    ws, nw = _scale(args.cal_write, "WRITE_SIZE")
    f = _region(args.fetch, "FETCH_SIZE", cfg["lanes"], warmup, steps)
    w = _region(args.write, "WRITE_SIZE", cfg["lanes"], warmup, steps)
    fk, wk = sum(f) / len(f), sum(w) / len(w)
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:  # the kernel's file and the device layout it includes
        with open(path, "rb") as fh:
            h.update(fh.read())
    sha = h.hexdigest()
    entry = {
        "kernel": f"force_kick<float, true, *, {cfg['lanes']}>",
        "kernel_source_sha256": sha,
        "config": cfg,
        "launches": len(f),
        "fetch_kib_per_launch": fk,
        "write_kib_per_launch": wk,
        "fetch_scale": fs,
        "write_scale": ws,
        "hbm_bytes_per_launch": 1024.0 * (fk * fs + wk * ws),
    }
    with open(args.out, "w") as fh:
        json.dump(entry, fh, indent=1)
        fh.write("\n")
    print(f"| calibration | FETCH_SIZE x{fs:.4f} ({nf} copies) | WRITE_SIZE x{ws:.4f} ({nw} copies) |")
    print(f"| {entry['kernel']} | {len(f)} launches | FETCH {fk:.0f} KiB | WRITE {wk:.0f} KiB | "
          f"{entry['hbm_bytes_per_launch'] / 1e6:.1f} MB scaled |")
    print(f"algorithmic bytes per launch (bench): {bench['roofline']['algorithmic_bytes_per_launch'] / 1e6:.1f} MB")


if __name__ == "__main__":
    main()

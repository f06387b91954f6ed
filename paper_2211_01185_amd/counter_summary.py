"""Hardware counters of the contact-force kernel from rocprofv3 counter runs.

Each run (`rocprofv3 --pmc C1 C2 ...` of the benchmark's main measurement,
its JSON line saved to a file) is reduced to the mean of every counter over
the step launches of the roofline window's replay (as pmc_summary selects
them), and
printed as a markdown table with these ratios where their counters are
present (the SQ cycle counters share one unit, four cycles):

  waiting      SQ_WAIT_ANY / SQ_WAVE_CYCLES: share of the wavefronts'
               lifetime spent waiting for anything (memory results, mostly)
  issue wait   SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES: share spent with an
               instruction waiting to issue
  VALU/wave    SQ_INSTS_VALU / SQ_WAVES
  L2 hits      TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum)

    python -m paper_2211_01185_amd.counter_summary --bench-json F --run D1 [--run D2 ...]
"""
from __future__ import annotations

import argparse
import json

from .pmc_summary import _region, _rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--bench-json", required=True)
    ap.add_argument("--run", action="append", required=True, help="rocprofv3 output directory of one --pmc run")
    args = ap.parse_args(argv)
    with open(args.bench_json) as fh:
        bench = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    lanes = int(bench["config"]["tuned"]["lanes"])
    window = bench["roofline"]["window"]
    warmup, steps = int(window["warmup"]), int(window["steps"])
    means = {}
    for d in args.run:
        for c in sorted({r["Counter_Name"] for r in _rows(d)}):
            v = _region(d, c, lanes, warmup, steps)
            means[c] = sum(v) / len(v)
    print(f"Contact-force kernel `force_kick<float, true, *, {lanes}>`, mean per launch over the "
          f"{steps} step launches of the roofline window's replay:")
    print()
    print("| counter | mean per launch |")
    print("|---|---|")
    for c, v in means.items():
        print(f"| {c} | {v:.4g} |")
    print()
    if "SQ_WAIT_ANY" in means and means.get("SQ_WAVE_CYCLES"):
        print(f"- waiting for anything: {means['SQ_WAIT_ANY'] / means['SQ_WAVE_CYCLES']:.2f} of the wavefront cycles")
    if "SQ_WAIT_INST_ANY" in means and means.get("SQ_WAVE_CYCLES"):
        print(f"- waiting to issue: {means['SQ_WAIT_INST_ANY'] / means['SQ_WAVE_CYCLES']:.2f} of the wavefront cycles")
    if "SQ_INSTS_VALU" in means and means.get("SQ_WAVES"):
        print(f"- VALU instructions per wavefront: {means['SQ_INSTS_VALU'] / means['SQ_WAVES']:.0f}")
    if "TCC_HIT_sum" in means and "TCC_MISS_sum" in means:
        tot = means["TCC_HIT_sum"] + means["TCC_MISS_sum"]
        if tot > 0:
            print(f"- L2 hits: {means['TCC_HIT_sum'] / tot:.3f} of the L2 requests")


if __name__ == "__main__":
    main()

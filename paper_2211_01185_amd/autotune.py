"""Autotuner of the launch and grid choices that do not change the results.

Knobs (dem_params and cfd_params fields):
  * skin          neighbour-list skin, as a multiple of the smallest diameter.
                  It also sets the DEM cell size (cells are at least
                  d_max + skin wide, nested in the mesh elements), so it
                  trades the cost of a broad search against how often one is
                  needed and how long the lists are;
  * resort_every  DEM steps between re-sorts of the particle arrays by cell;
  * lanes         lanes of a wavefront sharing one particle in the
                  contact-force kernel (the tile of list entries per lane);
  * elem_threads  threads per occupied element in the coupling step: 16 or 32
                  (several elements of few particles per wavefront), 64 or
                  128.  A candidate whose trial raises a device error (an
                  element past the capacity of its group) is never kept; a
                  bed that packs its elements denser later than the tuned
                  run reaches may still meet that capacity (256 or 512
                  particles per element for 16 or 32 threads), which the
                  sticky capacity error reports.

None of them changes a contact set, and forces only at the rounding level
(the order of a particle's contact sums depends on its list layout, that of
an element's sums on the threads computing it), which the invariance tests
check.  The tuner times coupled runs (a coupling step every
10 DEM steps, as the workloads run) from the beds' initial state on the device
for candidate values, one knob at a time starting from the defaults
(coordinate descent), and keeps the fastest.  Runs should be as long as the
runs being tuned for: a bed that starts at rest rebuilds its lists rarely at
first, which favours small skins on short runs.  Results are cached in a JSON file keyed by a signature of the
workload.
"""
from __future__ import annotations

import json
import os
import time

from . import cfddem

CANDIDATES = {
    "skin_factor": (0.05, 0.1, 0.2, 0.35),
    "resort_every": (25, 50, 100, 200),
    "lanes": (1, 2, 4),
    "elem_threads": (16, 32, 64, 128),
}
DEFAULT = {"skin_factor": 0.1, "resort_every": 100, "lanes": 2, "elem_threads": 128}
COUPLING_EVERY = 10


def cache_path() -> str:
    return os.environ.get("CFDDEM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "cfddem", "tune.json"))


def _load_cache() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(key: str, value: dict):
    data = _load_cache()
    data[key] = value
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass  # a read-only home only loses the cache


def bed_kwargs(wl, cfg: dict) -> dict:
    """Keyword arguments of cfddem.Bed for a tuned configuration."""
    d_min = 2.0 * float(wl.radius.min())
    return dict(skin=cfg["skin_factor"] * d_min, resort_every=int(cfg["resort_every"]), lanes=int(cfg["lanes"]),
                elem_threads=int(cfg.get("elem_threads", DEFAULT["elem_threads"])))


def signature(wls, precision) -> str:
    """Workload signature: what the best choice depends on (sizes, packing,
    fluid speed), rounded so that draws of the same recipe share an entry."""
    import numpy as np

    n = sum(w.n for w in wls)
    d = np.median([2.0 * float(np.median(w.radius)) for w in wls])
    u = np.median([float(np.abs(w.U[2]).mean()) if w.U is not None else 0.0 for w in wls])
    return f"{precision}|beds={len(wls)}|n~{float(f'{n:.1g}')}|d~{float(f'{d:.1g}')}|u~{u:.1f}"


def _time_single(wl, field, cfg, precision, steps, device):
    """One bed through the single-bed entry points (the path such a bed runs on)."""
    import torch

    bed = cfddem.bed_from_workload(wl, precision=precision, device=device, **bed_kwargs(wl, cfg))
    try:
        U, P = field
        out = bed.couple(U, P)
        chunks = max(1, steps // COUPLING_EVERY)

        def run(k):
            for _ in range(k):
                bed.couple(U, P, out=out)
                bed.step(COUPLING_EVERY)

        run(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(chunks)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = bed.poll()[0] == 0
    finally:
        bed.close()
    return dt / (chunks * COUPLING_EVERY) if ok else float("inf")


def _time_batch(wls, fields, cfg, precision, steps, device):
    import torch

    if len(wls) == 1:
        return _time_single(wls[0], fields[0], cfg, precision, steps, device)
    beds = [cfddem.bed_from_workload(w, precision=precision, device=device, **bed_kwargs(w, cfg)) for w in wls]
    try:
        batch = cfddem.Batch(beds, fields)
        chunks = max(1, steps // COUPLING_EVERY)
        batch.run(2, COUPLING_EVERY, couple=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.run(chunks, COUPLING_EVERY, couple=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = all(b.poll()[0] == 0 for b in beds)
        batch.close()
    finally:
        for b in beds:
            b.close()
    return dt / (chunks * COUPLING_EVERY) if ok else float("inf")


def tune(wls, precision="fp32", steps=100, device="cuda", use_cache=True, sample=8, min_gain=0.01):
    """Best configuration for running these beds, tuned on up to `sample` of
    them: one bed is timed through the single-bed entry points, several as a
    batch.  A candidate replaces the current best only when it is faster by
    more than `min_gain` (relative), and still so when both are timed once
    more (each keeps its fastest run), so that timing noise does not move the
    choice.  Returns (config, report)."""
    import torch

    key = signature(wls, precision)
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            return dict(hit["config"]), dict(hit, cached=True)
    sub = list(wls)[:sample]
    fields = [(torch.as_tensor(w.U, dtype=torch.float64, device=device).contiguous(),
               torch.as_tensor(w.P, dtype=torch.float64, device=device).contiguous()) for w in sub]
    best = dict(DEFAULT)
    trials = {}

    def timed(cfg, again=False):
        k = json.dumps(cfg, sort_keys=True)
        if k not in trials or again:
            trials.setdefault(k, []).append(_time_batch(sub, fields, cfg, precision, steps, device))
        return min(trials[k])

    t_best = timed(best)
    for knob, values in CANDIDATES.items():
        for v in values:
            cfg = dict(best, **{knob: v})
            t = timed(cfg)
            if t < t_best * (1.0 - min_gain):
                t, t_b = timed(cfg, again=True), timed(best, again=True)
                if t < t_b * (1.0 - min_gain):
                    best, t_best = cfg, t
                else:
                    t_best = t_b
    report = {"config": best, "ms_per_step": t_best * 1e3,
              "default_ms_per_step": min(trials[json.dumps(DEFAULT, sort_keys=True)]) * 1e3,
              "trials": sum(len(v) for v in trials.values()), "configs": len(trials), "tuned_on_beds": len(sub),
              "signature": key, "cached": False}
    if use_cache:
        _store_cache(key, {k: v for k, v in report.items() if k != "cached"})
    return best, report

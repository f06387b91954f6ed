"""Throughput benchmark of the particle-side CFD-DEM hot path on one MI355X.

Workload: the fluidized-bed slice (100,000 spheres, d = 1 mm, jittered lattice
at solid fraction 0.4 in 0.1 x 0.1 x 0.4 m; Q2 20x20x80 mesh with 864,000
quadrature points; fluid velocity (0,0,1.2) m/s + N(0, 0.05) per node and a
linear pressure; FP32 force/drag arithmetic with FP64 state; one coupling
step every 10 DEM steps).  A "step" is one DEM step; the coupling step that
falls on every tenth step is inside the timed region.  Inputs are generated
and copied to HBM before timing.

Prints ONE JSON line: metric/value (particle-steps/s) over K timed steps; the
roofline of the dominant kernel (contact search + forces), measured with HIP
events bound to each of its launches while the same K steps are replayed on a
fresh bed (the runs are deterministic); and the CPU oracle timed on a bounded
sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DEM+coupling particle-steps/s @100k spheres; batched jobs/s + p99 latency"
HBM_PEAK_GBS = 8000.0
COUPLING_EVERY = 10
RESORT_EVERY = 100
# algorithmic bytes of the contact-force kernel: per particle it must read
# x, v_half, w_half (72 B), radius and mass (16 B), the held fluid force (24 B)
# and write v, w (48 B); per contact (pair or wall) read + write the tangential
# overlap (48 B) and the partner index (8 B).
FORCE_BYTES_PER_PARTICLE = 160
BYTES_PER_CONTACT = 56
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_kick_fluidized_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2211_01185_amd", "csrc", "dem_kernels.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=100)
    return ap.parse_args()


def kernel_source_sha():
    with open(KERNEL_SOURCE, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def traffic_entry(n_contacts):
    """HBM bytes per launch of the force kernel from the committed rocprofv3
    counter summary, or None if it is absent or the kernel changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha256") != kernel_source_sha():
        return None
    return float(t["hbm_bytes_per_launch"])


def contact_counts(bed):
    i, j, _ = bed.read_contacts()
    walls = int((j < 0).sum())
    return len(i) - walls, walls


def cpu_baseline(wl, dem_steps):
    """The FP64 oracle, as it stands, on the same bed: dem_steps DEM steps with
    a coupling step every COUPLING_EVERY steps."""
    from oracle import oracle as O

    d, f = wl.dem, wl.fluid
    p = O.make_params(d["box_lo"], d["box_hi"], d["gravity"], d["dt"], d["E"], d["nu"], d["e"], d["mu"],
                      d["E_w"], d["nu_w"], d["e_w"], d["mu_w"])
    fl = O.make_fluid(f["order"], f["n_el"], f["rho_f"], f["mu_f"], f["model"], f["eps_min"])
    bed = O.OracleBed(p, wl.x, wl.v, wl.w, wl.radius, wl.density)
    t0 = time.perf_counter()
    for s in range(dem_steps):
        if s % COUPLING_EVERY == 0:
            bed.couple(fl, wl.U, wl.P)
        bed.step(1)
    dt = time.perf_counter() - t0
    return {"value": wl.n * dem_steps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{dem_steps} DEM steps + {dem_steps // COUPLING_EVERY} coupling steps of the same "
                      f"{wl.n}-sphere bed, single-threaded FP64 C oracle, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(beds shard by bed or by z-slab, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2211_01185_amd import cfddem, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    wl = synth.fluidized()
    U = torch.as_tensor(wl.U, dtype=torch.float64, device=dev).contiguous()
    P = torch.as_tensor(wl.P, dtype=torch.float64, device=dev).contiguous()

    def make_bed():
        bed = cfddem.bed_from_workload(wl, precision="fp32", device=dev, resort_every=RESORT_EVERY)
        out = bed.couple(U, P)  # allocates the output tensors once; the run re-couples at step 0
        return bed, out

    def run(bed, out, steps, start):
        s = start
        end = start + steps
        while s < end:
            if s % COUPLING_EVERY == 0:
                bed.couple(U, P, out=out)
            chunk = min(COUPLING_EVERY - s % COUPLING_EVERY, end - s)
            bed.step(chunk)
            s += chunk
        return s

    # throughput: W warmup steps, then exactly K timed steps without per-kernel
    # instrumentation
    bed, out = make_bed()
    stream = bed.stream
    step = run(bed, out, args.warmup, 0)
    torch.cuda.synchronize()
    err, _ = bed.poll()
    if err:
        raise SystemExit(f"device error after warmup: {cfddem.status_string(err)}")
    pairs0, walls0 = contact_counts(bed)
    start_ev = torch.cuda.Event(enable_timing=True)
    stop_ev = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start_ev.record(stream)
    step = run(bed, out, args.steps, step)
    stop_ev.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = start_ev.elapsed_time(stop_ev)
    err, _ = bed.poll()
    if err:
        raise SystemExit(f"device error in the timed region: {cfddem.status_string(err)}")
    pairs1, walls1 = contact_counts(bed)
    bed.close()
    del bed, out

    # roofline: the same deterministic trajectory replayed on a fresh bed, with
    # HIP events bound to every launch of the contact-force kernel on its
    # stream during the same K steps (the events add launch latency, so this
    # replay is not used for the throughput)
    bed, out = make_bed()
    step = run(bed, out, args.warmup, 0)
    bed.kernel_timing(True)
    step = run(bed, out, args.steps, step)
    torch.cuda.synchronize()
    bed.kernel_timing(False)
    launches, force_ms = bed.kernel_timing_read()
    pairs2, walls2 = contact_counts(bed)
    bed.close()

    elapsed = max(wall, gpu_ms / 1e3)
    value = wl.n * args.steps / elapsed
    contacts = 0.5 * (pairs0 + walls0 + pairs2 + walls2)
    force_avg_s = force_ms / 1e3 / max(launches, 1)
    alg_bytes = FORCE_BYTES_PER_PARTICLE * wl.n + BYTES_PER_CONTACT * contacts
    achieved = alg_bytes / force_avg_s / 1e9
    traffic = traffic_entry(contacts)

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 forces / f64 state",
        "data": "synthetic",
        "config": {
            "workload": "fluidized-bed slice: 100,000 spheres d=1 mm, solid fraction 0.4, "
                        "Q2 20x20x80 mesh (864,000 qpts), coupling every 10 DEM steps",
            "particles": wl.n,
            "mesh": "Q2 20x20x80",
            "coupling_every": COUPLING_EVERY,
            "precision": "FP32 pair-force and drag arithmetic, FP64 positions/velocities/history/sums",
            "contacts_pairs_walls": [int(round(0.5 * (pairs0 + pairs1))), int(round(0.5 * (walls0 + walls1)))],
            "resort_every": RESORT_EVERY,
            "parallelism": "1 GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "force_kick (contact search + Hertz-Mindlin forces + second half kick)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "avg_launch_us": force_avg_s * 1e6,
            "launches": launches,
            "algorithmic_bytes_per_launch": alg_bytes,
        },
    }
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

"""Throughput benchmark of the particle-side CFD-DEM hot path on one MI355X.

Workload: the fluidized-bed slice (100,000 spheres, d = 1 mm, jittered lattice
at solid fraction 0.4 in 0.1 x 0.1 x 0.4 m; Q2 20x20x80 mesh with 864,000
quadrature points; fluid velocity (0,0,1.2) m/s + N(0, 0.05) per node and a
linear pressure; FP32 force/drag arithmetic with FP64 state; one coupling
step every 10 DEM steps).  A "step" is one DEM step; the coupling step that
falls on every tenth step is inside the timed region.  Inputs are generated
and copied to HBM before timing.

Prints ONE JSON line: metric/value (particle-steps/s) over K timed steps; the
roofline of the dominant kernel (contact search + forces) over a fixed window,
the same for every K: a fresh bed run 20 steps, then 1,000 steps measured with
their re-sorts, broad searches and coupling steps, once without
instrumentation (the whole step's time) and once replayed on a fresh bed with
HIP events bound to each launch of the kernel (the runs are deterministic);
beside the kernel's fraction of the HBM peak, the whole step's (algorithmic
bytes of a DEM step plus a tenth of a coupling step over the time per step);
the CPU oracle timed on a bounded sample of the same workload at one thread
and at all the threads the process may use; and the other parts of the
metric:

  fp64:    the same bed and window with all arithmetic in FP64;
  plain_fp64_2k: the plain FP64 configuration (2,000 spheres d = 3 mm, Q2
           4x4x16, 100 DEM steps with a coupling step every 10), fresh beds,
           median of 5 runs;
  batched: 64 independent column beds (5k-80k spheres each, their own
           diameter, restitution, inlet velocity and Q1 mesh) advanced 1,000
           steps by shared launches replayed from a HIP graph (FP32 forces),
           next to the same beds run one by one through the single-bed FP64
           path;
  served:  a Poisson stream (20 jobs/s) of sedimentation / fluidization jobs of
           1k-200k spheres, served by continuous batching; p50/p99 latency and
           aggregate particle-steps/s over the jobs after the warm-up ones;
  smoothing: the benchmark bed with the smoothed void fraction (L^2 = 5 d^2):
           200 coupled steps, and the first coupling step timed alone;
  packed:  the main measurement on a physically packed bed: the settling run's
           bed at rest, then the fluidized bed's fluid from that state
           (far more contacts than the lattice), tuned on that bed;
  spouted: the 500,000-sphere polydisperse spouted bed (Q2 30x30x120, Gaussian
           jet), tuned, 500 coupled steps after 20 warm-up ones, with the
           contact-force kernel's launches timed on a replay;
  settling: the DEM-only preparation of a bed, 100,000 spheres (d = 1 mm)
           inserted at random above the floor of the same column and stepped
           without coupling until at rest (kinetic energy below 1e-4 of
           sum m g d, checked every 500 steps); steps to rest and
           particle-steps/s.

Beside particle-steps/s the main line gives contacts/s (contact pairs and
wall contacts resolved per second) and quadrature-points/s (points of the
coupling steps per second).  The CPU leg also compares both GPU paths (FP32
forces, all FP64) with the oracle on the main bed: the first coupling and DEM
step, and the end of the oracle's sample; on the first coupling and DEM
step, the spouted bed's path and a batched bed's path (FP32 forces); and the
plain FP64 configuration's whole run.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                       [--no-batched] [--no-served] [--no-smoothing] [--no-spouted]
                       [--no-packed] [--no-settling] [--no-fp64] [--no-config1]
                       [--served-jobs J] [--bed-config JSON]
"""
import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DEM+coupling particle-steps/s @100k spheres; batched jobs/s + p99 latency"
HBM_PEAK_GBS = 8000.0
COUPLING_EVERY = 10
RESORT_EVERY = 100


def _force_block():
    """Threads per block of the contact-force kernels, as the library's device
    header defines them (the batched line reports the grid it launches)."""
    hdr = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2211_01185_amd", "csrc", "device.h")
    with open(hdr) as f:
        return int(re.search(r"constexpr int kForceBlock = (\d+);", f.read()).group(1))


FORCE_BLOCK = _force_block()
# algorithmic bytes of one DEM step (one launch of the contact-force kernel):
# per particle it must read x, v_half, w_half (72 B), radius and mass (16 B) and
# the held fluid force (24 B), and write the next step's x, v_half, w_half
# (72 B); per contact (pair or wall) read + write the tangential overlap (48 B)
# and read the partner index (8 B).
FORCE_BYTES_PER_PARTICLE = 184
BYTES_PER_CONTACT = 56
# algorithmic bytes of one coupling step: per particle read x, v, r and its
# element (60 B) and write f_fp (24 B); per occupied element read its share of
# the velocity nodes (8 nodes x 24 B for Q2, 1 x 24 B for Q1) and of the
# pressure nodes (8 B); per quadrature point write eps, beta and F_pf (40 B)
CPL_BYTES_PER_PARTICLE = 84
CPL_NODE_BYTES = {1: 24, 2: 192}
CPL_PRESSURE_BYTES = 8
CPL_BYTES_PER_QPT = 40
# the roofline window: a fresh bed run WINDOW_WARMUP steps, then WINDOW_STEPS
# steps (with their re-sorts, broad searches and coupling steps) measured,
# whatever the timed region's length
WINDOW_WARMUP = 20
WINDOW_STEPS = 1000
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_kick_fluidized_traffic.json")
# the contact-force kernel's source: its file and the device layout it includes
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2211_01185_amd", "csrc", f) for f in ("dem_kernels.hip", "device.h")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--bed-config", default=None,
                    help="JSON of the main bed's skin, resort_every, lanes and elem_threads, used instead "
                         "of tuning "
                         "(to repeat a tuned run under a counter profiler)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched ensemble")
    ap.add_argument("--no-served", action="store_true", help="skip the served stream")
    ap.add_argument("--no-settling", action="store_true", help="skip the DEM-only settling run")
    ap.add_argument("--no-smoothing", action="store_true", help="skip the smoothed void-fraction run")
    ap.add_argument("--no-spouted", action="store_true", help="skip the spouted-bed run")
    ap.add_argument("--no-packed", action="store_true", help="skip the packed-bed run")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 line of the 100k bed")
    ap.add_argument("--no-config1", action="store_true", help="skip the plain FP64 2,000-sphere line")
    ap.add_argument("--batched-beds", type=int, default=64)
    ap.add_argument("--batched-steps", type=int, default=1000)
    ap.add_argument("--served-jobs", type=int, default=650)
    ap.add_argument("--served-warmup", type=int, default=50)
    return ap.parse_args()


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha():
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_entry(lanes, precision="fp32"):
    """HBM bytes per launch of the force kernel from the committed rocprofv3
    counter summary, with the configuration they were taken at, or (None,
    None) if it is absent or the kernel source or its launch shape (lanes per
    particle, precision) differs."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha256") != kernel_source_sha():
        return None, None
    cfg = t.get("config") or {}
    if cfg.get("lanes") != lanes or cfg.get("precision", "fp32") != precision:
        return None, None
    return float(t["hbm_bytes_per_launch"]), cfg


def occupied_elements(wl, x):
    """Mesh elements holding at least one particle centre (x: 3 x n)."""
    import numpy as np

    lo = np.asarray(wl.dem["box_lo"], dtype=np.float64)[:, None]
    hi = np.asarray(wl.dem["box_hi"], dtype=np.float64)[:, None]
    n_el = np.asarray(wl.fluid["n_el"], dtype=np.int64)[:, None]
    e = np.clip(np.floor((x - lo) / (hi - lo) * n_el).astype(np.int64), 0, n_el - 1)
    return int(np.unique((e[2] * n_el[1] + e[1]) * n_el[0] + e[0]).size)


def coupling_bytes(wl, n_occ):
    """Algorithmic bytes of one coupling step with n_occ occupied elements."""
    order = int(wl.fluid["order"])
    n_el = int(wl.fluid["n_el"][0]) * int(wl.fluid["n_el"][1]) * int(wl.fluid["n_el"][2])
    return (CPL_BYTES_PER_PARTICLE * wl.n + n_occ * (CPL_NODE_BYTES[order] + CPL_PRESSURE_BYTES)
            + CPL_BYTES_PER_QPT * n_el * (order + 1) ** 3)


def contact_counts(bed):
    i, j, _ = bed.read_contacts()
    walls = int((j < 0).sum())
    return len(i) - walls, walls


def make_coupled_bed(wl, U, P, bed_kw, dev, precision="fp32"):
    from paper_2211_01185_amd import cfddem

    bed = cfddem.bed_from_workload(wl, precision=precision, device=dev, **bed_kw)
    out = bed.couple(U, P)  # allocates the output tensors once; the run re-couples at step 0
    return bed, out


def run_coupled(bed, out, U, P, steps, start):
    """Steps start .. start+steps-1, with a coupling step before every step
    whose index is a multiple of COUPLING_EVERY."""
    s = start
    end = start + steps
    while s < end:
        if s % COUPLING_EVERY == 0:
            bed.couple(U, P, out=out)
        chunk = min(COUPLING_EVERY - s % COUPLING_EVERY, end - s)
        bed.step(chunk)
        s += chunk
    return s


def couplings_in(start, steps):
    return sum(1 for s in range(start, start + steps) if s % COUPLING_EVERY == 0)


def cpu_info():
    """The host CPU as lscpu reports it, and the threads this process may run
    (its CPU affinity, capped by OMP_NUM_THREADS when set and by the physical
    cores)."""
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass

    def num(key):
        try:
            return int(info.get(key, ""))
        except ValueError:
            return None

    sockets, per_socket, per_core = num("Socket(s)"), num("Core(s) per socket"), num("Thread(s) per core")
    physical = sockets * per_socket if sockets and per_socket else None
    threads = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        threads = min(threads, int(env))
    if physical:
        threads = min(threads, physical)
    return {"model": info.get("Model name"), "sockets": sockets, "physical_cores": physical,
            "threads_per_core": per_core, "logical_cpus": num("CPU(s)"),
            "affinity_cpus": len(os.sched_getaffinity(0)), "threads_used": max(1, threads)}


def oracle_sample(wl, dem_steps, keep=False):
    """One timed run of the oracle on the bed: dem_steps DEM steps with a
    coupling step every COUPLING_EVERY steps (creation not timed).  With
    keep, also the first coupling step's outputs, the state after the first
    step and the state at the end (copied outside the timed steps)."""
    from oracle import oracle as O

    d, f = wl.dem, wl.fluid
    p = O.make_params(d["box_lo"], d["box_hi"], d["gravity"], d["dt"], d["E"], d["nu"], d["e"], d["mu"],
                      d["E_w"], d["nu_w"], d["e_w"], d["mu_w"])
    fl = O.make_fluid(f["order"], f["n_el"], f["rho_f"], f["mu_f"], f["model"], f["eps_min"])
    bed = O.OracleBed(p, wl.x, wl.v, wl.w, wl.radius, wl.density)
    ref = {}
    dt = 0.0
    for s in range(dem_steps):
        t0 = time.perf_counter()
        if s % COUPLING_EVERY == 0:
            r = bed.couple(fl, wl.U, wl.P)
        bed.step(1)
        dt += time.perf_counter() - t0
        if keep and s == 0:
            ref["couple"] = r
            ref["step1"] = bed.state()
    if keep:
        ref["end"] = bed.state()
    return dt, ref


def cpu_baseline(wl, dem_steps, repeats=3):
    """The FP64 oracle, as it stands, on the same bed: dem_steps DEM steps with
    a coupling step every COUPLING_EVERY steps, timed at one thread and at all
    the threads this process may use, median of `repeats` runs each (the
    oracle's results do not depend on its thread count).  Also returns what
    the GPU paths are compared with (from the first run)."""
    import statistics

    from oracle import oracle as O

    cpu = cpu_info()
    times, ref = {}, None
    for threads in (1, cpu["threads_used"]):
        O.set_threads(threads)
        ts = []
        for _ in range(repeats):
            dt, r = oracle_sample(wl, dem_steps, keep=ref is None)
            ref = ref or r
            ts.append(dt)
        times[threads] = statistics.median(ts)
    nt = cpu["threads_used"]
    rate = {t: wl.n * dem_steps / v for t, v in times.items()}
    out = {"value": rate[nt], "unit": "particle-steps/s", "cores": nt, "kind": "oracle",
           "cpu_model": cpu["model"], "physical_cores": cpu["physical_cores"],
           "threads_per_core": cpu["threads_per_core"], "affinity_cpus": cpu["affinity_cpus"],
           "one_core": {"value": rate[1], "unit": "particle-steps/s", "cores": 1, "seconds": times[1]},
           "all_cores": {"value": rate[nt], "unit": "particle-steps/s", "cores": nt, "seconds": times[nt]},
           "sample": f"{dem_steps} DEM steps + {dem_steps // COUPLING_EVERY} coupling steps of the same "
                     f"{wl.n}-sphere bed, FP64 C oracle (OpenMP over independent per-particle, per-contact "
                     f"and per-element work; sums serial), median of {repeats} runs at 1 thread "
                     f"({times[1]:.1f} s) and at {nt} threads ({times[nt]:.1f} s)"}
    return out, ref


def rel_max_err(got, want):
    """max|got - want| / max|want| (the parity tests' measure)."""
    import numpy as np

    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = float(np.max(np.abs(want)))
    diff = float(np.max(np.abs(got - want)))
    return diff / scale if scale > 0.0 else diff


def first_step_errors(c, st, F, T, ref):
    """The parity tests' measure on the first coupling step (c: eps_q, beta_q,
    fpf_q) and the first DEM step (st: state, F, T: contact force and torque)."""
    o1 = ref["step1"]
    return {"eps_q": rel_max_err(c["eps_q"], ref["couple"]["eps_q"]),
            "beta_q": rel_max_err(c["beta_q"], ref["couple"]["beta_q"]),
            "fpf_q": rel_max_err(c["fpf_q"], ref["couple"]["fpf_q"]),
            "f_fp": rel_max_err(st["ffp"], o1["ffp"]),
            "contact_force": rel_max_err(F, o1["Fc"]), "contact_torque": rel_max_err(T, o1["Tc"]),
            "x": rel_max_err(st["x"], o1["x"]), "v": rel_max_err(st["v"], o1["v"]),
            "w": rel_max_err(st["w"], o1["w"])}


def oracle_first_step(wl):
    """The FP64 oracle's first coupling step and first DEM step on a workload."""
    from oracle import oracle as O

    d, f = wl.dem, wl.fluid
    p = O.make_params(d["box_lo"], d["box_hi"], d["gravity"], d["dt"], d["E"], d["nu"], d["e"], d["mu"],
                      d["E_w"], d["nu_w"], d["e_w"], d["mu_w"])
    fl = O.make_fluid(f["order"], f["n_el"], f["rho_f"], f["mu_f"], f["model"], f["eps_min"])
    bed = O.OracleBed(p, wl.x, wl.v, wl.w, wl.radius, wl.density)
    r = bed.couple(fl, wl.U, wl.P)
    bed.step(1)
    return {"couple": r, "step1": bed.state()}


def gpu_first_step_errors(wl, ref, dev, bed_kw, batch=False):
    """A GPU bed (FP32 forces) from the same inputs as the oracle: its first
    coupling step and first DEM step, through the single-bed entry points or
    as a batch of one (the batched kernels and graph replay)."""
    import torch

    from paper_2211_01185_amd import cfddem

    U = torch.as_tensor(wl.U, dtype=torch.float64, device=dev).contiguous()
    P = torch.as_tensor(wl.P, dtype=torch.float64, device=dev).contiguous()
    bed = cfddem.bed_from_workload(wl, precision="fp32", device=dev, **bed_kw)
    if batch:
        b = cfddem.Batch([bed], [(U, P)])
        out = b.couple()[0]
        c = {k: out[k].cpu().numpy() for k in ("eps_q", "beta_q", "fpf_q")}
        b.step(1)
        torch.cuda.synchronize()
        b.close()
    else:
        out = bed.couple(U, P)
        c = {k: out[k].cpu().numpy() for k in ("eps_q", "beta_q", "fpf_q")}
        bed.step(1)
    st = {k: v.cpu().numpy() for k, v in bed.read_state().items()}
    F, T = (t.cpu().numpy() for t in bed.read_forces())
    err, _ = bed.poll()
    bed.close()
    e = first_step_errors(c, st, F, T, ref)
    e["errors"] = int(err)
    return e


def errors_vs_oracle(wl, U, P, bed_kw, dev, ref, dem_steps):
    """The GPU paths (FP32 forces / FP64 state, and all FP64) against the FP64
    oracle on the main bed: the first coupling step and the first DEM step
    (where the paths must agree to 1e-5 and 1e-10 relative), and the state
    after the oracle's whole sample (a trajectory: reported, not bounded)."""
    import numpy as np

    res = {}
    for precision in ("fp32", "fp64"):
        bed, out = make_coupled_bed(wl, U, P, bed_kw, dev, precision)
        c = {k: out[k].cpu().numpy() for k in ("eps_q", "beta_q", "fpf_q")}
        bed.step(1)
        st = {k: v.cpu().numpy() for k, v in bed.read_state().items()}
        F, T = (t.cpu().numpy() for t in bed.read_forces())
        e = first_step_errors(c, st, F, T, ref)
        run_coupled(bed, out, U, P, dem_steps - 1, 1)
        st = {k: v.cpu().numpy() for k, v in bed.read_state().items()}
        err, _ = bed.poll()
        bed.close()
        d_min = 2.0 * float(wl.radius.min())
        e[f"x_after_{dem_steps}_steps_over_d"] = float(np.max(np.abs(st["x"] - ref["end"]["x"]))) / d_min
        e[f"v_after_{dem_steps}_steps"] = rel_max_err(st["v"], ref["end"]["v"])
        e["errors"] = int(err)
        res[precision] = e
    return {"measure": "max|gpu - oracle| / max|oracle| per array after the first coupling step and the first "
                       "DEM step; the end state of the oracle's sample as a trajectory deviation",
            "bound_single_step": {"fp32": 1e-5, "fp64": 1e-10}, **res}


def measure_coupled(wl, U, P, bed_kw, dev, steps, warmup, precision="fp32"):
    """`warmup` + `steps` coupled steps of a fresh bed with the `steps` timed
    (wall clock and HIP events on the bed's stream), then the same steps
    replayed on another fresh bed with the contact-force kernel's launches
    timed by HIP events (the runs are deterministic).  Returns the timing,
    the force kernel's roofline and the whole step's: algorithmic bytes of a
    DEM step plus a tenth of a coupling step over the measured time per
    step."""
    import torch

    bed, out = make_coupled_bed(wl, U, P, bed_kw, dev, precision)
    s = run_coupled(bed, out, U, P, warmup, 0)
    torch.cuda.synchronize()
    pairs0, walls0 = contact_counts(bed)
    occ0 = occupied_elements(wl, bed.read_state()["x"].cpu().numpy())
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(bed.stream)
    run_coupled(bed, out, U, P, steps, s)
    ev1.record(bed.stream)
    torch.cuda.synchronize()
    wall = max(time.perf_counter() - t0, ev0.elapsed_time(ev1) / 1e3)
    err, _ = bed.poll()
    pairs1, walls1 = contact_counts(bed)
    occ1 = occupied_elements(wl, bed.read_state()["x"].cpu().numpy())
    nq_total = bed.n_elem * bed.nq
    bed.close()
    bed, out = make_coupled_bed(wl, U, P, bed_kw, dev, precision)
    s = run_coupled(bed, out, U, P, warmup, 0)
    bed.kernel_timing(True)
    run_coupled(bed, out, U, P, steps, s)
    torch.cuda.synchronize()
    bed.kernel_timing(False)
    launches, force_ms = bed.kernel_timing_read()
    err2, _ = bed.poll()
    bed.close()
    contacts = 0.5 * (pairs0 + walls0 + pairs1 + walls1)
    force_avg_s = force_ms / 1e3 / max(launches, 1)
    alg_bytes = FORCE_BYTES_PER_PARTICLE * wl.n + BYTES_PER_CONTACT * contacts
    achieved = alg_bytes / force_avg_s / 1e9
    n_occ = 0.5 * (occ0 + occ1)
    step_bytes = alg_bytes + coupling_bytes(wl, n_occ) / COUPLING_EVERY
    step_s = wall / steps
    return {"wall": wall, "errors": int(err or err2), "nq_total": nq_total, "contacts": contacts,
            "pairs_walls": [int(round(0.5 * (pairs0 + pairs1))), int(round(0.5 * (walls0 + walls1)))],
            "force_kernel": {"avg_launch_us": force_avg_s * 1e6, "launches": launches,
                             "algorithmic_bytes_per_launch": alg_bytes, "achieved_GBs": achieved,
                             "frac_of_hbm_peak": achieved / HBM_PEAK_GBS},
            "whole_step": {"us_per_step": step_s * 1e6, "algorithmic_bytes_per_step": step_bytes,
                           "occupied_elements": n_occ, "achieved_GBs": step_bytes / step_s / 1e9,
                           "frac_of_hbm_peak": step_bytes / step_s / 1e9 / HBM_PEAK_GBS,
                           "bytes": "184 B/particle + 56 B/contact per DEM step, plus a tenth of "
                                    "84 B/particle + (node share + 8 B)/occupied element + 40 B/quadrature point"}}


def config1_run(dev, repeats=5):
    """The plain FP64 configuration (2,000 spheres d = 3 mm in 0.05 x 0.05 x
    0.2 m, Q2 4x4x16 with a uniform 0.5 m/s upflow): its 100 DEM steps with a
    coupling step every 10, all FP64, from a fresh bed each time (creation not
    timed); median of `repeats` runs."""
    import statistics

    import torch

    from paper_2211_01185_amd import synth

    wl = synth.plain()
    U = torch.as_tensor(wl.U, dtype=torch.float64, device=dev).contiguous()
    P = torch.as_tensor(wl.P, dtype=torch.float64, device=dev).contiguous()
    steps = int(wl.run["steps"])
    times, errs, contacts = [], 0, 0
    for _ in range(repeats):
        bed, out = make_coupled_bed(wl, U, P, dict(resort_every=RESORT_EVERY), dev, "fp64")
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(bed.stream)
        run_coupled(bed, out, U, P, steps, 0)
        ev1.record(bed.stream)
        torch.cuda.synchronize()
        times.append(max(time.perf_counter() - t0, ev0.elapsed_time(ev1) / 1e3))
        err, contacts = bed.poll()
        errs += 1 if err else 0
        bed.close()
    t = statistics.median(times)
    return {"workload": "plain FP64: 2,000 spheres d = 3 mm, rho 2500, random non-overlapping in "
                        "0.05 x 0.05 x 0.2 m, Q2 4x4x16 mesh with a uniform (0, 0, 0.5) m/s field, "
                        f"Di Felice, {steps} DEM steps with a coupling step every {COUPLING_EVERY}",
            "particles": wl.n, "steps": steps, "value": wl.n * steps / t, "unit": "particle-steps/s",
            "ms_per_step": t * 1e3 / steps, "ms_per_run": t * 1e3, "runs": repeats,
            "contacts_end": int(contacts), "errors": errs, "dtype": "f64",
            "launch": "single-bed entry points, fresh bed per run"}


def config1_errors(dev):
    """The plain FP64 configuration's whole run (100 steps) on the GPU against
    the oracle: the parity tests' measure on x, v and w at the end."""
    import numpy as np
    import torch

    from paper_2211_01185_amd import synth

    wl = synth.plain()
    steps = int(wl.run["steps"])
    _, ref = oracle_sample(wl, steps, keep=True)
    U = torch.as_tensor(wl.U, dtype=torch.float64, device=dev).contiguous()
    P = torch.as_tensor(wl.P, dtype=torch.float64, device=dev).contiguous()
    bed, out = make_coupled_bed(wl, U, P, dict(resort_every=RESORT_EVERY), dev, "fp64")
    run_coupled(bed, out, U, P, steps, 0)
    st = {k: v.cpu().numpy() for k, v in bed.read_state().items()}
    err, _ = bed.poll()
    bed.close()
    d = 2.0 * float(wl.radius.min())
    return {f"x_after_{steps}_steps_over_d": float(np.max(np.abs(st["x"] - ref["end"]["x"]))) / d,
            f"v_after_{steps}_steps": rel_max_err(st["v"], ref["end"]["v"]),
            f"w_after_{steps}_steps": rel_max_err(st["w"], ref["end"]["w"]), "errors": int(err)}


def spouted_run(dev, steps=500, warmup=20):
    """The spouted bed (500,000 polydisperse spheres, Q2 30x30x120, Gaussian
    jet), FP32 forces: tuned as the main bed, then `warmup` + `steps` coupled
    steps timed as the main measurement, and the same steps replayed on a
    fresh bed with the contact-force kernel's launches timed.  Returns the
    result, the workload and the tuned bed keyword arguments."""
    import torch

    from paper_2211_01185_amd import autotune, synth

    t0 = time.perf_counter()
    wl = synth.spouted()
    gen_s = time.perf_counter() - t0
    U = torch.as_tensor(wl.U, dtype=torch.float64, device=dev).contiguous()
    P = torch.as_tensor(wl.P, dtype=torch.float64, device=dev).contiguous()
    tuned, tune_report = autotune.tune([wl], "fp32", steps=warmup + steps, device=dev, use_cache=False)
    bed_kw = autotune.bed_kwargs(wl, tuned)
    m = measure_coupled(wl, U, P, bed_kw, dev, steps, warmup)
    wall, contacts = m["wall"], m["contacts"]
    return {"workload": "spouted bed: 500,000 spheres, d lognormal (median 2 mm, sigma 0.2, clipped 1-4 mm), "
                        "0.15 x 0.15 x 0.6 m, Q2 30x30x120 mesh (2,916,000 qpts), Gaussian inlet jet 20 m/s, "
                        f"coupling every {COUPLING_EVERY} steps",
            "particles": wl.n, "steps": steps, "warmup": warmup,
            "value": wl.n * steps / wall, "unit": "particle-steps/s", "ms_per_step": wall * 1e3 / steps,
            "contacts_per_s": contacts * steps / wall,
            "quadrature_points_per_s": m["nq_total"] * couplings_in(warmup, steps) / wall,
            "contacts_pairs_walls": m["pairs_walls"],
            "tuned": dict(bed_kw, trials=tune_report["trials"],
                          default_ms_per_step=tune_report["default_ms_per_step"]),
            "force_kernel": m["force_kernel"], "whole_step": m["whole_step"],
            "generation_s": gen_s, "errors": m["errors"], "dtype": "f32 forces / f64 state"}, wl, bed_kw


def batched_ensemble(n_beds, steps, dev):
    """The batched ensemble: every bed advanced by shared launches from one
    graph per chunk (coupling + 10 steps), FP32 forces; then the plain
    per-bed FP64 path on the same beds (single-bed entry points, one bed after
    another) over a tenth of the steps."""
    import torch

    from paper_2211_01185_amd import autotune, cfddem, synth

    wls = synth.batched(n_beds)
    n_total = sum(w.n for w in wls)
    fields = [(torch.as_tensor(w.U, dtype=torch.float64, device=dev).contiguous(),
               torch.as_tensor(w.P, dtype=torch.float64, device=dev).contiguous()) for w in wls]
    # tuned over as many steps as the measurement runs, from the same start
    cfg, tune_report = autotune.tune(wls, "fp32", steps=steps, device=dev, use_cache=False)
    beds = [cfddem.bed_from_workload(w, precision="fp32", device=dev, **autotune.bed_kwargs(w, cfg))
            for w in wls]
    batch = cfddem.Batch(beds, fields)
    chunks = steps // COUPLING_EVERY
    batch.run(2, COUPLING_EVERY, couple=True)  # warm-up, graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.run(chunks, COUPLING_EVERY, couple=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    errors = sum(1 for b in beds if b.poll()[0])
    contacts = sum(b.poll()[1] for b in beds)
    batch.close()
    for b in beds:
        b.close()
    del batch, beds
    # plain per-bed FP64 path
    plain_steps = max(COUPLING_EVERY, steps // 10)
    t_plain = 0.0
    for w, (U, P) in zip(wls, fields):
        bed = cfddem.bed_from_workload(w, precision="fp64", device=dev, resort_every=RESORT_EVERY)
        out = bed.couple(U, P)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(plain_steps // COUPLING_EVERY):
            bed.couple(U, P, out=out)
            bed.step(COUPLING_EVERY)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t1
        errors += 1 if bed.poll()[0] else 0
        bed.close()
    return {
        "workload": f"{n_beds} independent column beds, {n_total} spheres in total (5k-80k per bed, "
                    f"d 1-3 mm, e 0.7-0.95, inlet 0.5-2 m/s, Q1 meshes), coupling every {COUPLING_EVERY} steps",
        "beds": n_beds, "particles": n_total, "steps": chunks * COUPLING_EVERY,
        "value": n_total * chunks * COUPLING_EVERY / dt, "unit": "particle-steps/s",
        "jobs_per_s": n_beds / (dt * steps / (chunks * COUPLING_EVERY)),
        "ms_per_step": dt * 1e3 / (chunks * COUPLING_EVERY),
        "dtype": "f32 forces / f64 state", "launch": "shared launches per step, one HIP graph per chunk",
        "contacts_end": int(contacts), "errors": int(errors), "autotune": tune_report,
        # what a kernel trace of this leg needs to find the ensemble's launches
        # and to price them: their grid sizes (threads) and the algorithmic
        # bytes of one DEM step of the ensemble
        "grid_threads": {"force_kick_batch": sum(-(-w.n * cfg["lanes"] // FORCE_BLOCK) for w in wls) * FORCE_BLOCK,
                         "drift_bin_batch": sum(-(-w.n // 256) for w in wls) * 256},
        "algorithmic_bytes_per_step": FORCE_BYTES_PER_PARTICLE * n_total + BYTES_PER_CONTACT * int(contacts),
        "per_bed_fp64_path": {"value": n_total * plain_steps / t_plain, "unit": "particle-steps/s",
                              "steps": plain_steps, "dtype": "f64",
                              "launch": "single-bed entry points, one bed after another"},
    }


def smoothing_run(dev, steps=200):
    """The benchmark bed with the smoothed void fraction (L^2 = 5 d^2, the
    spouted-bed setting of the paper): coupled steps as in the main
    measurement, and the first coupling step timed on its own."""
    import torch

    from paper_2211_01185_amd import cfddem, synth

    wl = synth.fluidized()
    d = 2.0 * float(wl.radius[0])
    wl.fluid["smooth_L2"] = 5.0 * d * d
    U = torch.as_tensor(wl.U, dtype=torch.float64, device=dev).contiguous()
    P = torch.as_tensor(wl.P, dtype=torch.float64, device=dev).contiguous()
    bed = cfddem.bed_from_workload(wl, precision="fp32", device=dev, resort_every=RESORT_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = bed.couple(U, P)
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3
    bed.step(COUPLING_EVERY)
    for _ in range(2):  # warm-up chunks
        bed.couple(U, P, out=out)
        bed.step(COUPLING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // COUPLING_EVERY):
        bed.couple(U, P, out=out)
        bed.step(COUPLING_EVERY)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    err, _ = bed.poll()
    bed.close()
    n_steps = COUPLING_EVERY * (steps // COUPLING_EVERY)
    return {"workload": "fluidized-bed slice as the main measurement, smoothed void fraction L^2 = 5 d^2 "
                        "(Q2 field on 270,641 velocity nodes, solved directly at every coupling step)",
            "L2": wl.fluid["smooth_L2"], "steps": n_steps, "value": wl.n * n_steps / wall,
            "unit": "particle-steps/s", "ms_per_step": wall * 1e3 / n_steps,
            "first_coupling_ms": first_ms, "errors": int(err), "dtype": "f32 forces / f64 state and field"}


def settling_run(dev, max_steps=100_000):
    """The filling workload stepped to rest (no coupling), FP32 forces."""
    import torch

    from paper_2211_01185_amd import cfddem, settle, synth

    wl = synth.filling()
    bed = cfddem.bed_from_workload(wl, precision="fp32", device=dev, resort_every=200)
    torch.cuda.synchronize()
    res = settle.settle(bed, settle.energy_scale(wl), rest=1e-4, every=500, max_steps=max_steps)
    err, contacts = bed.poll()
    bed.close()
    return {"workload": "DEM-only filling: 100,000 spheres d=1 mm inserted at random (solid fraction 0.15) "
                        "above the floor of the 0.1 x 0.1 x 0.4 m column, stepped without coupling to rest",
            "particles": wl.n, "steps_to_rest": res.steps, "at_rest": res.at_rest,
            "simulated_s": res.steps * wl.dem["dt"], "wall_s": res.wall_s,
            "value": wl.n * res.steps / res.wall_s, "unit": "particle-steps/s",
            "kinetic_energy_over_mgd": res.kinetic / settle.energy_scale(wl),
            "contacts_at_rest": int(contacts), "errors": int(err),
            "dtype": "f32 forces / f64 state", "check_every_steps": 500}


def packed_run(dev, steps=1000, warmup=20):
    """The fluidized-bed measurement on a physically packed bed: the 100,000
    spheres of the filling workload settled to rest (as the settling run),
    then the fluidized bed's fluid (Q2 20x20x80, U = (0,0,1.2) + N(0, 0.05),
    linear pressure) from that state, FP32 forces; tuned on this bed, then
    coupled steps timed as the main measurement, and the contact-force
    kernel's launches timed on a replay of the same steps."""
    import torch

    from paper_2211_01185_amd import autotune, cfddem, settle, synth

    fw = synth.filling()
    bed = cfddem.bed_from_workload(fw, precision="fp32", device=dev, resort_every=200)
    res = settle.settle(bed, settle.energy_scale(fw), rest=1e-4, every=500, max_steps=100_000)
    st = {k: t.cpu().numpy() for k, t in bed.read_state().items()}
    bed.close()
    base = synth.fluidized()
    wl = synth.Workload("packed", st["x"], st["v"], st["w"], fw.radius, fw.density, base.dem, base.fluid,
                        base.run, base.U, base.P)
    U = torch.as_tensor(wl.U, dtype=torch.float64, device=dev).contiguous()
    P = torch.as_tensor(wl.P, dtype=torch.float64, device=dev).contiguous()
    tuned, tune_report = autotune.tune([wl], "fp32", steps=warmup + steps, device=dev, use_cache=False)
    bed_kw = autotune.bed_kwargs(wl, tuned)
    m = measure_coupled(wl, U, P, bed_kw, dev, steps, warmup)
    wall, contacts = m["wall"], m["contacts"]
    return {"workload": "packed fluidized bed: the 100,000-sphere filling (d = 1 mm) settled to rest in the "
                        "0.1 x 0.1 x 0.4 m column, then the fluidized bed's fluid (Q2 20x20x80, 1.2 m/s "
                        f"upflow) from that state, coupling every {COUPLING_EVERY} steps",
            "particles": wl.n, "steps": steps, "warmup": warmup, "settle_steps": res.steps,
            "value": wl.n * steps / wall, "unit": "particle-steps/s", "ms_per_step": wall * 1e3 / steps,
            "contacts_per_s": contacts * steps / wall,
            "quadrature_points_per_s": m["nq_total"] * couplings_in(warmup, steps) / wall,
            "contacts_pairs_walls": m["pairs_walls"],
            "tuned": dict(bed_kw, trials=tune_report["trials"],
                          default_ms_per_step=tune_report["default_ms_per_step"]),
            "force_kernel": m["force_kernel"], "whole_step": m["whole_step"],
            "errors": m["errors"], "dtype": "f32 forces / f64 state"}


def served_stream(n_jobs, warmup, dev, config=None):
    """The served stream: Poisson arrivals, continuous batching; statistics
    over the jobs after the first `warmup` ones.  config: the launch
    choices of every job's bed (the batched ensemble's tuned configuration:
    the jobs are beds of the same recipe), or None for the defaults."""
    from paper_2211_01185_amd import serve, synth

    jobs = synth.job_stream(n_jobs)
    server = serve.Server(device=dev, config=config)
    results, wall = server.run(jobs)
    measured = [r for r in results if r.index >= warmup]
    t_first = min(r.arrival for r in measured)
    t_last = max(r.finished for r in measured)
    s = serve.summarize(measured, t_last - t_first)
    offered = sum(j.n * j.steps for j in jobs) / jobs[-1].arrival
    return {
        "workload": f"{n_jobs} jobs ({warmup} warm-up), Poisson arrivals 20 jobs/s, sedimentation or "
                    "fluidization column beds of 1k-200k spheres, 200-2000 steps, coupling every 10",
        "jobs": s["jobs"], "latency_p50_s": s["latency_p50_s"], "latency_p99_s": s["latency_p99_s"],
        "value": s["particle_steps_per_s"], "unit": "particle-steps/s", "jobs_per_s": s["jobs_per_s"],
        "offered_particle_steps_per_s": offered, "errors": s["errors"], "chunks": server.chunks,
        "batches_created": server.batches, "slot_changes": server.layout_changes, "wall_s": wall, "dtype": "f32 forces / f64 state",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (across GPUs, "
              "independent beds would be placed whole, and one large bed split into z-slabs that "
              "exchange ghost particles every step)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2211_01185_amd import autotune, cfddem, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    wl = synth.fluidized()
    U = torch.as_tensor(wl.U, dtype=torch.float64, device=dev).contiguous()
    P = torch.as_tensor(wl.P, dtype=torch.float64, device=dev).contiguous()
    # skin (DEM cell size), re-sort interval and lanes per particle: tuned on
    # runs of this bed over the roofline window (from its start, the warm-up
    # and the measured steps: the rate of list rebuilds grows as the bed
    # fluidizes), whatever the timed region's length; results do not depend
    # on them
    if args.bed_config:
        given = json.loads(args.bed_config)
        bed_kw = {k: given[k] for k in ("skin", "resort_every", "lanes")}
        bed_kw["elem_threads"] = int(given.get("elem_threads", 128))
        tune_report = {"trials": 0, "default_ms_per_step": None}
    else:
        tuned, tune_report = autotune.tune([wl], "fp32", steps=WINDOW_WARMUP + WINDOW_STEPS, device=dev,
                                           use_cache=False)
        bed_kw = autotune.bed_kwargs(wl, tuned)
    progress(f"tuned {bed_kw} in {tune_report['trials']} trials")

    def make_bed():
        return make_coupled_bed(wl, U, P, bed_kw, dev)

    def run(bed, out, steps, start):
        return run_coupled(bed, out, U, P, steps, start)

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
    progress(f"timed region: {wall * 1e3 / args.steps:.4f} ms per step")

    # roofline: the fixed window (WINDOW_WARMUP + WINDOW_STEPS steps of a
    # fresh bed) run once without instrumentation for the whole step's time,
    # then replayed on another fresh bed with HIP events bound to every launch
    # of the contact-force kernel on its stream (the events add launch
    # latency, so the timed region runs without them)
    win = measure_coupled(wl, U, P, bed_kw, dev, WINDOW_STEPS, WINDOW_WARMUP)
    fk = win["force_kernel"]
    progress(f"roofline window: {fk['launches']} force-kernel launches, {fk['avg_launch_us']:.2f} us each; "
             f"{win['whole_step']['us_per_step']:.2f} us per step")
    if win["errors"]:
        raise SystemExit("device error in the roofline window")

    elapsed = max(wall, gpu_ms / 1e3)
    value = wl.n * args.steps / elapsed
    contacts = 0.5 * (pairs0 + walls0 + pairs1 + walls1)
    traffic, traffic_cfg = traffic_entry(bed_kw["lanes"], "fp32")
    qpts = wl.fluid["n_el"][0] * wl.fluid["n_el"][1] * wl.fluid["n_el"][2] * (wl.fluid["order"] + 1) ** 3

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
            "tuned": dict(bed_kw, trials=tune_report["trials"],
                          default_ms_per_step=tune_report["default_ms_per_step"],
                          tuned_over_steps=WINDOW_WARMUP + WINDOW_STEPS),
            "parallelism": "1 GPU",
        },
        "rates": {
            "particle_steps_per_s": value,
            "contacts_per_s": contacts * args.steps / elapsed,
            "quadrature_points_per_s": qpts * couplings_in(args.warmup, args.steps) / elapsed,
            "contacts": contacts, "quadrature_points": qpts,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"force_kick<float, true, *, {bed_kw['lanes']}> (contact search + Hertz-Mindlin "
                      "forces + second half kick)",
            "achieved": fk["achieved_GBs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": fk["frac_of_hbm_peak"],
            "traffic": traffic,
            "traffic_taken_with": traffic_cfg,
            "avg_launch_us": fk["avg_launch_us"],
            "launches": fk["launches"],
            "algorithmic_bytes_per_launch": fk["algorithmic_bytes_per_launch"],
            "window": {"warmup": WINDOW_WARMUP, "steps": WINDOW_STEPS,
                       "what": "a fresh bed, WINDOW_WARMUP steps, then WINDOW_STEPS measured steps with their "
                               "re-sorts, broad searches and coupling steps; the same for every --steps",
                       "contacts_pairs_walls": win["pairs_walls"], "ms_per_step": win["wall"] * 1e3 / WINDOW_STEPS,
                       "particle_steps_per_s": wl.n * WINDOW_STEPS / win["wall"]},
            "whole_step": win["whole_step"],
        },
    }
    if not args.no_fp64:
        progress("FP64 100k bed: starting")
        m = measure_coupled(wl, U, P, bed_kw, dev, WINDOW_STEPS, WINDOW_WARMUP, precision="fp64")
        result["fp64"] = {"workload": "the same fluidized bed, all FP64 (pair forces and drag too), the roofline "
                                      "window's steps with the FP32 bed's launch choices",
                          "particles": wl.n, "steps": WINDOW_STEPS, "warmup": WINDOW_WARMUP,
                          "value": wl.n * WINDOW_STEPS / m["wall"], "unit": "particle-steps/s",
                          "ms_per_step": m["wall"] * 1e3 / WINDOW_STEPS, "contacts_pairs_walls": m["pairs_walls"],
                          "force_kernel": m["force_kernel"], "whole_step": m["whole_step"],
                          "errors": m["errors"], "dtype": "f64"}
        progress(f"FP64: {result['fp64']['ms_per_step']:.4f} ms per step")
    if not args.no_config1:
        progress("plain FP64 configuration: starting")
        result["plain_fp64_2k"] = config1_run(dev)
        progress(f"plain FP64: {result['plain_fp64_2k']['ms_per_step']:.4f} ms per step")
    if not args.no_batched:
        result["batched"] = batched_ensemble(args.batched_beds, args.batched_steps, dev)
        progress(f"batched: {result['batched']['value']:.4g} particle-steps/s")
    if not args.no_served:
        progress("served stream: starting")
        cfg = result["batched"]["autotune"]["config"] if "batched" in result else None
        result["served"] = served_stream(args.served_jobs, args.served_warmup, dev, cfg)
        result["served"]["config"] = cfg
        progress(f"served: p99 {result['served']['latency_p99_s']:.4f} s")
    if not args.no_smoothing:
        progress("smoothing: starting")
        result["smoothing"] = smoothing_run(dev)
        progress(f"smoothing: {result['smoothing']['ms_per_step']:.4f} ms per step")
    if not args.no_settling:
        progress("settling: starting")
        result["settling"] = settling_run(dev)
        progress(f"settling: {result['settling']['steps_to_rest']} steps to rest")
    if not args.no_packed:
        progress("packed bed: starting")
        result["packed"] = packed_run(dev)
        progress(f"packed: {result['packed']['ms_per_step']:.4f} ms per step")
    if not args.no_spouted:
        progress("spouted bed: starting")
        result["spouted"], sp_wl, sp_kw = spouted_run(dev)
        progress(f"spouted: {result['spouted']['ms_per_step']:.4f} ms per step")
    if not args.no_cpu:
        progress("oracle sample: starting")
        result["cpu_baseline"], ref = cpu_baseline(wl, args.cpu_steps)
        progress("GPU paths against the oracle sample")
        result["error_vs_fp64_oracle"] = errors_vs_oracle(wl, U, P, bed_kw, dev, ref, args.cpu_steps)
        # the other results' paths on the first coupling and DEM step: the
        # spouted bed (tuned as measured), the first bed of the batched
        # ensemble run as a batch of one with the ensemble's tuned choices
        if not args.no_spouted:
            progress("spouted bed against the oracle")
            result["error_vs_fp64_oracle"]["spouted_fp32"] = gpu_first_step_errors(
                sp_wl, oracle_first_step(sp_wl), dev, sp_kw)
        if not args.no_config1:
            progress("plain FP64 configuration against the oracle")
            result["error_vs_fp64_oracle"]["plain_fp64_2k"] = config1_errors(dev)
        if not args.no_batched:
            from paper_2211_01185_amd import autotune, synth

            bw = synth.batched_bed(0)
            bkw = autotune.bed_kwargs(bw, result["batched"]["autotune"]["config"])
            result["error_vs_fp64_oracle"]["batched_bed0_fp32"] = gpu_first_step_errors(
                bw, oracle_first_step(bw), dev, bkw, batch=True)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

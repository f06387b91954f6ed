"""Continuous-batching server of simulation jobs on one GPU.

Jobs (independent beds, each with its own particle count, materials, mesh
and fluid field, a number of DEM steps and a coupling step every 10 steps)
arrive over time.  The server keeps every admitted job's state on the device
in one slot batch (dem_batch_create_slots) and advances all of them
together: each chunk is one coupling step plus ten DEM steps for every job
held, replayed from captured HIP graphs (dem_batch_run).  Around the chunks:

  * a job that has arrived is admitted into a free slot (dem_batch_admit),
    oldest first, while its device footprint fits the memory budget (a job
    that does not fit waits; later jobs do not overtake it); its bed is
    created on a side stream, so that creating it does not wait for the
    chunks in flight;
  * a job that has run all its steps leaves its slot (dem_batch_retire) as
    soon as its last chunk is enqueued; its final state is copied to pinned
    host memory on the stream, and the job is finished (its latency is the
    time from its arrival to that point) when that copy has completed;
  * at most `depth` chunks are in flight; the host waits on the oldest
    chunk's event, not on the whole stream, and generates the beds of jobs
    about to arrive on a worker thread meanwhile.

A job's arithmetic does not depend on the other jobs in the batch, so its
result is the same alone and in the mix.
"""
from __future__ import annotations

import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import autotune, cfddem

CHUNK_STEPS = 10  # DEM steps per coupling step


@dataclass
class JobResult:
    index: int
    n: int
    steps: int
    arrival: float
    admitted: float
    finished: float
    x: np.ndarray = field(repr=False)
    v: np.ndarray = field(repr=False)
    w: np.ndarray = field(repr=False)
    error: int = 0

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class _Active:
    def __init__(self, job, bed, U, P, slot, admitted):
        self.job = job
        self.bed = bed
        self.U = U
        self.P = P
        self.slot = slot
        self.left = job.steps
        self.admitted = admitted


class _Finishing:
    """A retired job whose final state is being copied to the host."""

    def __init__(self, a, host, event):
        self.a = a
        self.host = host
        self.event = event


def footprint(wl, precision="fp32", resort_every=100, **bed_kw) -> int:
    """Device bytes a job holds while active: its workspace, fluid field and
    coupling outputs (batch tables are small and not counted).  bed_kw: the
    launch choices of its bed (skin, lanes, elem_threads)."""
    d = 2.0 * float(wl.radius.max())
    dp, cp = cfddem.make_params(wl.dem, wl.fluid, wl.n, d, 2.0 * float(wl.radius.min()), precision,
                                resort_every=resort_every, **bed_kw)
    ws = cfddem.workspace_bytes(dp, cp)
    n_el = int(np.prod(wl.fluid["n_el"]))
    nq = (int(wl.fluid["order"]) + 1) ** 3
    return ws + 8 * (wl.U.size + wl.P.size) + 8 * 5 * n_el * nq


class Server:
    """Runs a job stream in real time (arrival times in seconds from start)."""

    def __init__(self, budget_bytes=64 << 30, precision="fp32", resort_every=100, device="cuda",
                 clock=time.perf_counter, speed=1.0, config=None, slots=256, depth=2, prefetch=4):
        import torch

        self.torch = torch
        self.budget = int(budget_bytes)
        self.precision = precision
        self.resort_every = resort_every
        # an autotuner configuration (skin factor, re-sort interval, lanes,
        # threads per element) for every job's bed, or None for the defaults
        # with resort_every; one configuration for all jobs, since the beds
        # of a batch must share their lanes and threads per element
        self.config = config
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.side = torch.cuda.Stream(self.device)  # bed creation
        self.clock = clock
        self.speed = float(speed)  # arrival times are divided by speed
        self.slots = int(slots)
        self.depth = max(1, int(depth))
        self.prefetch = int(prefetch)
        self.active: list[_Active] = []
        self.used = 0
        self.chunks = 0
        self.batches = 0         # slot batches created (one per run)
        self.layout_changes = 0  # admissions and retirements between chunks

    def _bed_kw(self, wl) -> dict:
        if self.config is None:
            return dict(resort_every=self.resort_every)
        return autotune.bed_kwargs(wl, self.config)

    def _prepare(self, job):
        """Host work of a job before it can be admitted (worker thread): its
        bed's arrays and its device footprint."""
        wl = job.workload()
        return wl, footprint(wl, self.precision, **self._bed_kw(wl))

    def _admit(self, sb, job, wl, now):
        torch = self.torch
        with torch.cuda.stream(self.side):
            bed = cfddem.bed_from_workload(wl, precision=self.precision, device=self.device, stream=self.side,
                                           **self._bed_kw(wl))
            U = torch.as_tensor(wl.U, dtype=torch.float64, device=self.device).contiguous()
            P = torch.as_tensor(wl.P, dtype=torch.float64, device=self.device).contiguous()
            self.side.synchronize()  # created (only the side stream's own work)
        # from now on the bed lives on the batch's stream
        for t in (bed.workspace, U, P):
            t.record_stream(self.stream)
        bed.stream = self.stream
        slot = self._free_slots.pop()
        sb.admit(slot, bed, (U, P))
        self.active.append(_Active(job, bed, U, P, slot, now))
        self.layout_changes += 1

    def _retire(self, sb, a) -> _Finishing:
        """Leaves the slot now; the final state is read behind the chunks
        already enqueued."""
        torch = self.torch
        sb.retire(a.slot)
        self._free_slots.append(a.slot)
        self.layout_changes += 1
        st = a.bed.read_state()
        host = {}
        for k in ("x", "v", "w"):
            h = torch.empty(st[k].shape, dtype=st[k].dtype, pin_memory=True)
            h.copy_(st[k], non_blocking=True)
            host[k] = h
        ev = torch.cuda.Event()
        ev.record(self.stream)
        return _Finishing(a, host, ev)

    def _finish(self, f, now, sizes) -> JobResult:
        a = f.a
        # the batch's stream is past this job's last work: its error flag is
        # read on the side stream, without waiting for the chunks after it
        a.bed.stream = self.side
        err, _ = a.bed.poll()
        x, v, w = (f.host[k].numpy().copy() for k in ("x", "v", "w"))
        res = JobResult(a.job.index, a.job.n, a.job.steps, a.job.arrival, a.admitted, now, x, v, w, err)
        a.bed.close()
        self.used -= sizes.pop(a.job.index)
        return res

    def run(self, jobs):
        """Serve `jobs` (objects with index, arrival, steps and workload()).
        Returns (results, wall seconds)."""
        torch = self.torch
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        sizes = {}
        prepared = {}   # job index -> future of (workload, footprint)
        results = []
        finishing: list[_Finishing] = []
        inflight = deque()  # events of enqueued chunks
        self._free_slots = list(range(self.slots - 1, -1, -1))
        held_n = 0
        # limits of what the batch may hold at once: the memory budget bounds
        # both (a bed's workspace takes more than 500 bytes per particle and
        # its coupling outputs more than 300 per element)
        sb = cfddem.SlotBatch(self.slots, max_particles=max(1, self.budget // 500),
                              max_elements=max(1, self.budget // 300), couples=True, device=self.device,
                              stream=self.stream)
        self.batches += 1
        pool = ThreadPoolExecutor(max_workers=2)
        t0 = self.clock()

        def now():
            return (self.clock() - t0) * self.speed

        def prefetch():
            for j in list(pending)[:self.prefetch]:
                if j.index not in prepared:
                    prepared[j.index] = pool.submit(self._prepare, j)

        def finish_ready(block=False):
            for f in list(finishing):
                if block:
                    f.event.synchronize()
                if f.event.query():
                    finishing.remove(f)
                    results.append(self._finish(f, now(), sizes))

        try:
            while pending or self.active or finishing:
                prefetch()
                # admissions: arrived jobs, oldest first, while the budget allows
                while pending and pending[0].arrival <= now() and self._free_slots:
                    j = pending[0]
                    wl, size = prepared.setdefault(j.index, pool.submit(self._prepare, j)).result()
                    # over the budget only when nothing else holds device memory
                    # (a retired job holds its memory until its result is read)
                    if (self.active or finishing) and (self.used + size > self.budget
                                                       or held_n + j.n > sb.limits.max_particles):
                        break
                    pending.popleft()
                    prepared.pop(j.index)
                    sizes[j.index] = size
                    self.used += size
                    held_n += j.n
                    self._admit(sb, j, wl, now())
                finish_ready()
                if not self.active:
                    if finishing:
                        finish_ready(block=True)  # releases memory a waiting job may need
                        continue
                    if not pending:
                        # the last result was read by finish_ready() above,
                        # after the loop's test: nothing is left
                        continue
                    # idle until the next arrival
                    wait = (pending[0].arrival - now()) / self.speed
                    if wait > 0:
                        time.sleep(wait)
                    continue
                # at most `depth` chunks in flight: wait for the oldest
                while len(inflight) >= self.depth:
                    ev = inflight.popleft()
                    while not ev.query():
                        finish_ready()
                        time.sleep(0)
                sb.run(1, CHUNK_STEPS, couple=True)
                ev = torch.cuda.Event()
                ev.record(self.stream)
                inflight.append(ev)
                self.chunks += 1
                for a in self.active:
                    a.left -= CHUNK_STEPS
                done = [a for a in self.active if a.left <= 0]
                if done:
                    self.active = [a for a in self.active if a.left > 0]
                    for a in done:
                        finishing.append(self._retire(sb, a))
                        held_n -= a.job.n
            finish_ready(block=True)
        finally:
            pool.shutdown(wait=True)
            self.stream.synchronize()
            sb.close()
        return results, (self.clock() - t0)


def summarize(results, wall):
    lat = np.array([r.latency for r in results])
    ps = sum(r.n * r.steps for r in results)
    return dict(jobs=len(results), wall_s=wall, particle_steps=ps,
                particle_steps_per_s=ps / wall if wall > 0 else None,
                jobs_per_s=len(results) / wall if wall > 0 else None,
                latency_p50_s=float(np.percentile(lat, 50)) if lat.size else None,
                latency_p99_s=float(np.percentile(lat, 99)) if lat.size else None,
                errors=int(sum(1 for r in results if r.error)))

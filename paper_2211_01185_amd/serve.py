"""Continuous-batching server of simulation jobs on one GPU.

Jobs (independent beds, each with its own particle count, materials, mesh
and fluid field, a number of DEM steps and a coupling step every 10 steps)
arrive over time.  The server keeps every admitted job's state on the device
and advances all of them together: each chunk is one coupling step plus ten
DEM steps for every active job, replayed from one captured HIP graph
(dem_batch_run).  Between chunks it

  * retires jobs that have run all their steps (final state copied to the
    host; the latency of a job is the time from its arrival to that point),
  * admits jobs that have arrived, oldest first, while their device
    footprint fits the memory budget (a job that does not fit waits; later
    jobs do not overtake it),
  * rebuilds the batch tables when the set of jobs changed.

A job's arithmetic does not depend on the other jobs in the batch, so its
result is the same alone and in the mix.
"""
from __future__ import annotations

import time
from collections import deque
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
    def __init__(self, job, wl, bed, U, P, admitted):
        self.job = job
        self.wl = wl
        self.bed = bed
        self.U = U
        self.P = P
        self.left = job.steps
        self.admitted = admitted


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
                 clock=time.perf_counter, speed=1.0, config=None):
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
        self.clock = clock
        self.speed = float(speed)  # arrival times are divided by speed
        self.active: list[_Active] = []
        self.used = 0
        self.batch = None
        self.dirty = False
        self.chunks = 0
        self.rebuilds = 0

    def _bed_kw(self, wl) -> dict:
        if self.config is None:
            return dict(resort_every=self.resort_every)
        return autotune.bed_kwargs(wl, self.config)

    def _admit(self, job, wl, now):
        torch = self.torch
        bed = cfddem.bed_from_workload(wl, precision=self.precision, device=self.device, stream=self.stream,
                                       **self._bed_kw(wl))
        U = torch.as_tensor(wl.U, dtype=torch.float64, device=self.device).contiguous()
        P = torch.as_tensor(wl.P, dtype=torch.float64, device=self.device).contiguous()
        self.active.append(_Active(job, wl, bed, U, P, now))
        self.dirty = True

    def _retire(self, a, now_fn) -> JobResult:
        err, _ = a.bed.poll()  # synchronizes the stream
        st = a.bed.read_state()
        x, v, w = (st[k].cpu().numpy() for k in ("x", "v", "w"))
        res = JobResult(a.job.index, a.job.n, a.job.steps, a.job.arrival, a.admitted, now_fn(), x, v, w, err)
        a.bed.close()
        self.dirty = True
        return res

    def _rebuild(self):
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        if self.active:
            self.batch = cfddem.Batch([a.bed for a in self.active], [(a.U, a.P) for a in self.active],
                                      stream=self.stream)
        self.dirty = False
        self.rebuilds += 1

    def run(self, jobs):
        """Serve `jobs` (objects with index, arrival, steps and workload()).
        Returns (results, wall seconds)."""
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        sizes = {}
        wls = {}
        results = []
        t0 = self.clock()

        def now():
            return (self.clock() - t0) * self.speed

        while pending or self.active:
            # admissions: arrived jobs, oldest first, while the budget allows
            while pending and pending[0].arrival <= now():
                j = pending[0]
                if j.index not in sizes:
                    wls[j.index] = j.workload()
                    sizes[j.index] = footprint(wls[j.index], self.precision, **self._bed_kw(wls[j.index]))
                if self.active and self.used + sizes[j.index] > self.budget:
                    break
                pending.popleft()
                self.used += sizes[j.index]
                self._admit(j, wls.pop(j.index), now())
            if not self.active:
                # idle until the next arrival
                wait = (pending[0].arrival - now()) / self.speed
                if wait > 0:
                    time.sleep(wait)
                continue
            if self.dirty:
                self._rebuild()
            self.batch.run(1, CHUNK_STEPS, couple=True)
            self.chunks += 1
            for a in self.active:
                a.left -= CHUNK_STEPS
            done = [a for a in self.active if a.left <= 0]
            if done:
                self.active = [a for a in self.active if a.left > 0]
                if self.batch is not None:
                    self.batch.close()  # the retiring beds leave the batch first
                    self.batch = None
                for a in done:
                    results.append(self._retire(a, now))
                    self.used -= sizes[a.job.index]
            else:
                self.stream.synchronize()
        if self.batch is not None:
            self.batch.close()
            self.batch = None
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

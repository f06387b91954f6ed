"""Continuous-batching server: every job's result in the mix equals its
result when it is served alone (bit for bit, since a bed's arithmetic does
not depend on the other beds of a batch), jobs that arrive while others run
are admitted between chunks, and a memory budget holds later jobs back."""
import numpy as np
import pytest

from paper_2211_01185_amd import serve, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _small_stream(n_jobs=8):
    # the served stream's job recipe with small beds and an arrival rate high
    # enough that several jobs overlap on the device
    return synth.job_stream(n_jobs, rate=400.0, n_min=1_000, n_max=6_000)


def test_results_alone_equal_results_in_the_mix():
    jobs = _small_stream()
    server = serve.Server()
    mixed, _ = server.run(jobs)
    assert len(mixed) == len(jobs)
    assert server.rebuilds > 1  # the set of active jobs changed while others ran
    assert max(len(set(r.index for r in mixed if r.admitted <= m.finished and r.finished >= m.admitted))
               for m in mixed) > 1  # some jobs were on the device together
    by_index = {r.index: r for r in mixed}
    for job in jobs:
        (alone,), _ = serve.Server().run([job])
        r = by_index[job.index]
        assert r.error == 0 and alone.error == 0
        for k in ("x", "v", "w"):
            assert np.array_equal(getattr(r, k), getattr(alone, k)), (job.index, k)


def test_budget_holds_jobs_back():
    jobs = _small_stream(4)
    wl_sizes = [serve.footprint(j.workload()) for j in jobs]
    # room for the largest job only: jobs run one at a time, in arrival order
    server = serve.Server(budget_bytes=max(wl_sizes))
    results, _ = server.run(jobs)
    assert [r.index for r in results] == [j.index for j in jobs]
    for a, b in zip(results, results[1:]):
        assert b.admitted >= a.finished - 1e-9

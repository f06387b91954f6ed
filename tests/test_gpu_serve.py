"""Continuous-batching server: every job's result in the mix equals its
result when it is served alone (bit for bit, since a bed's arithmetic does
not depend on the other beds of a batch), jobs that arrive while others run
are admitted between chunks, in arrival order, and the jobs on the device
never exceed the memory budget."""
import numpy as np
import pytest

from paper_2211_01185_amd import serve, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _small_stream(n_jobs=8):
    # the served stream's job recipe with small beds and an arrival rate high
    # enough that several jobs overlap on the device
    return synth.job_stream(n_jobs, rate=400.0, n_min=1_000, n_max=6_000)


@pytest.mark.parametrize("config", [None, {"skin_factor": 0.05, "resort_every": 200, "lanes": 2,
                                             "elem_threads": 16}])
def test_results_alone_equal_results_in_the_mix(config):
    jobs = _small_stream()
    server = serve.Server(config=config)
    mixed, _ = server.run(jobs)
    assert len(mixed) == len(jobs)
    assert server.batches == 1  # one slot batch for the whole stream
    assert server.layout_changes >= 2 * len(jobs)  # every job joined and left it
    assert max(len(set(r.index for r in mixed if r.admitted <= m.finished and r.finished >= m.admitted))
               for m in mixed) > 1  # some jobs were on the device together
    by_index = {r.index: r for r in mixed}
    for job in jobs:
        (alone,), _ = serve.Server(config=config).run([job])
        r = by_index[job.index]
        assert r.error == 0 and alone.error == 0
        for k in ("x", "v", "w"):
            assert np.array_equal(getattr(r, k), getattr(alone, k)), (job.index, k)


def test_budget_holds_jobs_back():
    jobs = _small_stream(6)
    sizes = {j.index: serve.footprint(j.workload()) for j in jobs}
    budget = max(sizes.values())  # the largest job fits alone
    server = serve.Server(budget_bytes=budget)
    results, _ = server.run(jobs)
    assert sorted(r.index for r in results) == [j.index for j in jobs]
    # admitted in arrival order (a job that does not fit is not overtaken)
    by_arrival = sorted(results, key=lambda r: r.arrival)
    assert all(a.admitted <= b.admitted for a, b in zip(by_arrival, by_arrival[1:]))
    # the jobs on the device together never exceed the budget
    for r in results:
        together = [q for q in results if q.admitted <= r.admitted < q.finished]
        assert sum(sizes[q.index] for q in together) <= budget

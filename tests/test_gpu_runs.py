"""Steps grouped into runs of any length give the bits of single steps.

Inside a run of steps, the cell grid of every step but the last lists only the
particles away from the cell they were sorted into at the last re-sort (the
others through their sorted index range), whereas a run of one step bins
every particle into the slots of its cell.  Equal bits pin the two listings to
the same neighbour lists: no pair missed, none listed twice.  The particles
are fast (about 1 m/s, 10 um a step), so that many leave their cell between
re-sorts, and the re-sorts fall on the same steps in both beds (every 30
steps: each group of runs below adds up to 30)."""
import numpy as np
import pytest

from paper_2211_01185_amd import synth
from tests.parity_util import compare_contacts, compare_states, gpu_bed, gpu_state, oracle_bed

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

RESORT = 30
RUNS = [1, 2, 3, 24, 30, 5, 25, 7, 1, 1, 21]  # 120 steps, re-sorts after each 30


def _workload(name):
    wl = synth.plain(seed_index=4) if name == "plain" else synth.lattice(n_side=(9, 9, 10), seed_index=7)
    wl.v = wl.v * 100.0
    return wl


def _bits(bed):
    st = gpu_state(bed)
    i, j, dt = bed.read_contacts()
    st["ci"], st["cj"], st["cdt"] = i, j, dt
    return st


@pytest.mark.parametrize("name", ["plain", "lattice"])
@pytest.mark.parametrize("lanes", [1, 2, 4])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_run_lengths_give_the_bits_of_single_steps(name, lanes, precision):
    wl = _workload(name)
    kw = dict(lanes=lanes, resort_every=RESORT, skin=1e-4)
    runs, single = gpu_bed(wl, precision, **kw), gpu_bed(wl, precision, **kw)
    homes, done = [], 0
    for n in RUNS:
        runs.step(n)
        done += n
        if done % RESORT == 0:  # the cells the next re-sort sorts by
            homes.append(runs.read_cells()[1].cpu().numpy())
    # a good share of the particles left their cell between re-sorts
    moved = [float(np.mean(h0 != h1)) for h0, h1 in zip(homes, homes[1:])]
    print("share of particles that changed cell between re-sorts", moved)
    assert min(moved) > 0.01
    for _ in range(sum(RUNS)):
        single.step(1)
    a, b = _bits(runs), _bits(single)
    assert len(a["ci"]) > 0
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    for bed in (runs, single):
        assert bed.poll()[0] == 0


def test_runs_against_the_oracle():
    """The same fast bed in runs of mixed lengths against the FP64 oracle."""
    wl = _workload("lattice")
    gb = gpu_bed(wl, "fp64", resort_every=RESORT, skin=1e-4)
    ob, _ = oracle_bed(wl)
    for n in RUNS[:4]:
        gb.step(n)
    ob.step(sum(RUNS[:4]))
    compare_contacts(gb, ob, 1e-8)
    compare_states(gb, ob, 1e-8)

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


def _snapshot(bed):
    st = gpu_state(bed)
    i, j, dt = bed.read_contacts()
    st["ci"], st["cj"], st["cdt"] = i, j, dt
    return st


@pytest.mark.parametrize("graph", [False, True])
def test_batch_chunk_lengths_give_the_bits_of_single_steps(graph):
    """The same for batches: chunks of 1, 2, 3 ... steps (direct launches or
    graph replay) against one-step chunks, three fast column beds re-sorted
    every 30 steps."""
    from paper_2211_01185_amd import cfddem

    wls = []
    for j, (n, d, e, u) in enumerate([(3000, 2.0e-3, 0.9, 1.0), (1700, 1.3e-3, 0.75, 0.0),
                                      (5200, 2.6e-3, 0.85, 1.6)]):
        w = synth.column_bed(synth.rng_for(4, 520 + j), n, d, e, u, name=f"r{j}", precision="fp32")
        w.v = w.v * 100.0
        wls.append(w)

    def make():
        beds = [gpu_bed(w, "fp32", resort_every=RESORT, skin=1e-4) for w in wls]
        fields = [(torch.as_tensor(w.U, dtype=torch.float64, device="cuda").contiguous(),
                   torch.as_tensor(w.P, dtype=torch.float64, device="cuda").contiguous()) for w in wls]
        return beds, cfddem.Batch(beds, fields)

    beds_a, a = make()
    beds_b, b = make()
    for n in RUNS:
        if graph:
            a.run(1, n, couple=False)
        else:
            a.step(n)
    for _ in range(sum(RUNS)):
        b.step(1)
    for x, y in zip(beds_a, beds_b):
        sa, sb = _snapshot(x), _snapshot(y)
        assert len(sa["ci"]) > 0
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), k
        assert x.poll()[0] == 0 and y.poll()[0] == 0
    a.close()
    b.close()


@pytest.mark.parametrize("resort_every", [0, 50])
def test_cell_capacity_overflow_is_reported_by_the_end_of_a_run(resort_every):
    """Cell capacity 1, two spheres in neighbouring cells of a 3 x 3 x 3 cell
    grid; the second crosses into the first one's cell at the second step
    without touching it.  Whether the run's inner grids list it as an arrival
    (with a re-sort at creation) or every grid lists every particle, the
    sticky capacity error is set by the end of the run."""
    from paper_2211_01185_amd import cfddem

    d, lo, hi = 3e-3, [0.0, 0.0, 0.0], [0.012, 0.012, 0.012]
    x = np.array([[1.6e-3, 4.05e-3], [1.6e-3, 3.9e-3], [1.6e-3, 3.9e-3]])
    v = np.array([[0.0, -5.0], [0.0, 0.0], [0.0, 0.0]])
    fluid = dict(order=1, n_el=[1, 1, 1], rho_f=1.2, mu_f=1.8e-5, model=0, eps_min=0.1)
    U = np.zeros((3, synth.node_grid(lo, hi, fluid["n_el"], 1).shape[1]))
    P = np.zeros(U.shape[1])
    dem = dict(box_lo=lo, box_hi=hi, gravity=[0.0, 0.0, 0.0], dt=1e-5, **synth._material())
    wl = synth.Workload("two", x, v, np.zeros((3, 2)), np.full(2, 0.5 * d), np.full(2, 2500.0), dem, fluid,
                        dict(steps=5, coupling_every=5, precision="fp64"), U, P)
    gb = gpu_bed(wl, "fp64", cell_capacity=1, resort_every=resort_every, skin=1e-4)
    assert gb.poll()[0] == 0
    assert gb.read_cells()[2] == [3, 3, 3]
    gb.step(5)
    assert gb.poll()[0] == cfddem.DEM_E_CAPACITY

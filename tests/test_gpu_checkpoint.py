"""Checkpoint and resume (dem_read_checkpoint / dem_write_state): a run of
n coupled steps, a checkpoint and m more steps gives bit for bit the state of
the same calls run on a context restored from the checkpoint, whatever that
context held before (another bed of the same shape, or the same context
rewound), with re-sorts and broad searches on both sides of the checkpoint;
the blob survives a trip through host memory; mismatched shapes are refused."""
import numpy as np
import pytest

from paper_2211_01185_amd import cfddem, synth
from tests.parity_util import gpu_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fields(wl):
    U = torch.as_tensor(wl.U, dtype=torch.float64, device="cuda").contiguous()
    P = torch.as_tensor(wl.P, dtype=torch.float64, device="cuda").contiguous()
    return U, P


def _snapshot(bed, out=None):
    st = gpu_state(bed)
    i, j, dt = bed.read_contacts()
    st["pairs_i"], st["pairs_j"], st["dt"] = i, j, dt
    elem, cell, _ = bed.read_cells()
    st["cell"] = cell.cpu().numpy()
    if out is not None:
        for k, v in out.items():
            st["out_" + k] = v.cpu().numpy()
    st["ke"] = np.array(bed.kinetic_energy())
    return st


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def _chunks(bed, U, P, n_chunks, steps=7):
    out = None
    for _ in range(n_chunks):
        out = bed.couple(U, P, elem_sums=True)
        bed.step(steps)
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("smooth", [False, True])
def test_resume_is_bit_identical(precision, smooth):
    wl = synth.lattice(n_side=(9, 8, 10), seed_index=4)
    if smooth:
        wl.fluid.update(smooth_L2=5.0 * (2 * float(wl.radius[0])) ** 2, model=1)
    U, P = _fields(wl)
    kw = dict(resort_every=5, skin=2e-5)
    a = cfddem.bed_from_workload(wl, precision=precision, **kw)
    _chunks(a, U, P, 3)
    blob = a.checkpoint()
    host = blob.cpu().numpy().copy()  # through host memory
    out_a = _chunks(a, U, P, 4)
    want = _snapshot(a, out_a)

    # another bed of the same shape (different positions and velocities)
    other = synth.lattice(n_side=(9, 8, 10), seed_index=5)
    if smooth:
        other.fluid.update(smooth_L2=wl.fluid["smooth_L2"], model=1)
    b = cfddem.bed_from_workload(other, precision=precision, **kw)
    b.step(3)  # its own step counter and grids
    b.restore(torch.from_numpy(host))
    out_b = _chunks(b, U, P, 4)
    _same(want, _snapshot(b, out_b))

    # the first context rewound to the checkpoint
    a.restore(blob)
    out_c = _chunks(a, U, P, 4)
    _same(want, _snapshot(a, out_c))
    assert a.poll()[0] == 0 and b.poll()[0] == 0


def test_restore_refuses_another_shape():
    wl = synth.lattice(n_side=(6, 6, 6), seed_index=1)
    a = cfddem.bed_from_workload(wl, precision="fp64")
    blob = a.checkpoint()
    other = synth.lattice(n_side=(6, 6, 7), seed_index=1)  # another particle count
    b = cfddem.bed_from_workload(other, precision="fp64")
    with pytest.raises(cfddem.CfddemError) as ei:
        b.restore(blob)
    assert ei.value.status == cfddem.DEM_E_ARG
    c = cfddem.bed_from_workload(wl, precision="fp32")  # another precision
    with pytest.raises(cfddem.CfddemError) as ei:
        c.restore(blob)
    assert ei.value.status == cfddem.DEM_E_ARG
    bad = blob.clone()
    bad[:8] = 0  # not a checkpoint
    with pytest.raises(cfddem.CfddemError) as ei:
        a.restore(bad)
    assert ei.value.status == cfddem.DEM_E_ABI

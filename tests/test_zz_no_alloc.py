"""The allocation-free kinetic-energy entry point (dem_kinetic_energy_noalloc,
per-block partial sums in the library's fixed device array) called through
the C ABI: its output equals dem_kinetic_energy's bit for bit, on two calls
in a row of which the second has a smaller bed (fewer blocks than the first
left partials for), and again after both beds have stepped."""
import ctypes as C

import numpy as np
import pytest

from paper_2211_01185_amd import cfddem, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _noalloc(lib, bed):
    out = torch.full((2,), float("nan"), dtype=torch.float64, device=bed.device)
    st = C.c_void_p(bed.stream.cuda_stream)
    assert lib.dem_kinetic_energy_noalloc(bed._h, C.c_void_p(out.data_ptr()), st) == cfddem.DEM_OK
    bed.stream.synchronize()
    return out.cpu().numpy()


def test_noalloc_kinetic_energy_equals_the_workspace_one():
    lib = cfddem.load()
    big = cfddem.bed_from_workload(synth.lattice(n_side=(12, 12, 14), seed_index=2), precision="fp64")
    small = cfddem.bed_from_workload(synth.lattice(n_side=(7, 9, 5), seed_index=3), precision="fp64")
    assert big.n > 7 * 256 and small.n < 2 * 256  # the second call has fewer blocks
    for _ in range(2):
        for bed in (big, small):  # two calls in a row, the second smaller
            got = _noalloc(lib, bed)
            want = np.array(bed.kinetic_energy())
            assert np.array_equal(got, want), (got, want)
            assert got[0] > 0.0 and got[1] > 0.0
        big.step(5)
        small.step(5)
    assert big.poll()[0] == 0 and small.poll()[0] == 0

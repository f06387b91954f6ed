"""DEM-only filling and settling on the GPU (the bed preparation that
precedes the coupled cases, Sections 3.2 and 3.3): spheres inserted at
random above the floor fall and come to rest, stepped without coupling.

* Against the oracle through the free fall and the first impacts (contact
  sets bit for bit, states within ten times the single-step tolerance).
* Run to rest (dem_kinetic_energy below 1e-6 of sum m g d): the walls carry
  the bed's weight (static equilibrium), and the settled bed's centre of mass
  and contact count match the oracle's settled bed statistically (the packing
  itself is chaotic).
* dem_kinetic_energy equals 1/2 m v^2 + 1/2 I w^2 summed from the state, and
  is reproducible bit for bit.
* The 100,000-sphere filling of the benchmark column settles as well."""
import math

import numpy as np
import pytest

from paper_2211_01185_amd import settle, synth
from tests.parity_util import TOL, compare_contacts, compare_states, gpu_bed, gpu_state, oracle_bed

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = 9.81


def _small():
    return synth.filling(n=300, d=3e-3, width=0.02, height=0.12, solid_fraction=0.25)


def _mass(wl):
    return wl.density * math.pi / 6.0 * (2.0 * wl.radius) ** 3


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_filling_parity_through_the_first_impacts(precision):
    wl = _small()
    gb = gpu_bed(wl, precision)
    ob, _ = oracle_bed(wl)
    tol = TOL[precision]
    for k in (1000, 2500, 500):  # free fall, first floor contacts at ~3500 steps
        gb.step(k)
        ob.step(k)
        compare_contacts(gb, ob, 10 * tol)
        compare_states(gb, ob, 10 * tol)
    i, j, _ = gb.read_contacts()
    assert i.size > 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_settles_to_rest_in_static_equilibrium(precision):
    wl = _small()
    gb = gpu_bed(wl, precision)
    scale = settle.energy_scale(wl)
    res = settle.settle(gb, scale, rest=1e-6, every=1000, max_steps=80_000)
    assert res.at_rest, res.history[-5:]
    m = _mass(wl)
    W = float(np.sum(m) * G)
    st = gpu_state(gb)
    F = st["Fc"].sum(axis=1)
    assert abs(F[2] / W - 1.0) < 5e-3
    assert np.all(np.abs(F[:2]) < 5e-3 * W)
    # the energy reduction: the definition, and bit-for-bit reproducible
    inertia = 0.4 * m * wl.radius ** 2
    et, er = gb.kinetic_energy()
    assert (et, er) == gb.kinetic_energy()
    want_t = 0.5 * np.sum(m * (st["v"] ** 2).sum(0))
    want_r = 0.5 * np.sum(inertia * (st["w"] ** 2).sum(0))
    assert et == pytest.approx(want_t, rel=1e-12, abs=1e-30)
    assert er == pytest.approx(want_r, rel=1e-12, abs=1e-30)
    # statistics of the settled bed against the oracle's, settled the same way
    ob, _ = oracle_bed(wl)
    inert = 0.4 * m * wl.radius ** 2
    for _ in range(80):
        ob.step(1000)
        so = ob.state()
        ke = 0.5 * np.sum(m * (so["v"] ** 2).sum(0)) + 0.5 * np.sum(inert * (so["w"] ** 2).sum(0))
        if ke <= 1e-6 * scale:
            break
    zg, zo = np.mean(st["x"][2]), np.mean(so["x"][2])
    assert abs(zg / zo - 1.0) < 0.03
    ng, no = gb.read_contacts()[0].size, ob.contacts()[0].size
    assert abs(ng / no - 1.0) < 0.15


def test_full_size_filling_settles():
    wl = synth.filling()
    gb = gpu_bed(wl, "fp32", resort_every=200)
    res = settle.settle(gb, settle.energy_scale(wl), rest=1e-5, every=1000, max_steps=100_000)
    assert res.at_rest, res.history[-5:]
    err, ncont = gb.poll()
    assert err == 0 and ncont > wl.n  # a packed bed: more contacts than spheres
    F = gpu_state(gb)["Fc"].sum(axis=1)
    W = float(np.sum(_mass(wl)) * G)
    assert abs(F[2] / W - 1.0) < 2e-2

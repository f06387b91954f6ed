"""The oracle's parallel loops change no result: a coupled run of a bed with
many contacts gives the same bits at one thread and at several (every sum over
particles or contacts is accumulated in the serial order)."""
import numpy as np

from paper_2211_01185_amd import synth


def _run(O, wl, threads, steps=12):
    O.set_threads(threads)
    d, f = wl.dem, wl.fluid
    p = O.make_params(d["box_lo"], d["box_hi"], d["gravity"], d["dt"], d["E"], d["nu"], d["e"], d["mu"])
    fl = O.make_fluid(f["order"], f["n_el"], f["rho_f"], f["mu_f"], 1, f["eps_min"], shear=1)
    bed = O.OracleBed(p, wl.x, wl.v, wl.w, wl.radius, wl.density)
    outs = []
    for s in range(steps):
        if s % 5 == 0:
            outs.append(bed.couple(fl, wl.U, wl.P))
        bed.step(1)
    return outs, bed.state(), bed.contacts()


def test_results_do_not_depend_on_the_thread_count(oracle_mod):
    O = oracle_mod
    wl = synth.lattice(n_side=(12, 12, 14), spacing_factor=0.97)
    before = O.get_threads()
    try:
        one = _run(O, wl, 1)
        many = _run(O, wl, 4)
    finally:
        O.set_threads(before)
    (c1, s1, k1), (c4, s4, k4) = one, many
    assert len(k1[0]) > wl.n  # a bed with many contacts
    for a, b in zip(c1, c4):
        for key in a:
            assert np.array_equal(a[key], b[key]), key
    for key in s1:
        assert np.array_equal(s1[key], s4[key]), key
    for a, b in zip(k1, k4):
        assert np.array_equal(a, b)

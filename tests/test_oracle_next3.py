"""Pins of the oracle's rolling friction torque (Eq. "angular_momentum") and
shear force -V_p div(tau_f) (Eqs. "fa", "fb", "stress").

* A sphere rolling without slip on the floor under the constant rolling
  torque mu_r R |f_n| decelerates at 5/7 mu_r g (rolling constraint with
  I = 2/5 m R^2) and stops at t = 7 v0 / (5 mu_r g).
* Second derivatives of the 1D Lagrange basis: 0 for Q1; 4, -8, 4 for Q2
  (from 2(t - 1/2)(t - 1), -4t(t - 1), 2t(t - 1/2)).
* div(tau_f) = mu (lap u + grad(div u)/3) for any field Q2 reproduces (per-axis
  quadratics), against derivatives of the polynomial taken term by term; for
  the trilinear field (xy, yz, zx) of Q1 it is mu/3 (1, 1, 1).
* In the coupling, the shear force changes f_fp by exactly -V_p div(tau) of
  the particle, the element sums of the undisturbed-flow forces by their sum,
  and (model B only) F_pf by minus that sum over V_e.

Parity unpinned: the form of the rolling torque itself (the paper names M^r
without a formula; the constant-torque reading is stated in the oracle)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_01185_amd import synth

G = 9.81


def test_rolling_resistance_decelerates_at_five_sevenths_mu_r_g():
    d, rho, E, nu, mu, mu_r, v0, dt = 3e-3, 2500.0, 1e6, 0.3, 0.3, 0.3, 0.1, 1e-5
    R = d / 2
    m = rho * math.pi / 6 * d ** 3
    Ye = 1.0 / (2 * (1 - nu * nu) / E)
    dn = (3 * m * G / (4 * Ye * math.sqrt(R))) ** (2.0 / 3.0)
    x = np.array([[0.005], [0.02], [R - dn]])
    v = np.array([[v0], [0.0], [0.0]])
    w = np.array([[0.0], [v0 / R], [0.0]])  # rolling without slip from the start
    p = O.make_params([0, 0, 0], [0.1, 0.04, 0.04], [0, 0, -G], dt, E, nu, 0.3, mu, mu_r=0.0, mu_r_w=mu_r)
    bed = O.OracleBed(p, x, v, w, np.full(1, R), np.full(1, rho))
    a = 5.0 / 7.0 * mu_r * G
    t_stop = v0 / a
    quarter = int(0.25 * t_stop / dt)
    for k in (1, 2, 3):
        bed.step(quarter)
        st = bed.state()
        t = k * quarter * dt
        assert abs(st["v"][0, 0] - (v0 - a * t)) / v0 < 5e-3, k
        assert abs(st["v"][0, 0] - R * st["w"][1, 0]) / v0 < 5e-3  # still rolling
    bed.step(int(0.5 * t_stop / dt))
    st = bed.state()
    assert abs(st["v"][0, 0]) / v0 < 2e-2  # at rest (up to the torque's chatter)


def test_rolling_torque_vanishes_without_coefficient_or_spin():
    wl = synth.lattice(n_side=(5, 5, 5))
    d = wl.dem
    base = O.make_params(d["box_lo"], d["box_hi"], d["gravity"], d["dt"], d["E"], d["nu"], d["e"], d["mu"])
    rolled = O.make_params(d["box_lo"], d["box_hi"], d["gravity"], d["dt"], d["E"], d["nu"], d["e"], d["mu"],
                           mu_r=0.2, mu_r_w=0.3)
    w0 = np.zeros_like(wl.w)
    a = O.OracleBed(base, wl.x, wl.v, w0, wl.radius, wl.density)
    b = O.OracleBed(rolled, wl.x, wl.v, w0, wl.radius, wl.density)
    # at the creation-time evaluation no particle spins: identical torques
    assert np.array_equal(a.state()["Tc"], b.state()["Tc"])
    c = O.OracleBed(rolled, wl.x, wl.v, wl.w, wl.radius, wl.density)
    e = O.OracleBed(base, wl.x, wl.v, wl.w, wl.radius, wl.density)
    assert np.array_equal(c.state()["Fc"], e.state()["Fc"])  # forces untouched
    assert not np.array_equal(c.state()["Tc"], e.state()["Tc"])
    # every pair torque acts on both bodies with opposite signs: over a bed
    # without walls or gravity the rolling torques sum to zero
    lifted = wl.x.copy()
    lifted[2] += 0.005
    nog = dict(box_lo=d["box_lo"], box_hi=d["box_hi"])
    pa = O.make_params(nog["box_lo"], nog["box_hi"], [0, 0, 0], d["dt"], d["E"], d["nu"], d["e"], d["mu"])
    pb = O.make_params(nog["box_lo"], nog["box_hi"], [0, 0, 0], d["dt"], d["E"], d["nu"], d["e"], d["mu"],
                       mu_r=0.2, mu_r_w=0.3)
    ta = O.OracleBed(pa, lifted, wl.v, wl.w, wl.radius, wl.density).state()["Tc"]
    tb = O.OracleBed(pb, lifted, wl.v, wl.w, wl.radius, wl.density).state()["Tc"]
    diff = (tb - ta).sum(axis=1)
    assert np.all(np.abs(diff) <= 1e-12 * np.abs(tb - ta).sum())


@pytest.mark.parametrize("t", [0.0, 0.1, 0.37, 0.5, 0.93, 1.0])
def test_lagrange_second_derivatives(t):
    for k in range(2):
        assert O.lagrange_deriv2(1, k, t) == 0.0
    assert O.lagrange_deriv2(2, 0, t) == pytest.approx(4.0, abs=1e-12)
    assert O.lagrange_deriv2(2, 1, t) == pytest.approx(-8.0, abs=1e-12)
    assert O.lagrange_deriv2(2, 2, t) == pytest.approx(4.0, abs=1e-12)


def _mesh(order, n_el, lo, hi):
    f = O.make_fluid(order, n_el, 1.2, 1.8e-5)
    axes = [np.linspace(lo[a], hi[a], order * n_el[a] + 1) for a in range(3)]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return f, X.ravel(), Y.ravel(), Z.ravel()


def _poly(coef, x, y, z, dx=0, dy=0, dz=0):
    """sum c[i,j,k] x^i y^j z^k (i, j, k <= 2), or a partial derivative of it."""
    out = np.zeros_like(x, dtype=np.float64)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                if i < dx or j < dy or k < dz:
                    continue
                fi = math.factorial(i) / math.factorial(i - dx)
                fj = math.factorial(j) / math.factorial(j - dy)
                fk = math.factorial(k) / math.factorial(k - dz)
                out += coef[i, j, k] * fi * fj * fk * x ** (i - dx) * y ** (j - dy) * z ** (k - dz)
    return out


def test_stress_divergence_exact_for_q2_fields():
    rng = np.random.default_rng(7)
    lo, hi, n_el = np.array([0.0, -0.1, 0.2]), np.array([0.3, 0.2, 0.8]), [3, 2, 4]
    f, X, Y, Z = _mesh(2, n_el, lo, hi)
    coefs = [rng.normal(size=(3, 3, 3)) for _ in range(3)]
    U = np.stack([_poly(c, X, Y, Z) for c in coefs])
    pts = rng.uniform(lo, hi, size=(200, 3)).T
    got = O.stress_divergence(f, lo, hi, pts, U)
    x, y, z = pts
    mu = f.mu_f
    lap = [sum(_poly(c, x, y, z, *(2 * np.eye(3, dtype=int)[a])) for a in range(3)) for c in coefs]
    # d_a (div u) = sum_j d_a d_j u_j
    gdiv = []
    for a in range(3):
        tot = 0.0
        for j in range(3):
            o = np.zeros(3, dtype=int)
            o[a] += 1
            o[j] += 1
            tot = tot + _poly(coefs[j], x, y, z, *o)
        gdiv.append(tot)
    want = np.stack([mu * (lap[c] + gdiv[c] / 3.0) for c in range(3)])
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-11 * scale


def test_stress_divergence_of_trilinear_q1_field():
    lo, hi, n_el = np.zeros(3), np.array([0.2, 0.3, 0.4]), [2, 3, 4]
    f, X, Y, Z = _mesh(1, n_el, lo, hi)
    U = np.stack([X * Y + 0.3 * Z, Y * Z - X, Z * X + 2.0])
    pts = np.random.default_rng(1).uniform(lo, hi, size=(100, 3)).T
    got = O.stress_divergence(f, lo, hi, pts, U)
    want = np.full_like(got, f.mu_f / 3.0)
    assert np.abs(got - want).max() <= 1e-12 * f.mu_f


@pytest.mark.parametrize("model", [0, 1])
def test_shear_force_enters_the_coupling_as_defined(model):
    wl = synth.plain(n=300)
    d, fl = wl.dem, wl.fluid
    p = O.make_params(d["box_lo"], d["box_hi"], d["gravity"], d["dt"], d["E"], d["nu"], d["e"], d["mu"])
    off = O.make_fluid(fl["order"], fl["n_el"], fl["rho_f"], fl["mu_f"], model, fl["eps_min"])
    on = O.make_fluid(fl["order"], fl["n_el"], fl["rho_f"], fl["mu_f"], model, fl["eps_min"], shear=1)
    a = O.OracleBed(p, wl.x, wl.v, wl.w, wl.radius, wl.density)
    b = O.OracleBed(p, wl.x, wl.v, wl.w, wl.radius, wl.density)
    ra = a.couple(off, wl.U, wl.P)
    rb = b.couple(on, wl.U, wl.P)
    dtau = O.stress_divergence(on, d["box_lo"], d["box_hi"], wl.x, wl.U)
    Vp = 4.0 / 3.0 * np.pi * wl.radius ** 3
    fs = -Vp * dtau
    assert np.abs(fs).max() > 0.0
    dffp = b.state()["ffp"] - a.state()["ffp"]
    assert np.allclose(dffp, fs, rtol=0, atol=1e-9 * np.abs(b.state()["ffp"]).max())
    # element sums of the undisturbed-flow forces gain the per-element shear sums
    es_a, es_b = ra["elem_sums"], rb["elem_sums"]
    nel = es_a.shape[1]
    lo, hi = np.array(d["box_lo"]), np.array(d["box_hi"])
    n_el = np.array(fl["n_el"])
    e3 = np.clip(np.floor((wl.x.T - lo) * n_el / (hi - lo)).astype(int), 0, n_el - 1)
    el = (e3[:, 2] * n_el[1] + e3[:, 1]) * n_el[0] + e3[:, 0]
    per_el = np.stack([np.bincount(el, weights=fs[c], minlength=nel) for c in range(3)])
    assert np.allclose(es_b[9:12] - es_a[9:12], per_el, rtol=0, atol=1e-12 * np.abs(es_b[9:12]).max())
    assert np.array_equal(es_b[:9], es_a[:9])  # drag side untouched
    # the fluid receives it in model B only
    Ve = np.prod((hi - lo) / n_el)
    nq = (fl["order"] + 1) ** 3
    dF = (rb["fpf_q"] - ra["fpf_q"]).reshape(3, nel, nq)
    if model == 0:
        assert np.array_equal(rb["fpf_q"], ra["fpf_q"])
    else:
        want = -(per_el / Ve)[:, :, None] * np.ones(nq)
        assert np.allclose(dF, want, rtol=0, atol=1e-9 * np.abs(rb["fpf_q"]).max())

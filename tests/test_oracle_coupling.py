"""Pins of the oracle's coupling step: printed values of Section 3 (settling
velocity, fluidization pressure drop), closed forms of the Di Felice closure,
polynomial reproduction of the Q2/Q1 interpolation, solid-volume conservation
of the particle-centroid void fraction and the momentum balance of the
quadrature-point reduction."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_2211_01185_amd import synth
from tests.golden import load

G = 9.81


def gauss01(npts):
    """Gauss-Legendre points/weights on [0, 1] from numpy's Legendre module."""
    x, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (x + 1.0), 0.5 * w


def qpt_weights(n_el, lo, hi, order):
    """w_q |J| of every quadrature point, in the element-major, x-fastest order."""
    pts, wts = gauss01(order + 1)
    h = (np.asarray(hi) - np.asarray(lo)) / np.asarray(n_el)
    wz, wy, wx = np.meshgrid(wts, wts, wts, indexing="ij")
    wq = (wx * wy * wz).ravel() * h[0] * h[1] * h[2]
    return np.tile(wq, int(np.prod(n_el)))


# ---------------------------------------------------------------- closure
def test_settling_velocity_printed_in_section_3_1(oracle_mod):
    """Drag balances buoyant weight at the settling velocity quoted for the
    sedimentation case (water, 2 mm glass bead, Di Felice at eps = 1)."""
    O = oracle_mod
    gd = load("sedimentation.txt")
    d, rho_p, rho_f = gd["diameter_m"], gd["particle_density"], gd["fluid_density"]
    mu_f = gd["kinematic_viscosity"] * rho_f
    vp = math.pi / 6 * d ** 3
    weight = vp * (rho_p - rho_f) * G

    def excess(u):
        return O.difelice_beta(rho_f, mu_f, 1.0, d, u) * u - weight

    lo, hi = 0.01, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if excess(mid) < 0 else (lo, mid)
    vt = 0.5 * (lo + hi)
    assert round(vt, int(gd["settling_velocity_digits"])) == gd["settling_velocity_m_s"]
    # closed form at eps = 1: 0.63 s^2 + 4.8 sqrt(nu/d) s - sqrt(K) = 0, s = sqrt(v)
    K = weight / (0.5 * rho_f * math.pi * (d / 2) ** 2)
    b = 4.8 * math.sqrt(gd["kinematic_viscosity"] / d)
    s = (-b + math.sqrt(b * b + 4 * 0.63 * math.sqrt(K))) / (2 * 0.63)
    assert abs(vt / (s * s) - 1) < 1e-6
    # the dynamic-viscosity reading of the table would not reproduce it
    vt_bad_lo, vt_bad_hi = 0.01, 1.0
    for _ in range(200):
        mid = 0.5 * (vt_bad_lo + vt_bad_hi)
        f = O.difelice_beta(rho_f, gd["kinematic_viscosity"], 1.0, d, mid) * mid - weight
        vt_bad_lo, vt_bad_hi = (mid, vt_bad_hi) if f < 0 else (vt_bad_lo, mid)
    assert abs(vt_bad_lo - gd["settling_velocity_m_s"]) > 0.05


def test_stokes_limit(oracle_mod):
    """At vanishing Reynolds number (eps = 1) the closure gives
    beta -> 0.5 rho pi r^2 4.8^2 mu/(rho d) = 0.96 x Stokes' 3 pi mu d."""
    O = oracle_mod
    mu_f, rho_f, d = 1.8e-5, 1.2, 1e-3
    stokes = 3 * math.pi * mu_f * d
    assert abs(O.difelice_beta(rho_f, mu_f, 1.0, d, 0.0) / stokes - 0.96) < 1e-12
    assert abs(O.difelice_beta(rho_f, mu_f, 1.0, d, 1e-16) / stokes - 0.96) < 1e-6


@pytest.mark.parametrize("slip,exponent", [(1e-9, -2.7), (1e9, -1.7)])
def test_voidage_exponent_limits(oracle_mod, slip, exponent):
    """Di Felice's exponent chi -> 3.7 away from Re ~ 10^1.5: beta scales as
    eps^(1-chi) = eps^-2.7 in the viscous limit (C_D ~ 1/Re, Re ~ eps) and
    eps^(2-chi) = eps^-1.7 in the inertial limit (C_D constant)."""
    O = oracle_mod
    mu_f, rho_f, d = 1.8e-5, 1.2, 1e-3
    for eps in (0.4, 0.7):
        ratio = O.difelice_beta(rho_f, mu_f, eps, d, slip) / O.difelice_beta(rho_f, mu_f, 1.0, d, slip)
        assert abs(math.log(ratio) / math.log(eps) - exponent) < 2e-3


def test_fluidization_pressure_drop_printed_in_section_3_2(oracle_mod):
    """Buoyancy on every particle of the fluidized-bed table: the bed's
    buoyant weight over the cross-section equals the quoted pressure drop."""
    O = oracle_mod
    gd = load("fluidization_pressure_drop.txt")
    d, rho_p, rho_f = gd["diameter_m"], gd["particle_density"], gd["fluid_density"]
    lo, hi = [0, 0, 0], [0.02, 0.02, 0.02]
    p = O.make_params(lo, hi, [0, 0, -gd["gravity"]], 1e-5, 1e6, 0.3, 0.9, 0.1)
    x = np.array([[0.01], [0.01], [0.01]])
    bed = O.OracleBed(p, x, np.zeros((3, 1)), np.zeros((3, 1)), np.full(1, d / 2), np.full(1, rho_p))
    fl = O.make_fluid(1, [1, 1, 1], rho_f, 1e-5)
    bed.couple(fl, np.zeros((3, 8)), np.zeros(8))
    f_b = bed.state()["ffp"][2, 0]  # buoyancy only: no slip, no pressure gradient
    weight = rho_p * math.pi / 6 * d ** 3 * gd["gravity"]
    dp = gd["particles"] * (weight - f_b) / (math.pi * gd["bed_radius_m"] ** 2)
    assert abs(dp - gd["pressure_drop_pa"]) < 0.01


# ---------------------------------------------------------------- interpolation
def test_q2_reproduces_quadratics_and_q1_gradient_is_exact(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(3)
    lo, hi, n_el = [0.0, -0.1, 0.2], [0.3, 0.2, 0.8], [3, 4, 5]
    fl = O.make_fluid(2, n_el, 1.2, 1.8e-5)
    cu = rng.normal(size=(3, 3, 3, 3))  # component, x-power, y-power, z-power

    def quad(c, x, y, z):
        return sum(c[i, j, k] * x ** i * y ** j * z ** k for i in range(3) for j in range(3) for k in range(3))

    nodes = synth.node_grid(lo, hi, n_el, 2)
    U = np.stack([quad(cu[c], *nodes) for c in range(3)])
    cp = rng.normal(size=(2, 2, 2))
    pn = synth.node_grid(lo, hi, n_el, 1)
    P = sum(cp[i, j, k] * pn[0] ** i * pn[1] ** j * pn[2] ** k for i in range(2) for j in range(2) for k in range(2))
    x = np.asarray(lo)[:, None] + (np.asarray(hi) - np.asarray(lo))[:, None] * rng.random((3, 500))
    u, gp = O.interpolate(fl, lo, hi, x, U, P)
    want = np.stack([quad(cu[c], *x) for c in range(3)])
    assert np.max(np.abs(u - want)) < 1e-13 * np.max(np.abs(want)) * 10
    X, Y, Z = x
    gx = sum(cp[1, j, k] * Y ** j * Z ** k for j in range(2) for k in range(2))
    gy = sum(cp[i, 1, k] * X ** i * Z ** k for i in range(2) for k in range(2))
    gz = sum(cp[i, j, 1] * X ** i * Y ** j for i in range(2) for j in range(2))
    g_want = np.stack([gx, gy, gz])
    assert np.max(np.abs(gp - g_want)) < 1e-12 * np.max(np.abs(g_want))


def test_q1_velocity_reproduces_trilinear(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(4)
    lo, hi, n_el = [0, 0, 0], [1, 2, 3], [2, 3, 4]
    fl = O.make_fluid(1, n_el, 1.2, 1.8e-5)
    c = rng.normal(size=(2, 2, 2))
    nodes = synth.node_grid(lo, hi, n_el, 1)
    f = sum(c[i, j, k] * nodes[0] ** i * nodes[1] ** j * nodes[2] ** k for i in range(2) for j in range(2) for k in range(2))
    U = np.stack([f, 2 * f, -f])
    x = np.asarray(lo)[:, None] + (np.asarray(hi) - np.asarray(lo))[:, None] * rng.random((3, 200))
    u, _ = O.interpolate(fl, lo, hi, x, U, np.zeros(nodes.shape[1]))
    want = sum(c[i, j, k] * x[0] ** i * x[1] ** j * x[2] ** k for i in range(2) for j in range(2) for k in range(2))
    assert np.max(np.abs(u[0] - want)) < 1e-13 * 10 * np.max(np.abs(want))
    assert np.max(np.abs(u[2] + want)) < 1e-13 * 10 * np.max(np.abs(want))


def test_lagrange_partition_of_unity_and_nodality(oracle_mod):
    O = oracle_mod
    for p in (1, 2):
        for t in np.linspace(0, 1, 11):
            assert abs(sum(O.lagrange(p, k, t) for k in range(p + 1)) - 1) < 1e-15
            assert abs(sum(O.lagrange_deriv(p, k, t) for k in range(p + 1))) < 1e-13
        for k in range(p + 1):
            for m in range(p + 1):
                assert O.lagrange(p, k, m / p) == (1.0 if k == m else 0.0)


# ---------------------------------------------------------------- PCM + reduction
def _bed_and_fields(O, wl, model=0):
    d = wl.dem
    p = O.make_params(d["box_lo"], d["box_hi"], d["gravity"], d["dt"], d["E"], d["nu"], d["e"], d["mu"])
    bed = O.OracleBed(p, wl.x, wl.v, wl.w, wl.radius, wl.density)
    f = wl.fluid
    fl = O.make_fluid(f["order"], f["n_el"], f["rho_f"], f["mu_f"], model, f["eps_min"])
    return bed, fl


def test_pcm_conserves_solid_volume_and_counts(oracle_mod):
    O = oracle_mod
    wl = synth.lattice(n_side=(10, 10, 12))
    bed, fl = _bed_and_fields(O, wl)
    out = bed.couple(fl, wl.U, wl.P)
    lo, hi, n_el = wl.dem["box_lo"], wl.dem["box_hi"], wl.fluid["n_el"]
    vp = 4.0 / 3.0 * math.pi * wl.radius ** 3
    wq = qpt_weights(n_el, lo, hi, wl.fluid["order"])
    solid = np.sum(wq * (1.0 - out["eps_q"]))
    assert abs(solid / vp.sum() - 1) < 1e-12
    edges = [np.linspace(lo[a], hi[a], n_el[a] + 1) for a in range(3)]
    counts, _ = np.histogramdd(wl.x.T[:, ::-1], bins=edges[::-1])  # z, y, x -> x fastest
    assert np.array_equal(out["elem_sums"][0], counts.ravel())


@pytest.mark.parametrize("model", [0, 1])
def test_reduction_momentum_balance(oracle_mod, model):
    """Uniform fluid velocity: the force density handed to the fluid,
    integrated over the quadrature weights, equals minus the drag on the
    particles (model A), plus minus the pressure-gradient force (model B)."""
    O = oracle_mod
    wl = synth.lattice(n_side=(10, 10, 12))
    U = np.zeros_like(wl.U)
    U[0], U[2] = 0.1, 0.7
    bed, fl = _bed_and_fields(O, wl, model)
    out = bed.couple(fl, U, wl.P)
    wq = qpt_weights(wl.fluid["n_el"], wl.dem["box_lo"], wl.dem["box_hi"], wl.fluid["order"])
    total = (out["fpf_q"] * wq).sum(axis=1)
    fD = out["elem_sums"][6:9].sum(axis=1)
    fG = out["elem_sums"][9:12].sum(axis=1)
    want = -(fD + fG) if model == 1 else -fD
    assert np.max(np.abs(total - want)) < 1e-12 * np.max(np.abs(want))
    assert np.max(np.abs(fG)) > 0
    # particle-side force = drag + buoyancy + pressure gradient, per element
    st = bed.state()
    vp = 4.0 / 3.0 * math.pi * wl.radius ** 3
    fB = -wl.fluid["rho_f"] * vp.sum() * np.asarray(wl.dem["gravity"])
    assert np.allclose(st["ffp"].sum(axis=1), fD + fG + fB, rtol=1e-12, atol=1e-18)


def test_sedimentation_transient_follows_the_ode(oracle_mod):
    """Section 3.1: one bead released at rest in water, drag and buoyancy only.
    The DEM+coupling trajectory follows m du/dt = F_D - V_p (rho_p - rho_f) g
    (integrated here by scipy) and settles at the quoted velocity."""
    O = oracle_mod
    gd = load("sedimentation.txt")
    d, rho_p, rho_f = gd["diameter_m"], gd["particle_density"], gd["fluid_density"]
    mu_f = gd["kinematic_viscosity"] * rho_f
    lo, hi = [0, 0, 0], [0.1, 0.1, 0.3]
    vp = math.pi / 6 * d ** 3
    m = rho_p * vp

    def run(f_coupling, t_end, record):
        dt = 1e-5
        p = O.make_params(lo, hi, [0, 0, -G], dt, 1e6, 0.3, 0.2, 0.1)
        bed = O.OracleBed(p, np.array([[0.05], [0.05], [0.28]]), np.zeros((3, 1)), np.zeros((3, 1)),
                          np.full(1, d / 2), np.full(1, rho_p))
        fl = O.make_fluid(1, [1, 1, 1], rho_f, mu_f)
        ts, vs = [0.0], [0.0]
        for c in range(int(round(t_end / (f_coupling * dt)))):
            bed.couple(fl, np.zeros((3, 8)), np.zeros(8))
            bed.step(f_coupling)
            if record:
                ts.append((c + 1) * f_coupling * dt)
                vs.append(-bed.state()["v"][2, 0])
        return np.array(ts), np.array(vs), bed

    eps = 1.0 - vp / 3e-3

    def rhs(_t, u):
        return [(O.difelice_beta(rho_f, mu_f, eps, d, abs(u[0])) * (-u[0]) + vp * (rho_p - rho_f) * G) / m]

    ts, vs, _ = run(10, 0.1, True)
    sol = solve_ivp(rhs, (0, 0.1), [0.0], t_eval=ts, rtol=1e-10, atol=1e-12)
    assert np.max(np.abs(vs - sol.y[0])) < 5e-3 * gd["settling_velocity_m_s"]
    _, vs100, _ = run(int(gd["coupling_frequency"]), 0.25, True)
    assert abs(vs100[-1] - gd["settling_velocity_m_s"]) < 1e-3 * gd["settling_velocity_m_s"] + 5e-5

"""Helpers shared by the GPU parity tests: build the same bed in the oracle and
on the GPU from one seeded workload, and compare arrays."""
import numpy as np

from oracle import oracle as O

# Tolerances on max|gpu - oracle| / max|oracle| per array (single steps).
TOL = {"fp64": 1e-10, "fp32": 1e-5}


def oracle_bed(wl, model=None):
    d = wl.dem
    p = O.make_params(d["box_lo"], d["box_hi"], d["gravity"], d["dt"], d["E"], d["nu"], d["e"], d["mu"],
                      d["E_w"], d["nu_w"], d["e_w"], d["mu_w"], d.get("mu_r", 0.0),
                      d.get("mu_r_w", d.get("mu_r", 0.0)))
    f = wl.fluid
    fl = O.make_fluid(f["order"], f["n_el"], f["rho_f"], f["mu_f"],
                      f.get("model", 0) if model is None else model, f["eps_min"],
                      f.get("drag", 0), f.get("beta_over_eps", 0), 1 if f.get("shear") else 0)
    return O.OracleBed(p, wl.x, wl.v, wl.w, wl.radius, wl.density), fl


def gpu_bed(wl, precision="fp64", **kw):
    from paper_2211_01185_amd import cfddem
    return cfddem.bed_from_workload(wl, precision=precision, **kw)


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = np.max(np.abs(want)) if want.size else 0.0
    diff = np.max(np.abs(got - want)) if want.size else 0.0
    if scale == 0.0:
        return diff
    return diff / scale


def assert_close(name, got, want, tol):
    e = rel_err(got, want)
    assert e <= tol, f"{name}: relative max-norm error {e:.3e} > {tol:.1e}"


def gpu_state(bed):
    st = bed.read_state()
    F, T = bed.read_forces()
    out = {k: v.cpu().numpy() for k, v in st.items()}
    out["Fc"] = F.cpu().numpy()
    out["Tc"] = T.cpu().numpy()
    return out


def contact_set(i, j):
    return set(zip(np.asarray(i).tolist(), np.asarray(j).tolist()))


def compare_contacts(gbed, obed, tol):
    gi, gj, gdt = gbed.read_contacts()
    oi, oj, odt = obed.contacts()
    assert contact_set(gi, gj) == contact_set(oi, oj)
    # both are sorted by (i, j)
    assert np.array_equal(gi, oi) and np.array_equal(gj, oj)
    if odt.size and np.max(np.abs(odt)) > 0:
        assert_close("delta_t", gdt, odt, tol)
    else:
        assert np.max(np.abs(gdt)) == 0.0 if gdt.size else True
    return len(oi)


def compare_states(gbed, obed, tol, keys=("x", "v", "w", "ffp", "Fc", "Tc")):
    g = gpu_state(gbed)
    o = obed.state()
    for k in keys:
        if np.max(np.abs(o[k])) == 0.0:
            assert np.max(np.abs(g[k])) <= 1e-300, k
        else:
            assert_close(k, g[k], o[k], tol)

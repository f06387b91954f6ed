"""ctypes wrapper of the FP64 CPU oracle (oracle/cfddem_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the HIP library or its binding.

Arrays are numpy float64, component-major (shape (3, n) for vectors).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

ERR_DOMAIN = 1
ERR_NAN = 2


class OrcParams(C.Structure):
    _fields_ = [
        ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3), ("gravity", C.c_double * 3),
        ("dt", C.c_double),
        ("E", C.c_double), ("nu", C.c_double), ("e", C.c_double), ("mu", C.c_double),
        ("E_w", C.c_double), ("nu_w", C.c_double), ("e_w", C.c_double), ("mu_w", C.c_double),
        ("mu_r", C.c_double), ("mu_r_w", C.c_double),
    ]


class OrcFluid(C.Structure):
    _fields_ = [
        ("order", C.c_int), ("n_el", C.c_int * 3), ("rho_f", C.c_double), ("mu_f", C.c_double),
        ("model", C.c_int), ("eps_min", C.c_double), ("drag", C.c_int), ("beta_over_eps", C.c_int),
        ("shear", C.c_int),
    ]


DRAG = {"difelice": 0, "dallavalle": 1, "rong": 2, "koch_hill": 3, "beetstra": 4, "gidaspow": 5}


_lib = None
_dp = C.POINTER(C.c_double)
_lp = C.POINTER(C.c_long)
_ip = C.POINTER(C.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from oracle import build as _b  # build on first use (gcc, seconds)
        _b.build()
    lib = C.CDLL(LIB_PATH)
    lib.orc_bin.restype = C.c_long
    lib.orc_bin.argtypes = [C.c_long, _dp, _dp, _dp, _ip, _ip, _ip, _lp]
    lib.orc_find_pairs.restype = C.c_long
    lib.orc_find_pairs.argtypes = [C.c_long, _dp, _dp, _dp, _dp, C.c_long, _lp, _lp]
    lib.orc_lagrange.restype = C.c_double
    lib.orc_lagrange.argtypes = [C.c_int, C.c_int, C.c_double]
    lib.orc_lagrange_deriv.restype = C.c_double
    lib.orc_lagrange_deriv.argtypes = [C.c_int, C.c_int, C.c_double]
    lib.orc_lagrange_deriv2.restype = C.c_double
    lib.orc_lagrange_deriv2.argtypes = [C.c_int, C.c_int, C.c_double]
    lib.orc_stress_divergence.restype = None
    lib.orc_stress_divergence.argtypes = [C.POINTER(OrcFluid), _dp, _dp, C.c_long, _dp, _dp, _dp]
    lib.orc_interpolate.restype = None
    lib.orc_interpolate.argtypes = [C.POINTER(OrcFluid), _dp, _dp, C.c_long, _dp, _dp, _dp, _dp, _dp]
    lib.orc_difelice_beta.restype = C.c_double
    lib.orc_difelice_beta.argtypes = [C.c_double] * 5
    lib.orc_drag_beta.restype = C.c_double
    lib.orc_drag_beta.argtypes = [C.c_int] + [C.c_double] * 5
    lib.orc_dem_create.restype = C.c_void_p
    lib.orc_dem_create.argtypes = [C.POINTER(OrcParams), C.c_long, _dp, _dp, _dp, _dp, _dp]
    lib.orc_dem_step.restype = C.c_int
    lib.orc_dem_step.argtypes = [C.c_void_p, C.c_long]
    lib.orc_dem_couple.restype = C.c_int
    lib.orc_dem_couple.argtypes = [C.c_void_p, C.POINTER(OrcFluid), _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_dem_couple_field.restype = C.c_int
    lib.orc_dem_couple_field.argtypes = [C.c_void_p, C.POINTER(OrcFluid), _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_dem_get.restype = None
    lib.orc_dem_get.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_dem_set_ffp.restype = None
    lib.orc_dem_set_ffp.argtypes = [C.c_void_p, _dp]
    lib.orc_dem_ncontacts.restype = C.c_long
    lib.orc_dem_ncontacts.argtypes = [C.c_void_p]
    lib.orc_dem_contacts.restype = None
    lib.orc_dem_contacts.argtypes = [C.c_void_p, _lp, _lp, _dp]
    lib.orc_dem_error.restype = C.c_int
    lib.orc_dem_error.argtypes = [C.c_void_p]
    lib.orc_dem_free.restype = None
    lib.orc_dem_free.argtypes = [C.c_void_p]
    lib.orc_set_threads.restype = None
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_get_threads.restype = C.c_int
    lib.orc_get_threads.argtypes = []
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (results do not depend on it)."""
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def make_params(box_lo, box_hi, gravity, dt, E, nu, e, mu, E_w=None, nu_w=None, e_w=None,
                mu_w=None, mu_r=0.0, mu_r_w=None) -> OrcParams:
    p = OrcParams()
    p.box_lo[:] = [float(v) for v in box_lo]
    p.box_hi[:] = [float(v) for v in box_hi]
    p.gravity[:] = [float(v) for v in gravity]
    p.dt = dt
    p.E, p.nu, p.e, p.mu = E, nu, e, mu
    p.E_w = E if E_w is None else E_w
    p.nu_w = nu if nu_w is None else nu_w
    p.e_w = e if e_w is None else e_w
    p.mu_w = mu if mu_w is None else mu_w
    p.mu_r = float(mu_r)
    p.mu_r_w = float(mu_r if mu_r_w is None else mu_r_w)
    return p


def make_fluid(order, n_el, rho_f, mu_f, model=0, eps_min=0.1, drag=0, beta_over_eps=0,
               shear=0) -> OrcFluid:
    f = OrcFluid()
    f.order = int(order)
    f.n_el[:] = [int(v) for v in n_el]
    f.rho_f, f.mu_f = float(rho_f), float(mu_f)
    f.model = int(model)
    f.eps_min = float(eps_min)
    f.drag = DRAG[drag] if isinstance(drag, str) else int(drag)
    f.beta_over_eps = int(beta_over_eps)
    f.shear = int(shear)
    return f


def stress_divergence(f: OrcFluid, lo, hi, x, U):
    """div(tau_f) of Eq. "stress" at the points x (3, n) of the field U (3, n_v)."""
    lib = _load()
    x = _f64(x)
    n = x.shape[1]
    U = _f64(U)
    out = np.zeros((3, n))
    lib.orc_stress_divergence(C.byref(f), _d(_f64(lo)), _d(_f64(hi)), n, _d(x), _d(U), _d(out))
    return out


def lagrange_deriv2(p, k, t):
    return _load().orc_lagrange_deriv2(int(p), int(k), float(t))


def element_matrices(order, he):
    """Mass, stiffness and load of one element of size he (3,) in the Q_order
    space: M_ij = int phi_i phi_j, K_ij = int grad phi_i . grad phi_j,
    b_i = int phi_i, by (order+1)-point Gauss quadrature per axis (exact for
    these polynomial integrands).  Local node l = (ic (p+1) + ib) (p+1) + ia."""
    lib = _load()
    p = int(order)
    gx, gw = np.polynomial.legendre.leggauss(p + 1)
    t, w = 0.5 * (gx + 1.0), 0.5 * gw
    L = np.array([[lib.orc_lagrange(p, k, tq) for tq in t] for k in range(p + 1)])
    dL = np.array([[lib.orc_lagrange_deriv(p, k, tq) for tq in t] for k in range(p + 1)])
    loc = [(ia, ib, ic) for ic in range(p + 1) for ib in range(p + 1) for ia in range(p + 1)]
    nl = len(loc)
    M, K, b = np.zeros((nl, nl)), np.zeros((nl, nl)), np.zeros(nl)
    J = float(np.prod(he))
    for qz in range(p + 1):
        for qy in range(p + 1):
            for qx in range(p + 1):
                wq = w[qx] * w[qy] * w[qz] * J
                phi = np.array([L[a, qx] * L[bb, qy] * L[c, qz] for a, bb, c in loc])
                grad = np.array([[dL[a, qx] * L[bb, qy] * L[c, qz] / he[0],
                                  L[a, qx] * dL[bb, qy] * L[c, qz] / he[1],
                                  L[a, qx] * L[bb, qy] * dL[c, qz] / he[2]] for a, bb, c in loc])
                M += wq * np.outer(phi, phi)
                K += wq * grad @ grad.T
                b += wq * phi
    return M, K, b


def element_nodes(order, n_el):
    """Global velocity-node index (x fastest) of local node l of element e,
    shape (n_elements, (order+1)^3)."""
    p = int(order)
    n_el = [int(v) for v in n_el]
    nx, ny = p * n_el[0] + 1, p * n_el[1] + 1
    ez, ey, ex = np.meshgrid(np.arange(n_el[2]), np.arange(n_el[1]), np.arange(n_el[0]), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    cols = []
    for ic in range(p + 1):
        for ib in range(p + 1):
            for ia in range(p + 1):
                cols.append(((p * ez + ic) * ny + (p * ey + ib)) * nx + (p * ex + ia))
    return np.stack(cols, axis=1)


def smooth_void_fraction(fluid: OrcFluid, lo, hi, eps_e, L2):
    """Continuous void fraction from the element PCM values eps_e: the field
    eps_h of the velocity space Q_order with, for every basis function phi_i,
        int eps_h phi_i + L2 int grad eps_h . grad phi_i = int eps_PCM phi_i
    (natural boundary conditions; L2 = 0 is the L2 projection).  Global
    assembly of the element matrices and a direct sparse solve.  Returns the
    nodal values."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.linalg import spsolve

    lo, hi = _f64(lo), _f64(hi)
    n_el = np.array([int(v) for v in fluid.n_el])
    he = (hi - lo) / n_el
    M, K, be = element_matrices(fluid.order, he)
    Ae = M + float(L2) * K
    g = element_nodes(fluid.order, n_el)
    nv = int(np.prod(int(fluid.order) * n_el + 1))
    ne, nl = g.shape
    rows = np.repeat(g, nl, axis=1).ravel()
    cols = np.tile(g, (1, nl)).ravel()
    A = coo_matrix((np.tile(Ae.ravel(), ne), (rows, cols)), shape=(nv, nv)).tocsc()
    b = np.bincount(g.ravel(), weights=(np.asarray(eps_e, float)[:, None] * be[None, :]).ravel(),
                    minlength=nv)
    return spsolve(A, b)


def bin_particles(x, lo, hi, n_el, k):
    """Element and cell index of every particle (hierarchical binning)."""
    lib = _load()
    x = _f64(x)
    n = x.shape[1]
    elem = np.zeros(n, dtype=np.int32)
    cell = np.zeros(n, dtype=np.int64)
    lo_a, hi_a = _f64(lo), _f64(hi)
    ne = (C.c_int * 3)(*[int(v) for v in n_el])
    kk = (C.c_int * 3)(*[int(v) for v in k])
    outside = lib.orc_bin(n, _d(x), _d(lo_a), _d(hi_a), ne, kk, elem.ctypes.data_as(_ip),
                          cell.ctypes.data_as(_lp))
    return elem, cell, int(outside)


def find_pairs(x, r, lo, hi):
    """Sorted (i, j), i < j, of all touching pairs."""
    lib = _load()
    x = _f64(x)
    r = _f64(r)
    n = x.shape[1]
    lo_a, hi_a = _f64(lo), _f64(hi)
    cnt = lib.orc_find_pairs(n, _d(x), _d(r), _d(lo_a), _d(hi_a), 0, None, None)
    pi = np.zeros(max(cnt, 1), dtype=np.int64)
    pj = np.zeros(max(cnt, 1), dtype=np.int64)
    lib.orc_find_pairs(n, _d(x), _d(r), _d(lo_a), _d(hi_a), cnt, pi.ctypes.data_as(_lp),
                       pj.ctypes.data_as(_lp))
    return pi[:cnt], pj[:cnt]


def lagrange(p, k, t):
    return _load().orc_lagrange(int(p), int(k), float(t))


def lagrange_deriv(p, k, t):
    return _load().orc_lagrange_deriv(int(p), int(k), float(t))


def interpolate(fluid: OrcFluid, lo, hi, x, U, P):
    lib = _load()
    x = _f64(x)
    n = x.shape[1]
    U = _f64(U)
    P = _f64(P)
    u = np.zeros((3, n))
    gp = np.zeros((3, n))
    lo_a, hi_a = _f64(lo), _f64(hi)
    lib.orc_interpolate(C.byref(fluid), _d(lo_a), _d(hi_a), n, _d(x), _d(U), _d(P), _d(u), _d(gp))
    return u, gp


def difelice_beta(rho_f, mu_f, eps, d, slip):
    return _load().orc_difelice_beta(float(rho_f), float(mu_f), float(eps), float(d), float(slip))


def drag_beta(drag, rho_f, mu_f, eps, d, slip):
    """Momentum-exchange coefficient of one particle for closure `drag`
    (a name of DRAG or its number)."""
    k = DRAG[drag] if isinstance(drag, str) else int(drag)
    return _load().orc_drag_beta(k, float(rho_f), float(mu_f), float(eps), float(d), float(slip))


class OracleBed:
    """One DEM bed in the oracle: create (with priming), step, couple, read."""

    def __init__(self, params: OrcParams, x, v, w, radius, density):
        self._lib = _load()
        x, v, w = _f64(x), _f64(v), _f64(w)
        self.n = x.shape[1]
        self.params = params
        r = _f64(radius)
        rho = _f64(density)
        self._h = self._lib.orc_dem_create(C.byref(params), self.n, _d(x), _d(v), _d(w), _d(r), _d(rho))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_dem_free(h)
            self._h = None

    def step(self, nsteps=1) -> int:
        return self._lib.orc_dem_step(self._h, int(nsteps))

    def couple(self, fluid: OrcFluid, U, P, smooth_L2=None):
        """One coupling step.  smooth_L2: None for the element PCM void
        fraction, else the smoothing length L^2 of the continuous field."""
        n_el = int(fluid.n_el[0]) * int(fluid.n_el[1]) * int(fluid.n_el[2])
        nq = (fluid.order + 1) ** 3
        U = _f64(U)
        P = _f64(P)
        eps_q = np.zeros(n_el * nq)
        beta_q = np.zeros(n_el * nq)
        fpf_q = np.zeros((3, n_el * nq))
        sums = np.zeros((12, n_el))
        err = self._lib.orc_dem_couple(self._h, C.byref(fluid), _d(U), _d(P), _d(eps_q), _d(beta_q),
                                       _d(fpf_q), _d(sums))
        out = dict(eps_q=eps_q, beta_q=beta_q, fpf_q=fpf_q, elem_sums=sums, err=err)
        if smooth_L2 is None:
            return out
        # smoothed void fraction: element PCM values, projection, then the
        # coupling step again with the continuous field
        hi = np.array(self.params.box_hi[:])
        lo = np.array(self.params.box_lo[:])
        Ve = float(np.prod((hi - lo) / np.array(fluid.n_el[:])))
        eps_e = 1.0 - sums[1] / Ve
        eps_nodes = smooth_void_fraction(fluid, lo, hi, eps_e, smooth_L2)
        err = self._lib.orc_dem_couple_field(self._h, C.byref(fluid), _d(U), _d(P), _d(eps_nodes), _d(eps_q),
                                             _d(beta_q), _d(fpf_q), _d(sums))
        return dict(eps_q=eps_q, beta_q=beta_q, fpf_q=fpf_q, elem_sums=sums, err=err, eps_nodes=eps_nodes,
                    eps_e=eps_e)

    def state(self):
        n = self.n
        out = {k: np.zeros((3, n)) for k in ("x", "v", "w", "ffp", "Fc", "Tc")}
        self._lib.orc_dem_get(self._h, _d(out["x"]), _d(out["v"]), _d(out["w"]), _d(out["ffp"]),
                              _d(out["Fc"]), _d(out["Tc"]))
        return out

    def set_ffp(self, ffp):
        ffp = _f64(ffp)
        self._lib.orc_dem_set_ffp(self._h, _d(ffp))

    def contacts(self):
        c = self._lib.orc_dem_ncontacts(self._h)
        i = np.zeros(max(c, 1), dtype=np.int64)
        j = np.zeros(max(c, 1), dtype=np.int64)
        dt = np.zeros((max(c, 1), 3))
        self._lib.orc_dem_contacts(self._h, i.ctypes.data_as(_lp), j.ctypes.data_as(_lp), _d(dt))
        return i[:c], j[:c], dt[:c]

    @property
    def error(self) -> int:
        return self._lib.orc_dem_error(self._h)

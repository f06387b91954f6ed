"""Pins of the oracle's smoothed void fraction (NEXT-2): the element PCM
values (Eq. "void_fraction") projected onto the continuous velocity space
with smoothing length L^2 (Tables "tab:setup2", "tab:setup4": 4 d^2, 5 d^2):
    int eps_h phi + L^2 int grad eps_h . grad phi = int eps_PCM phi.

* Solid volume is conserved for every L^2 (phi = 1 is in the space): the
  field integrated at the Gauss points equals sum_e eps_e V_e.
* A uniform PCM field is reproduced exactly (the stiffness of a constant
  vanishes).
* A cosine mode along the column, cos(k z) with k = m pi / H (a Neumann
  eigenfunction), comes out damped by 1 / (1 + L^2 k^2), to the
  discretization error O((k h)^2); L^2 = 0 gives the mode itself.
* For L^2 much larger than the box, the field tends to the mean.

Parity unpinned: the scheme itself is described in a companion paper, not in
this one; the weak form above is the reading."""
import numpy as np
import pytest

from oracle import oracle as O


def _gauss(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _field_at_qpts(order, n_el, lo, hi, eps_nodes):
    """The nodal field evaluated at the Gauss points of every element
    (same numbering as the coupling outputs), and the quadrature weights."""
    lib = O._load()
    p = order
    t, w = _gauss(p + 1)
    L = np.array([[lib.orc_lagrange(p, k, tq) for tq in t] for k in range(p + 1)])
    g = O.element_nodes(p, n_el)
    vals = eps_nodes[g]  # (ne, nl)
    loc = [(a, b, c) for c in range(p + 1) for b in range(p + 1) for a in range(p + 1)]
    q = []
    wq = []
    for qz in range(p + 1):
        for qy in range(p + 1):
            for qx in range(p + 1):
                phi = np.array([L[a, qx] * L[b, qy] * L[c, qz] for a, b, c in loc])
                q.append(vals @ phi)
                wq.append(w[qx] * w[qy] * w[qz])
    he = (np.asarray(hi) - np.asarray(lo)) / np.asarray(n_el)
    return np.stack(q, axis=1), np.array(wq) * np.prod(he)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("L2", [0.0, 4e-6, 1.25e-6, 3e-4])
def test_volume_conserved(order, L2):
    rng = np.random.default_rng(3)
    n_el, lo, hi = [3, 4, 5], [0.0, 0.0, 0.0], [0.015, 0.02, 0.03]
    f = O.make_fluid(order, n_el, 1.2, 1.8e-5)
    eps_e = rng.uniform(0.3, 1.0, size=int(np.prod(n_el)))
    nodes = O.smooth_void_fraction(f, lo, hi, eps_e, L2)
    q, wq = _field_at_qpts(order, n_el, lo, hi, nodes)
    Ve = np.prod((np.array(hi) - np.array(lo)) / np.array(n_el))
    assert np.sum(q * wq[None, :]) == pytest.approx(np.sum(eps_e) * Ve, rel=1e-12)
    if L2 > 10 * (0.005 ** 2):
        # smoothing over more than the element size: flatter than the element
        # values (a projection with L^2 << h^2 may overshoot them)
        assert np.ptp(nodes) < np.ptp(eps_e)


@pytest.mark.parametrize("order", [1, 2])
def test_uniform_field_reproduced(order):
    n_el, lo, hi = [2, 3, 4], [0.0, 0.0, 0.0], [0.01, 0.02, 0.02]
    f = O.make_fluid(order, n_el, 1.2, 1.8e-5)
    nodes = O.smooth_void_fraction(f, lo, hi, np.full(24, 0.62), 5e-6)
    assert np.allclose(nodes, 0.62, rtol=0, atol=1e-13)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("damping", [0.0, 1.0, 3.0])  # L^2 k^2
def test_cosine_mode_damped(order, damping):
    H, nz = 0.2, 200
    n_el, lo, hi = [1, 1, nz], [0.0, 0.0, 0.0], [0.01, 0.01, H]
    k = 4.0 * np.pi / H
    L2 = damping / k ** 2
    f = O.make_fluid(order, n_el, 1.2, 1.8e-5)
    z = np.linspace(0.0, H, nz + 1)
    a = 0.1
    # element averages of 0.5 + a cos(k z)
    eps_e = 0.5 + a * (np.sin(k * z[1:]) - np.sin(k * z[:-1])) / (k * (H / nz))
    nodes = O.smooth_void_fraction(f, lo, hi, eps_e, L2)
    nzn = order * nz + 1
    zn = np.linspace(0.0, H, nzn)
    line = nodes.reshape(nzn, -1)[:, 0]  # x = y = 0 column of nodes (x fastest)
    want = 0.5 + a * np.cos(k * zn) / (1.0 + damping)
    assert np.abs(line - want).max() < 3e-3 * a


def test_large_smoothing_tends_to_mean():
    rng = np.random.default_rng(9)
    n_el, lo, hi = [3, 3, 6], [0.0, 0.0, 0.0], [0.01, 0.01, 0.02]
    f = O.make_fluid(2, n_el, 1.2, 1.8e-5)
    eps_e = rng.uniform(0.4, 1.0, size=54)
    nodes = O.smooth_void_fraction(f, lo, hi, eps_e, 1e3 * 0.02 ** 2)
    assert np.abs(nodes - eps_e.mean()).max() < 1e-4

"""Seeded synthetic workloads (particle beds and given fluid fields).

This module only draws inputs: it holds none of the method's arithmetic and
imports nothing from the rest of the package, so the HIP path and the CPU
oracle can both be fed from it.  Every generator takes its seed from
``seed_for(config, index)`` and uses numpy's PCG64.

Workloads (stand-ins for the paper's beds, whose meshes and packings are not
available):
  * ``plain``     2,000 spheres, d = 3 mm, random sequential addition in a
                  0.05 x 0.05 x 0.2 m box; Q2 4x4x16 mesh; uniform (0,0,0.5) m/s.
  * ``fluidized`` 100,000 spheres, d = 1 mm, jittered simple-cubic lattice at
                  solid fraction 0.4 in 0.1 x 0.1 x 0.4 m; Q2 20x20x80 mesh;
                  (0,0,1.2) m/s + N(0, 0.05) per velocity node; linear pressure
                  carrying the bed's buoyant weight (Eq. "dpf").
  * ``spouted``   500,000 spheres, lognormal d (median 2 mm, sigma 0.2, clipped
                  to 1-4 mm), random sequential addition in z < 0.45 m of a
                  0.15 x 0.15 x 0.6 m box; Q2 30x30x120 mesh; Gaussian jet of
                  peak 20 m/s and width 0.01 m decaying as exp(-z/0.2).
  * ``lattice``   the plain geometry on a simple-cubic lattice of spacing
                  0.98 d: every neighbour overlaps (contact-heavy parity case).
  * ``batched``   64 independent column beds of 5k-80k spheres with their own
                  diameter, restitution and inlet velocity and their own Q1 mesh.
  * ``job_stream`` Poisson arrivals of sedimentation / fluidization column beds
                  of 1k-200k spheres (the served workload).
  * ``filling``   DEM-only bed preparation: 100,000 spheres, d = 1 mm, at rest
                  at solid fraction 0.15 in a layer above the floor of the
                  fluidized-bed column, left to settle under gravity.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 2211011850
G = 9.81


def seed_for(config: int, index: int = 0) -> int:
    return BASE_SEED + 1000 * config + index


def rng_for(config: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_for(config, index)))


@dataclass
class Workload:
    name: str
    x: np.ndarray        # (3, N) positions
    v: np.ndarray        # (3, N) velocities
    w: np.ndarray        # (3, N) angular velocities
    radius: np.ndarray   # (N,)
    density: np.ndarray  # (N,)
    dem: dict            # box_lo, box_hi, gravity, dt, E, nu, e, mu, E_w, nu_w, e_w, mu_w
    fluid: dict          # order, n_el, rho_f, mu_f, model, eps_min
    run: dict            # steps, coupling_every, precision ("fp64" | "fp32")
    U: np.ndarray = field(default=None)  # (3, n_v) nodal velocity
    P: np.ndarray = field(default=None)  # (n_p,) nodal Q1 pressure

    @property
    def n(self) -> int:
        return int(self.x.shape[1])


def _material(**over) -> dict:
    base = dict(E=1e6, nu=0.3, e=0.9, mu=0.3)
    base.update(over)
    out = dict(base)
    for k in ("E", "nu", "e", "mu"):
        out[k + "_w"] = over.get(k + "_w", base[k])
    return out


def node_grid(lo, hi, n_el, order):
    """Coordinates (3, n_nodes) of the structured Q_order node lattice, x fastest."""
    axes = [np.linspace(lo[a], hi[a], order * n_el[a] + 1) for a in range(3)]
    zz, yy, xx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()])


def rsa_monodisperse(rng, n, d, lo, hi, max_tries=2000000):
    """Random sequential addition: centres at least d/2 from every wall and
    strictly more than d apart."""
    r = 0.5 * d
    lo_c = np.asarray(lo, float) + r
    hi_c = np.asarray(hi, float) - r
    pts = np.zeros((0, 3))
    tries = 0
    while pts.shape[0] < n and tries < max_tries:
        cand = lo_c + (hi_c - lo_c) * rng.random((min(4 * (n - pts.shape[0]), 4096), 3))
        tries += cand.shape[0]
        for c in cand:
            if pts.shape[0] and np.min(np.sum((pts - c) ** 2, axis=1)) <= d * d:
                continue
            pts = np.vstack([pts, c])
            if pts.shape[0] == n:
                break
    if pts.shape[0] < n:
        raise RuntimeError("random sequential addition did not reach the requested count")
    return pts.T.copy()


def rsa_polydisperse(rng, radius, lo, hi):
    """Random sequential addition of spheres with the given radii inside
    [lo, hi], wall distance >= r, centre distance > r_i + r_j.  The radii are
    placed largest first (the small ones then fill the gaps; in the drawn order
    the last large spheres find no room long before the target fraction), and
    the returned centres are listed in the order of ``radius`` on return, which
    the caller shuffles.  Candidates come in batches; clashes with accepted
    spheres are found with one vectorized k-d tree distance query per batch,
    clashes inside a batch keep the earlier candidate, and rejected radii are
    retried in the next batch."""
    from scipy.spatial import cKDTree

    n = radius.shape[0]
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    radius[:] = np.sort(radius)[::-1]
    rmax = float(radius.max())
    pts = np.zeros((n, 3))
    placed = 0
    # accepted centres in two trees: an old one, rebuilt only when the recent
    # one has grown to a fifth of it, and a recent one rebuilt every batch
    old_n, old_tree, trees = 0, None, []
    while placed < n:
        left = n - placed
        batch = min(left, 50000)
        # few spheres left: several candidate positions for each, copy c of
        # every sphere before copy c + 1 (at most as many candidates as fill
        # the box once, so that a small box is not flooded)
        fill = float(np.prod(hi - lo)) / (batch * 4.0 / 3.0 * math.pi * rmax ** 3)
        copies = max(1, min(20000 // batch, int(fill)))
        sid = np.tile(np.arange(batch), copies)
        rb = radius[placed:placed + batch][sid]
        cand = lo + rb[:, None] + (hi - lo - 2 * rb[:, None]) * rng.random((sid.shape[0], 3))
        ok = np.ones(sid.shape[0], dtype=bool)
        ctree = cKDTree(cand)
        for first_id, tree in trees:
            m = tree.sparse_distance_matrix(ctree, 2 * rmax, output_type="ndarray")
            if m.shape[0]:
                clash = m["v"] <= radius[first_id + m["i"]] + rb[m["j"]]
                ok[m["j"][clash]] = False
        # inside the batch, in order: a candidate is dropped if it overlaps an
        # earlier candidate of the batch that is still accepted
        pairs = ctree.query_pairs(2 * rmax, output_type="ndarray")
        if pairs.shape[0]:
            a, b = pairs.min(axis=1), pairs.max(axis=1)
            dd = np.sqrt(np.sum((cand[a] - cand[b]) ** 2, axis=1))
            keep = (dd <= rb[a] + rb[b]) | (sid[a] == sid[b])
            a, b = a[keep], b[keep]
            for p in np.argsort(b, kind="stable"):
                if ok[a[p]]:
                    ok[b[p]] = False
        # the first surviving copy of each sphere is placed
        first = np.full(batch, -1)
        cand_ok = np.nonzero(ok)[0]
        u, at = np.unique(sid[cand_ok], return_index=True)
        first[u] = cand_ok[at]
        acc = np.nonzero(first >= 0)[0]
        rej = np.nonzero(first < 0)[0]
        r_here = radius[placed:placed + batch].copy()
        radius[placed:placed + batch] = np.concatenate([r_here[acc], r_here[rej]])
        pts[placed:placed + acc.shape[0]] = cand[first[acc]]
        placed += acc.shape[0]
        if placed - old_n > max(old_n // 5, 50000):
            old_n = placed
            old_tree = cKDTree(pts[:old_n])
        trees = [(0, old_tree)] if old_n else []
        if placed > old_n:
            trees.append((old_n, cKDTree(pts[old_n:placed])))
    return pts.T.copy()


def jittered_lattice(rng, n, d, lo, hi, solid_fraction):
    """Simple-cubic lattice of spacing s = d (pi/(6 phi))^(1/3) filled layer by
    layer from the floor, each centre jittered uniformly by +-0.4999 (s - d) per
    axis (no initial overlap)."""
    s = d * (math.pi / (6.0 * solid_fraction)) ** (1.0 / 3.0)
    nx = int((hi[0] - lo[0]) // s)
    ny = int((hi[1] - lo[1]) // s)
    per_layer = nx * ny
    layers = -(-n // per_layer)
    if lo[2] + layers * s > hi[2]:
        raise ValueError("lattice does not fit the box")
    k = np.arange(n)
    ix = k % nx
    iy = (k // nx) % ny
    iz = k // per_layer
    off_x = lo[0] + 0.5 * ((hi[0] - lo[0]) - nx * s)
    off_y = lo[1] + 0.5 * ((hi[1] - lo[1]) - ny * s)
    x = np.stack([off_x + (ix + 0.5) * s, off_y + (iy + 0.5) * s, lo[2] + (iz + 0.5) * s])
    jit = 0.4999 * (s - d)
    x += rng.uniform(-jit, jit, size=x.shape)
    return x


def plain(n=2000, seed_index=0) -> Workload:
    """2,000 monodisperse spheres, d = 3 mm, rho = 2500 (FP64 correctness config)."""
    rng = rng_for(1, seed_index)
    d = 3e-3
    lo, hi = [0.0, 0.0, 0.0], [0.05, 0.05, 0.2]
    x = rsa_monodisperse(rng, n, d, lo, hi)
    v = rng.normal(0.0, 0.01, size=(3, n))
    fluid = dict(order=2, n_el=[4, 4, 16], rho_f=1.2, mu_f=1.8e-5, model=0, eps_min=0.1)
    nodes = node_grid(lo, hi, fluid["n_el"], 2)
    U = np.zeros((3, nodes.shape[1]))
    U[2] = 0.5
    P = np.zeros(node_grid(lo, hi, fluid["n_el"], 1).shape[1])
    dem = dict(box_lo=lo, box_hi=hi, gravity=[0.0, 0.0, -G], dt=1e-5, **_material())
    return Workload("plain", x, v, np.zeros((3, n)), np.full(n, 0.5 * d), np.full(n, 2500.0), dem,
                    fluid, dict(steps=100, coupling_every=10, precision="fp64"), U, P)


def lattice(n_side=(12, 12, 14), spacing_factor=0.98, seed_index=0, d=3e-3) -> Workload:
    """Plain-config spheres on a simple-cubic lattice of spacing 0.98 d, small
    random velocities and spins; every lattice neighbour overlaps by 2 %."""
    rng = rng_for(1, 100 + seed_index)
    s = spacing_factor * d
    nx, ny, nz = n_side
    lo = [0.0, 0.0, 0.0]
    hi = [nx * s + 0.01, ny * s + 0.01, nz * s + 0.02]
    k = np.arange(nx * ny * nz)
    x = np.stack([0.005 + (k % nx + 0.5) * s, 0.005 + ((k // nx) % ny + 0.5) * s,
                  0.5 * d + (k // (nx * ny)) * s])
    x += rng.uniform(-0.002 * d, 0.002 * d, size=x.shape)
    n = x.shape[1]
    v = rng.normal(0.0, 0.01, size=(3, n))
    w = rng.normal(0.0, 5.0, size=(3, n))
    # mesh: elements of ~4 d
    n_el = [max(1, int((hi[a] - lo[a]) // (4 * d))) for a in range(3)]
    fluid = dict(order=2, n_el=n_el, rho_f=1.2, mu_f=1.8e-5, model=0, eps_min=0.1)
    nodes = node_grid(lo, hi, n_el, 2)
    U = np.zeros((3, nodes.shape[1]))
    U[2] = 0.5 + 0.05 * rng.standard_normal(nodes.shape[1])
    P = 100.0 * (1.0 - node_grid(lo, hi, n_el, 1)[2] / hi[2])
    dem = dict(box_lo=lo, box_hi=hi, gravity=[0.0, 0.0, -G], dt=1e-5, **_material())
    return Workload("lattice", x, v, w, np.full(n, 0.5 * d), np.full(n, 2500.0), dem, fluid,
                    dict(steps=20, coupling_every=10, precision="fp64"), U, P)


def on_faces(seed_index=0) -> Workload:
    """Spheres of d = 3 mm centred on cell, element and box faces.

    Box 0.0625 x 0.0625 x 0.125 m with 4 x 4 x 8 elements: with the default
    skin (0.1 d) the contact cells are 2^-8 m wide, so every multiple of
    2^-8 is a cell face and sits exactly in binary.  Sites every two cells
    along each axis, from one box face to the other (the outermost centred
    on the walls, overlapping them by a radius); a third of the sites moved
    one ulp down on each axis (just below a face); half of the sites with a
    partner 0.98 d up along a random axis that does not leave the box, so
    that touching pairs straddle faces or sit on them.  Any two spheres other
    than a site and its partner are at least 4.8 mm apart."""
    rng = rng_for(1, 200 + seed_index)
    d = 3e-3
    h = 2.0 ** -8
    lo, hi = [0.0, 0.0, 0.0], [0.0625, 0.0625, 0.125]
    ns = [int(round((hi[a] - lo[a]) / (2 * h))) + 1 for a in range(3)]
    k = np.arange(ns[0] * ns[1] * ns[2])
    idx = np.stack([k % ns[0], (k // ns[0]) % ns[1], k // (ns[0] * ns[1])])
    sites = idx * (2 * h)
    down = rng.random(sites.shape[1]) < 1.0 / 3.0
    for a in range(3):
        moved = down & (sites[a] > lo[a])
        sites[a, moved] = np.nextafter(sites[a, moved], -np.inf)
    pick = rng.random(sites.shape[1]) < 0.5
    axis = rng.integers(0, 3, size=sites.shape[1])
    part = []
    for i in np.flatnonzero(pick):
        # up along the drawn axis, or the next one off the upper box face (a
        # site on the upper face of all three axes gets no partner)
        for t in range(3):
            a = (axis[i] + t) % 3
            if idx[a, i] < ns[a] - 1:
                q = sites[:, i].copy()
                q[a] += 0.98 * d
                part.append(q)
                break
    x = np.concatenate([sites, np.array(part).T], axis=1)
    n = x.shape[1]
    v = rng.normal(0.0, 0.01, size=(3, n))
    w = rng.normal(0.0, 5.0, size=(3, n))
    n_el = [4, 4, 8]
    fluid = dict(order=2, n_el=n_el, rho_f=1.2, mu_f=1.8e-5, model=0, eps_min=0.1)
    nodes = node_grid(lo, hi, n_el, 2)
    U = np.zeros((3, nodes.shape[1]))
    U[2] = 0.5 + 0.05 * rng.standard_normal(nodes.shape[1])
    P = np.zeros(node_grid(lo, hi, n_el, 1).shape[1])
    dem = dict(box_lo=lo, box_hi=hi, gravity=[0.0, 0.0, -G], dt=1e-5, **_material())
    return Workload("on_faces", x, v, w, np.full(n, 0.5 * d), np.full(n, 2500.0), dem, fluid,
                    dict(steps=3, coupling_every=10, precision="fp64"), U, P)


def fluidized(n=100_000, seed_index=0, height=0.4) -> Workload:
    """100,000 spheres, d = 1 mm, rho = 2500, jittered lattice at solid fraction
    0.4; Q2 20x20x80; U = (0,0,1.2) + N(0,0.05) per node; linear pressure."""
    rng = rng_for(2, seed_index)
    d = 1e-3
    lo, hi = [0.0, 0.0, 0.0], [0.1, 0.1, height]
    x = jittered_lattice(rng, n, d, lo, hi, 0.4)
    v = rng.normal(0.0, 0.01, size=(3, n))
    n_el = [20, 20, int(round(80 * height / 0.4))]
    fluid = dict(order=2, n_el=n_el, rho_f=1.2, mu_f=1.8e-5, model=0, eps_min=0.1)
    nodes = node_grid(lo, hi, n_el, 2)
    U = rng.normal(0.0, 0.05, size=(3, nodes.shape[1]))
    U[2] += 1.2
    # pressure drop equal to the buoyant weight of the bed over the cross-section
    vp = math.pi / 6.0 * d ** 3
    area = (hi[0] - lo[0]) * (hi[1] - lo[1])
    dp = n * vp * (2500.0 - fluid["rho_f"]) * G / area
    P = dp * (1.0 - node_grid(lo, hi, n_el, 1)[2] / hi[2])
    dem = dict(box_lo=lo, box_hi=hi, gravity=[0.0, 0.0, -G], dt=1e-5, **_material())
    return Workload("fluidized", x, v, np.zeros((3, n)), np.full(n, 0.5 * d), np.full(n, 2500.0), dem,
                    fluid, dict(steps=1000, coupling_every=10, precision="fp32"), U, P)


def spouted(n=500_000, seed_index=0, box=(0.15, 0.15, 0.6), fill_height=0.45, n_el=(30, 30, 120)) -> Workload:
    """500,000 polydisperse spheres (lognormal d, median 2 mm, sigma 0.2,
    clipped to [1, 4] mm), rho = 2500; Q2 mesh; Gaussian jet."""
    rng = rng_for(3, seed_index)
    d = np.exp(rng.normal(math.log(2e-3), 0.2, size=n))
    d = np.clip(d, 1e-3, 4e-3)
    radius = 0.5 * d
    lo, hi = [0.0, 0.0, 0.0], list(box)
    x = rsa_polydisperse(rng, radius, lo, [hi[0], hi[1], fill_height])
    perm = rng.permutation(n)  # particle IDs independent of size
    x = x[:, perm].copy()
    radius = radius[perm].copy()
    v = rng.normal(0.0, 0.01, size=(3, n))
    fluid = dict(order=2, n_el=list(n_el), rho_f=1.2, mu_f=1.8e-5, model=0, eps_min=0.1)
    nodes = node_grid(lo, hi, fluid["n_el"], 2)
    cx, cy = 0.5 * hi[0], 0.5 * hi[1]
    rr = (nodes[0] - cx) ** 2 + (nodes[1] - cy) ** 2
    U = np.zeros((3, nodes.shape[1]))
    U[2] = 20.0 * np.exp(-rr / (2 * 0.01 ** 2)) * np.exp(-nodes[2] / 0.2)
    P = np.zeros(node_grid(lo, hi, fluid["n_el"], 1).shape[1])
    dem = dict(box_lo=lo, box_hi=hi, gravity=[0.0, 0.0, -G], dt=1e-5, **_material())
    return Workload("spouted", x, v, np.zeros((3, n)), radius, np.full(n, 2500.0), dem, fluid,
                    dict(steps=500, coupling_every=10, precision="fp32"), U, P)


def filling(n=100_000, d=1e-3, seed_index=0, width=0.1, height=0.4, solid_fraction=0.15, e=0.9) -> Workload:
    """DEM-only filling of a square column (stand-in for the bed preparation
    that precedes each coupled case of the paper, Sections 3.2 and 3.3): n
    spheres of diameter d, rho = 2500, placed at random (random sequential
    addition) at solid fraction `solid_fraction` in a layer that starts 2 d
    above the floor, at rest, under gravity, to be stepped without coupling
    until the bed is at rest.  The mesh (Q1, elements of about 5 d) only hosts
    the cell grid; the fluid field is zero."""
    rng = rng_for(6, seed_index)
    vp = math.pi / 6.0 * d ** 3
    layer = n * vp / (solid_fraction * width * width)
    if 2.0 * d + layer > height:
        raise ValueError("the insertion layer does not fit in the column")
    radius = np.full(n, 0.5 * d)
    x = rsa_polydisperse(rng, radius, [0.0, 0.0, 2.0 * d], [width, width, 2.0 * d + layer])
    x = x[:, rng.permutation(n)].copy()
    lo, hi = [0.0, 0.0, 0.0], [width, width, height]
    m = max(1, int(round(width / (5.0 * d))))
    h = width / m
    n_el = [m, m, max(1, int(round(height / h)))]
    fluid = dict(order=1, n_el=n_el, rho_f=1.2, mu_f=1.8e-5, model=0, eps_min=0.1)
    nodes = node_grid(lo, hi, n_el, 1)
    U = np.zeros((3, nodes.shape[1]))
    P = np.zeros(nodes.shape[1])
    dem = dict(box_lo=lo, box_hi=hi, gravity=[0.0, 0.0, -G], dt=1e-5, **_material(e=e))
    return Workload("filling", x, np.zeros((3, n)), np.zeros((3, n)), np.full(n, 0.5 * d), np.full(n, 2500.0),
                    dem, fluid, dict(steps=0, coupling_every=0, precision="fp32"), U, P)


def column_bed(rng, n, d, e, u_in, name="column", precision="fp32", steps=1000, rho=2500.0) -> Workload:
    """A bed of the batched and served workloads: n spheres of diameter d in a
    square column of width W = (n V_p / (0.4 * 2))^(1/3) (a packed height of
    2 W at solid fraction 0.4) and height 4 W, packed as the fluidized bed
    (jittered simple-cubic lattice); restitution e for particle-particle and
    particle-wall contacts; Q1 mesh of h = W / round(W / (4 d)).  u_in > 0:
    fluidization, U = (0, 0, u_in) + N(0, 0.05) per node and the linear
    pressure carrying the bed's buoyant weight (Eq. "dpf"); u_in == 0:
    sedimentation in still fluid (U = 0, P = 0)."""
    vp = math.pi / 6.0 * d ** 3
    W = (n * vp / 0.8) ** (1.0 / 3.0)
    lo, hi = [0.0, 0.0, 0.0], [W, W, 4.0 * W]
    x = jittered_lattice(rng, n, d, lo, hi, 0.4)
    v = rng.normal(0.0, 0.01, size=(3, n))
    m = max(1, int(round(W / (4.0 * d))))
    n_el = [m, m, 4 * m]
    fluid = dict(order=1, n_el=n_el, rho_f=1.2, mu_f=1.8e-5, model=0, eps_min=0.1)
    nodes = node_grid(lo, hi, n_el, 1)
    if u_in > 0.0:
        U = rng.normal(0.0, 0.05, size=(3, nodes.shape[1]))
        U[2] += u_in
        dp = n * vp * (rho - fluid["rho_f"]) * G / (W * W)
        P = dp * (1.0 - nodes[2] / hi[2])
    else:
        U = np.zeros((3, nodes.shape[1]))
        P = np.zeros(nodes.shape[1])
    dem = dict(box_lo=lo, box_hi=hi, gravity=[0.0, 0.0, -G], dt=1e-5, **_material(e=e))
    return Workload(name, x, v, np.zeros((3, n)), np.full(n, 0.5 * d), np.full(n, rho), dem, fluid,
                    dict(steps=steps, coupling_every=10, precision=precision), U, P)


def batched_bed(index: int) -> Workload:
    """Bed `index` of the batched ensemble: n ~ U{5k..80k}, d ~ U[1, 3] mm,
    e ~ U[0.7, 0.95], inlet velocity ~ U[0.5, 2] m/s, 1,000 steps."""
    rng = rng_for(4, index)
    n = int(rng.integers(5_000, 80_001))
    d = float(rng.uniform(1e-3, 3e-3))
    e = float(rng.uniform(0.7, 0.95))
    u_in = float(rng.uniform(0.5, 2.0))
    return column_bed(rng, n, d, e, u_in, name=f"batched{index}")


def batched(n_beds: int = 64):
    """The batched ensemble: n_beds independent beds (see batched_bed)."""
    return [batched_bed(b) for b in range(n_beds)]


@dataclass
class Job:
    index: int
    arrival: float   # s after the start of the stream
    kind: str        # "sedimentation" | "fluidization"
    n: int
    steps: int       # a multiple of the coupling period (10 DEM steps)

    def workload(self) -> Workload:
        rng = rng_for(5, self.index)
        rng.random(3)  # the draws that fixed kind, n and steps
        d = float(rng.uniform(1e-3, 3e-3))
        e = float(rng.uniform(0.7, 0.95))
        u_in = float(rng.uniform(0.5, 2.0)) if self.kind == "fluidization" else 0.0
        return column_bed(rng, self.n, d, e, u_in, name=f"job{self.index}", steps=self.steps)


def job_stream(n_jobs: int, rate: float = 20.0, n_min: int = 1_000, n_max: int = 200_000):
    """The served stream: Poisson arrivals at `rate` jobs/s; each job is a
    sedimentation or fluidization bed (50/50) of n log-uniform in
    [n_min, n_max] spheres run for U{200..2000} steps rounded up to whole
    coupling periods.  Geometry and parameters are drawn per job as in the
    batched ensemble."""
    arr = rng_for(5, 100_000)
    t = np.cumsum(arr.exponential(1.0 / rate, size=n_jobs))
    jobs = []
    for j in range(n_jobs):
        rng = rng_for(5, j)
        u = rng.random(3)
        kind = "sedimentation" if u[0] < 0.5 else "fluidization"
        n = int(round(math.exp(math.log(n_min) + u[1] * (math.log(n_max) - math.log(n_min)))))
        steps = 200 + int(u[2] * 1801)
        steps = 10 * ((steps + 9) // 10)
        jobs.append(Job(j, float(t[j]), kind, n, steps))
    return jobs


WORKLOADS = {"plain": plain, "lattice": lattice, "fluidized": fluidized, "spouted": spouted}

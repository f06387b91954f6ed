"""DEM-only filling and settling of a bed.

The paper prepares every bed with DEM alone before a coupled run: particles
inserted at random in the vessel fall under gravity until their kinetic
energy has dissipated (Sections 3.2 and 3.3).  ``settle`` runs DEM steps on a
bed (no coupling step, so no fluid force) in chunks and checks the kinetic
energy between chunks (dem_kinetic_energy, a deterministic device
reduction), until it falls below a fraction of the bed's potential-energy
scale sum(m g d): the bed is then at rest.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class SettleResult:
    steps: int
    kinetic: float            # translational + rotational kinetic energy at the end
    at_rest: bool
    wall_s: float
    history: list = field(default_factory=list)  # (steps, kinetic energy) after each chunk


def energy_scale(wl) -> float:
    """sum over particles of m |g| d (J): the kinetic energy of a particle
    that fell through one diameter, summed."""
    g = float(np.linalg.norm(wl.dem["gravity"]))
    d = 2.0 * wl.radius
    m = wl.density * math.pi / 6.0 * d ** 3
    return float(np.sum(m * g * d))


def settle(bed, scale: float, rest: float = 1e-4, every: int = 500, max_steps: int = 200_000) -> SettleResult:
    """Step `bed` (no coupling) until its kinetic energy is at most
    rest * scale, checking every `every` steps, or until max_steps."""
    steps = 0
    kin = float("inf")
    hist = []
    t0 = time.perf_counter()
    while steps < max_steps:
        k = min(every, max_steps - steps)
        bed.step(k)
        steps += k
        et, er = bed.kinetic_energy()
        kin = et + er
        hist.append((steps, kin))
        if kin <= rest * scale:
            return SettleResult(steps, kin, True, time.perf_counter() - t0, hist)
    return SettleResult(steps, kin, False, time.perf_counter() - t0, hist)

"""Born-Oppenheimer molecular dynamics driven through the C ABI.

Each ionic step follows the paper's coupling (Sec. I flow chart, Sec. V C):
new ion positions in, density re-minimised from the previous density (warm
start), free energy and forces out, velocity-Verlet update of the ions.
Energy conservation is monitored with E_cons = sum M v^2/2 + F_tot (the
"Ekin + Etot" of the paper's output block).
"""
from __future__ import annotations

import dataclasses
import time
from typing import List

import numpy as np

from .binding import Context

AMU_ME = 1822.888486209          # unified atomic mass unit / electron mass (CODATA 2018)
H_MASS_ME = 1.00794 * AMU_ME
KB_HA = 3.1668115634556e-6       # hartree per kelvin
FS_AU = 41.341373335             # atomic time units per femtosecond


@dataclasses.dataclass
class MDRecord:
    step: int
    F_total: float
    kinetic: float
    iterations: int
    evaluations: int
    wall_ms: float


def maxwell_boltzmann(nat: int, T_K: float, mass: float, seed: int) -> np.ndarray:
    """Seeded Maxwell-Boltzmann velocities at T, centre-of-mass motion removed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.normal(0.0, np.sqrt(KB_HA * T_K / mass), size=(nat, 3))
    return v - v.mean(axis=0)


def step_forces(ctx: Context, positions: np.ndarray, charges: np.ndarray):
    ctx.set_ions(positions, charges)
    rep = ctx.minimize_density()
    F, _, forces = ctx.free_energy_and_forces(forces=True)
    return F, forces, rep


def velocity_verlet(ctx: Context, positions, velocities, charges, masses, dt: float, n_steps: int,
                    callback=None) -> List[MDRecord]:
    x = np.array(positions, dtype=np.float64)
    v = np.array(velocities, dtype=np.float64)
    m = np.asarray(masses, dtype=np.float64)[:, None]
    t0 = time.perf_counter()
    F, f, rep = step_forces(ctx, x, charges)
    recs = [MDRecord(0, F, float(0.5 * np.sum(m * v * v)), rep.iterations, rep.evaluations,
                     1e3 * (time.perf_counter() - t0))]
    for k in range(1, n_steps + 1):
        t0 = time.perf_counter()
        v += 0.5 * dt * f / m
        x += dt * v
        F, f, rep = step_forces(ctx, x, charges)
        v += 0.5 * dt * f / m
        rec = MDRecord(k, F, float(0.5 * np.sum(m * v * v)), rep.iterations, rep.evaluations,
                       1e3 * (time.perf_counter() - t0))
        recs.append(rec)
        if callback:
            callback(rec, x, v, f)
    return recs

"""Born-Oppenheimer velocity-Verlet dynamics on the finite-T free-energy surface.

TEST INFRASTRUCTURE (oracle).

Each ionic step re-minimises the electronic free energy (warm-started from the
previous density) and takes the forces of Eq. M12, as in the paper's MD flow
(Sec. I figure, Sec. V D).  The conserved quantity is
E_cons = sum_I M_I v_I^2 / 2 + F_tot (the paper prints Ekin + Etot, Sec. V D).
"""
from __future__ import annotations

import dataclasses
from typing import Callable

import numpy as np

AMU_ME = 1822.888486209           # unified atomic mass unit in electron masses (CODATA 2018)
H_MASS_ME = 1.00794 * AMU_ME


@dataclasses.dataclass
class MDFrame:
    step: int
    positions: np.ndarray
    velocities: np.ndarray
    F_tot: float
    kinetic: float
    forces: np.ndarray


def velocity_verlet(positions, velocities, masses, dt, n_steps,
                    energy_forces: Callable, callback=None):
    """energy_forces(positions) -> (F_tot, forces); returns the list of frames."""
    x = np.array(positions, dtype=np.float64)
    v = np.array(velocities, dtype=np.float64)
    m = np.asarray(masses, dtype=np.float64)[:, None]
    E, F = energy_forces(x)
    frames = [MDFrame(0, x.copy(), v.copy(), E, float(0.5 * np.sum(m * v * v)), F.copy())]
    for step in range(1, n_steps + 1):
        v += 0.5 * dt * F / m
        x += dt * v
        E, F = energy_forces(x)
        v += 0.5 * dt * F / m
        fr = MDFrame(step, x.copy(), v.copy(), E, float(0.5 * np.sum(m * v * v)), F.copy())
        frames.append(fr)
        if callback:
            callback(fr)
    return frames

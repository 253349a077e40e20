"""Born-Oppenheimer molecular dynamics driven through the C ABI.

Each ionic step follows the paper's coupling (Sec. I flow chart, Sec. V D):
new ion positions in, density re-minimised from the previous density (warm
start), free energy and forces out, velocity-Verlet update of the ions.
Energy conservation is monitored with E_cons = sum M v^2/2 + F_tot (the
"Ekin + Etot" of the paper's output block).  NVT runs use an Andersen
thermostat (as the paper's AIMD runs do, Sec. VI): after each step every ion,
with probability 1 - exp(-nu dt), draws a new velocity from the
Maxwell-Boltzmann distribution at the ion temperature (Andersen, J. Chem.
Phys. 72, 2384 (1980)).  output_block() prints the per-step energies in the
layout of the paper's output sample (Sec. V D), write_xyz() the trajectory (md.xyz).
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional, Sequence

import numpy as np

from .binding import Context

AMU_ME = 1822.888486209          # unified atomic mass unit / electron mass (CODATA 2018)
H_MASS_ME = 1.00794 * AMU_ME
KB_HA = 3.1668115634556e-6       # hartree per kelvin
FS_AU = 41.341373335             # atomic time units per femtosecond
BOHR_ANGSTROM = 0.529177210903


@dataclasses.dataclass
class MDRecord:
    step: int
    F_total: float
    kinetic: float
    iterations: int
    evaluations: int
    wall_ms: float
    E_internal: float = 0.0      # F_tot + T S_s + T S_xc (EinternEl)
    TS: float = 0.0              # T S = T S_s + T S_xc
    E_xc: float = 0.0            # XC free energy F_xc
    TS_xc: float = 0.0           # T S_xc (KSDT; 0 for the T-independent PZ81)
    T_ion: float = 0.0           # kelvin, from the kinetic energy
    pressure: Optional[float] = None   # hartree/bohr^3 (electrons + ions' potential part)


@dataclasses.dataclass
class Thermostat:
    """Andersen thermostat: collision rate nu (per atomic time unit) at T_K kelvin."""
    T_K: float
    nu: float
    seed: int = 0


def maxwell_boltzmann(nat: int, T_K: float, mass: float, seed: int) -> np.ndarray:
    """Seeded Maxwell-Boltzmann velocities at T, centre-of-mass motion removed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.normal(0.0, np.sqrt(KB_HA * T_K / mass), size=(nat, 3))
    return v - v.mean(axis=0)


def andersen(v: np.ndarray, masses: np.ndarray, T_K: float, nu: float, dt: float,
             rng: np.random.Generator) -> int:
    """Andersen collisions in place: each ion with probability 1 - exp(-nu dt) gets a new
    Maxwell-Boltzmann velocity at T_K.  Returns the number of collisions."""
    hit = rng.random(v.shape[0]) < -np.expm1(-nu * dt)
    k = int(np.count_nonzero(hit))
    if k:
        sd = np.sqrt(KB_HA * T_K / np.asarray(masses, dtype=np.float64)[hit])
        v[hit] = rng.normal(0.0, 1.0, size=(k, 3)) * sd[:, None]
    return k


def ion_temperature(v: np.ndarray, masses) -> float:
    m = np.asarray(masses, dtype=np.float64)[:, None]
    return float(np.sum(m * v * v)) / (3.0 * v.shape[0] * KB_HA)


def step_forces(ctx: Context, positions: np.ndarray, charges: np.ndarray):
    ctx.set_ions(positions, charges)
    rep = ctx.minimize_density()
    F, _, forces = ctx.free_energy_and_forces(forces=True)
    return F, forces, rep


def velocity_verlet(ctx: Context, positions, velocities, charges, masses, dt: float, n_steps: int,
                    callback=None, thermostat: Optional[Thermostat] = None, pressure: bool = False,
                    step: Optional[Callable] = None) -> List[MDRecord]:
    """n_steps of velocity Verlet.  step(x) -> (F, forces, report) replaces the library call
    (step_forces) when given; pressure=True also evaluates ofdft_stress every step."""
    x = np.array(positions, dtype=np.float64)
    v = np.array(velocities, dtype=np.float64)
    m = np.asarray(masses, dtype=np.float64)[:, None]
    rng = np.random.Generator(np.random.PCG64(thermostat.seed)) if thermostat else None
    run = step if step is not None else (lambda xx: step_forces(ctx, xx, charges))

    def record(k, F, rep, t0):
        P = ctx.pressure() if (pressure and step is None) else None
        return MDRecord(k, F, float(0.5 * np.sum(m * v * v)), rep.iterations, rep.evaluations,
                        1e3 * (time.perf_counter() - t0), E_internal=getattr(rep, "E_internal", 0.0),
                        TS=getattr(rep, "TS_s", 0.0) + getattr(rep, "TS_xc", 0.0), E_xc=getattr(rep, "E_xc", 0.0),
                        TS_xc=getattr(rep, "TS_xc", 0.0),
                        T_ion=ion_temperature(v, masses), pressure=P)

    t0 = time.perf_counter()
    F, f, rep = run(x)
    recs = [record(0, F, rep, t0)]
    for k in range(1, n_steps + 1):
        t0 = time.perf_counter()
        v += 0.5 * dt * f / m
        x += dt * v
        F, f, rep = run(x)
        v += 0.5 * dt * f / m
        if thermostat:
            andersen(v, masses, thermostat.T_K, thermostat.nu, dt, rng)
        rec = record(k, F, rep, t0)
        recs.append(rec)
        if callback:
            callback(rec, x, v, f)
    return recs


def output_block(rec: MDRecord) -> str:
    """The per-step energy block of the paper's output sample (Sec. V D), in hartree.  Fxc is
    the XC free energy and Exc = Fxc + T S_xc its internal energy (equal for the T-independent
    PZ81, different for KSDT)."""
    lines = [f"     MD step {rec.step}"]
    if rec.pressure is not None:
        lines.append(f"     P          = {rec.pressure:20.10f} Ha/bohr^3")
    lines += [
        f"     Fxc        = {rec.E_xc:20.10f} Ha",
        f"     Exc        = {rec.E_xc + rec.TS_xc:20.10f} Ha",
        f"     Ekin       = {rec.kinetic:20.10f} Ha",
        f"     T_ion      = {rec.T_ion:20.4f} K",
        f"     Ekin+Etot  = {rec.kinetic + rec.F_total:20.10f} Ha",
        f"     Etot       = {rec.F_total:20.10f} Ha",
        f"     EinternEl  = {rec.E_internal:20.10f} Ha",
        f"     Eint       = {rec.kinetic + rec.E_internal:20.10f} Ha",
        f"     -TS        = {-rec.TS:20.10f} Ha",
    ]
    return "\n".join(lines)


def write_xyz(path: str, frames: Sequence, symbols: Sequence[str]) -> None:
    """Trajectory in XYZ format (angstrom): frames = [(step, positions_bohr, F_total), ...]."""
    with open(path, "w") as fh:
        for step, pos, F in frames:
            pos = np.asarray(pos)
            fh.write(f"{len(symbols)}\nstep {step} Etot {F:.10f} Ha\n")
            for s, r in zip(symbols, pos * BOHR_ANGSTROM):
                fh.write(f"{s} {r[0]:.8f} {r[1]:.8f} {r[2]:.8f}\n")

"""Seeded synthetic inputs for the finite-temperature orbital-free DFT hot path.

This module is shared by the CPU oracle tests and the HIP path tests/benchmarks.
It holds no part of the method's arithmetic: only geometry of random hydrogen
cells (cell size from a mass density, random sequential addition of ions with a
minimum-image separation), smooth positive trial amplitudes phi on a grid, and
the draw of a heterogeneous batch of cells.  Every generator takes an explicit
seed and uses numpy's PCG64.

Workloads follow the paper's hydrogen AIMD setting (Sec. VI: 128 H atoms,
~1 g/cm^3, 64^3 grid, temperatures from 2 kK to 4 MK) and the sizes of the
benchmark configurations built on it.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Unit constants (CODATA 2018) used only to turn a mass density into a cell edge.
AMU_G = 1.66053906660e-24          # g
BOHR_CM = 0.529177210903e-8        # cm
H_MASS_AMU = 1.00794               # hydrogen standard atomic weight

SEED_BASE = 1406 * 100


@dataclasses.dataclass
class HCell:
    """A cubic periodic cell of hydrogen ions (Z = 1)."""
    lattice: np.ndarray      # (3,3) rows a1, a2, a3 in bohr
    positions: np.ndarray    # (nat,3) Cartesian bohr
    charges: np.ndarray      # (nat,) valence charges
    grid: Tuple[int, int, int]
    temperature_K: float
    rho_gcc: float
    seed: int

    @property
    def nat(self) -> int:
        return int(self.positions.shape[0])

    @property
    def edge(self) -> float:
        return float(self.lattice[0, 0])


def cubic_edge_bohr(n_atoms: int, rho_gcc: float, mass_amu: float = H_MASS_AMU) -> float:
    """Edge (bohr) of the cubic cell holding n_atoms of the given mass at rho (g/cm^3)."""
    vol_cm3 = n_atoms * mass_amu * AMU_G / rho_gcc
    return (vol_cm3 / BOHR_CM ** 3) ** (1.0 / 3.0)


def random_positions(n_atoms: int, edge: float, rng: np.random.Generator,
                     min_sep: float = 0.8, max_tries: int = 200000) -> np.ndarray:
    """Random sequential addition in a cubic box with a minimum-image separation."""
    pos = np.empty((n_atoms, 3))
    placed = 0
    tries = 0
    while placed < n_atoms:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place ions at the requested separation")
        cand = rng.random(3) * edge
        if placed:
            d = pos[:placed] - cand
            d -= edge * np.round(d / edge)
            if np.min(np.einsum("ij,ij->i", d, d)) < min_sep * min_sep:
                continue
        pos[placed] = cand
        placed += 1
    return pos


def h_cell(n_atoms: int, rho_gcc: float, grid, temperature_K: float,
           seed: int, min_sep: float = 0.8) -> HCell:
    """A seeded random hydrogen cell."""
    if isinstance(grid, int):
        grid = (grid, grid, grid)
    edge = cubic_edge_bohr(n_atoms, rho_gcc)
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = random_positions(n_atoms, edge, rng, min_sep)
    return HCell(lattice=np.eye(3) * edge, positions=pos,
                 charges=np.ones(n_atoms), grid=tuple(int(g) for g in grid),
                 temperature_K=float(temperature_K), rho_gcc=float(rho_gcc), seed=seed)


def h_cell_spaced(shape, seed: int, spacing: float = 0.15, rho_gcc: float = 1.0,
                  temperature_K: float = 5.0e4) -> HCell:
    """A seeded hydrogen cell on an orthorhombic box with the same grid spacing (bohr) along
    every axis, for grids whose axes differ in length: the atom count follows from rho."""
    lengths = np.array(shape, dtype=float) * spacing
    n_per_bohr3 = rho_gcc / 1.00794 * 6.02214076e23 * (0.529177210903e-8) ** 3
    nat = max(2, int(round(n_per_bohr3 * float(np.prod(lengths)))))
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.random((nat, 3)) * lengths
    return HCell(lattice=np.diag(lengths), positions=pos, charges=np.ones(nat),
                 grid=tuple(int(g) for g in shape), temperature_K=float(temperature_K),
                 rho_gcc=float(rho_gcc), seed=seed)


# The five benchmark workloads (seed = SEED_BASE + index).
def small_tf_cell() -> HCell:
    """16 H, 1.0 g/cm^3, 32^3, 10 kK (plain FP64 ftTF minimization)."""
    return h_cell(16, 1.0, 32, 1.0e4, SEED_BASE + 0)


def gga_64_cell(temperature_K: float = 5.0e4) -> HCell:
    """128 H, 2.0 g/cm^3, 64^3; temperatures 2 kK, 50 kK, 1 MK."""
    return h_cell(128, 2.0, 64, temperature_K, SEED_BASE + 1)


def gga_128_cell(temperature_K: float = 1.0e5) -> HCell:
    """1024 H, 4.0 g/cm^3, 128^3; temperatures 100 kK, 4 MK."""
    return h_cell(1024, 4.0, 128, temperature_K, SEED_BASE + 2)


def batch_cells(n_cells: int = 64, seed: int = SEED_BASE + 3,
                grids: Sequence[int] = (32, 48, 64, 96)) -> List[HCell]:
    """Heterogeneous batch: 16-256 atoms, grid in grids, rho U[0.5,5], T log-U[2e3,4e6] K."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cells = []
    for c in range(n_cells):
        nat = int(rng.integers(16, 257))
        g = int(rng.choice(np.asarray(grids)))
        rho = float(rng.uniform(0.5, 5.0))
        T = float(math.exp(rng.uniform(math.log(2.0e3), math.log(4.0e6))))
        cells.append(h_cell(nat, rho, g, T, seed * 1000 + c))
    return cells


def md_cell() -> HCell:
    """128 H, 1.0 g/cm^3, 64^3, 50 kK (MD trajectory start)."""
    return h_cell(128, 1.0, 64, 5.0e4, SEED_BASE + 4)


AL_MASS_AMU = 26.9815385
# Heine-Abarenkov local pseudopotential of Al (parameters quoted in the paper's
# pseudopotential section, Eq. E4A): r_c (bohr), A (hartree), q_c (1/bohr)
AL_HA_LPP = {"kind": "ha", "rc": 1.15, "A": 0.1107, "qc": 3.5}


def fcc_al_cell(n_rep: int, grid, temperature_K: float = 100.0, rho_gcc: float = 2.70) -> HCell:
    """fcc aluminium (Z = 3 valence electrons per ion), n_rep^3 conventional cells of four
    ions at rho (the static scaling workload: 2.70 g/cm^3, 100 K, 2048 ions for n_rep = 8)."""
    if isinstance(grid, int):
        grid = (grid, grid, grid)
    a = cubic_edge_bohr(4, rho_gcc, AL_MASS_AMU)
    basis = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    cells = np.array([[i, j, k] for i in range(n_rep) for j in range(n_rep) for k in range(n_rep)], dtype=float)
    pos = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    nat = pos.shape[0]
    return HCell(lattice=np.eye(3) * a * n_rep, positions=pos, charges=np.full(nat, 3.0),
                 grid=tuple(int(g) for g in grid), temperature_K=float(temperature_K), rho_gcc=float(rho_gcc),
                 seed=0)


def fcc_symmetrize(a: np.ndarray) -> np.ndarray:
    """Project a field on the grid of ONE conventional fcc cell (ions at the origin and the
    face centres, even grid) onto the fields with the lattice's symmetry: the average over
    the three face-centring translations and the inversion through the ion at the origin
    (grid index i -> -i mod n).  A geometric helper for checks at the symmetric density."""
    if a.ndim != 3 or any(m % 2 for m in a.shape):
        raise ValueError("a 3-D field on an even grid is required")
    h1, h2, h3 = (m // 2 for m in a.shape)
    acc = np.zeros_like(a)
    for sh in [(0, 0, 0), (h1, h2, 0), (h1, 0, h3), (0, h2, h3)]:
        r = np.roll(a, sh, axis=(0, 1, 2))
        acc += r
        acc += np.roll(np.flip(r, axis=(0, 1, 2)), 1, axis=(0, 1, 2))
    return acc / 8.0


def smooth_field(shape, n_modes: int, seed: int, max_freq: int = 3) -> np.ndarray:
    """A smooth real field on a periodic grid: a sum of random low-order cosines, max |.| = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n1, n2, n3 = shape
    j1 = np.arange(n1)[:, None, None] / n1
    j2 = np.arange(n2)[None, :, None] / n2
    j3 = np.arange(n3)[None, None, :] / n3
    out = np.zeros(shape)
    for _ in range(n_modes):
        m = rng.integers(-max_freq, max_freq + 1, size=3)
        amp = rng.normal()
        ph = rng.uniform(0, 2 * math.pi)
        out += amp * np.cos(2 * math.pi * (m[0] * j1 + m[1] * j2 + m[2] * j3) + ph)
    mx = np.max(np.abs(out))
    return out / mx if mx > 0 else out


def trial_phi(shape, n_mean: float, seed: int, contrast: float = 0.5,
              n_modes: int = 12, max_freq: int = 3) -> np.ndarray:
    """Positive amplitude phi with phi^2 = n_mean * (1 + contrast * smooth field)."""
    f = smooth_field(shape, n_modes, seed, max_freq)
    return np.sqrt(n_mean * (1.0 + contrast * f))


def random_density_samples(count: int, seed: int, log10_min: float = -4.0,
                           log10_max: float = 1.5) -> np.ndarray:
    """Log-uniform densities (bohr^-3) for pointwise kernel checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return 10.0 ** rng.uniform(log10_min, log10_max, size=count)

"""Ionic forces at the converged density.

TEST INFRASTRUCTURE (oracle).

At electronic equilibrium the implicit density dependence drops out (the
Euler equation holds and N_e is fixed, Eq. M12a -> Eq. M12), leaving
    F_I = - int n grad_{R_I} v_ext - grad_{R_I} E_ion .
With v_ext(G) = sum_I v_I(|G|) exp(-i G.R_I) over the kept G != 0 set and
E_ext = V sum_G conj(n(G)) v_ext(G), the first term is
    F_I^ext = - V sum_G G Im[ conj(n(G)) v_I(|G|) exp(-i G.R_I) ],
a brute-force sum over the full spectrum, one ion at a time.  The second term
is the Ewald force.

Pins: frozen-density central differences of E_ext with respect to R_I and the
total force against central differences of the re-minimised F_tot
(tests/test_oracle_energy.py); the force on one ion from a Gaussian electron
density against the gradient of the periodic Gaussian-Gaussian interaction,
computed independently by Poisson summation, which fixes the sign of the phase
exp(-i G.R_I) (tests/test_oracle_orientation.py).
"""
from __future__ import annotations

import numpy as np

from . import potentials as pot
from .energy import System


def external_forces(system: System, nhat, ions=None) -> np.ndarray:
    g = system.grid
    sel = g.keep_nonzero
    q = np.sqrt(g.G2[sel])
    Gs = g.G[:, sel]
    nconj = np.conj(nhat[sel])
    idx = list(range(system.positions.shape[0])) if ions is None else list(ions)
    out = np.zeros((len(idx), 3))
    for k, i in enumerate(idx):
        R = system.positions[i]
        vI = pot.form_factor(q, system.charges[i], system.lpp, g.volume)
        ph = np.exp(-1j * (R @ Gs))
        im = np.imag(nconj * vI * ph)
        out[k] = -g.volume * (Gs @ im)
    return out


def total_forces(system: System, nhat) -> np.ndarray:
    return external_forces(system, nhat) + system.F_ion


def external_energy(system: System, nhat) -> float:
    """V sum_G conj(n(G)) v_ext(G) for the system's current ions (frozen density)."""
    vext, _ = pot.external_potential(system.grid, system.positions, system.charges, system.lpp)
    return system.grid.volume * float(np.real(np.sum(np.conj(nhat) * vext)))

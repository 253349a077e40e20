"""One evaluation of the total electronic free energy and its functional derivative.

TEST INFRASTRUCTURE (oracle).

With n = phi^2 on the grid (the variational variable of the direct
minimisation, Sec. II):
  F_tot = F_s[n] + E_xc[n] + E_H[n] + int n v_ext + E_alphaZ + E_ion
(Eqs. E1, E3, E4 with the Euler-equation objective of Sec. II), where
  F_s   : ftTF or finite-T GGA (Eqs. TF, FGGA), integrated as dv * sum_r
  E_xc  : PZ81 LDA, dv * sum n eps_xc, or the finite-T KSDT LDA free energy
          dv * sum n f_xc(rs, t) (Sec. IV A, Eq. fit2), or none
  E_H   : Eq. E2 in reciprocal space (background-neutralised)
  v_ext : local pseudopotential structure-factor sum (Eq. E4A or Gaussian)
  E_alphaZ = N_e sum_I alpha_I, E_ion = Ewald.
The functional derivative (Eqs. vTF, vftGGA, E10)
  v = df/dn - div(2 df/dsigma grad n) + v_xc + v_H + v_ext + sum_I alpha_I
and, on the electron-count sphere dv * sum phi^2 = N_e, the Euler multiplier
mu = int n v / N_e and the projected gradient g = 2 dv phi (v - mu).

Pointwise terms are evaluated at max(n, 1e-12) (a reading: the paper gives no
density floor); phi itself is never clamped.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import fermi_dirac as fdm
from . import functionals as fnl
from . import potentials as pot
from .grid import Grid

KB_HARTREE_PER_K = 3.1668115634556e-6     # CODATA 2018 k_B / E_h


@dataclasses.dataclass
class System:
    lattice: np.ndarray
    shape: tuple
    positions: np.ndarray
    charges: np.ndarray
    temperature_K: float
    functional: str = "TF"
    xc: str = "PZ81"
    lpp: dict = dataclasses.field(default_factory=lambda: {"kind": "gauss", "rc": 0.5})
    mu_sga: float = fnl.MU_SGA
    with_ions: bool = True

    def __post_init__(self):
        self.lattice = np.asarray(self.lattice, dtype=np.float64).reshape(3, 3)
        self.positions = np.asarray(self.positions, dtype=np.float64).reshape(-1, 3)
        self.charges = np.asarray(self.charges, dtype=np.float64).ravel()
        self.grid = Grid(self.lattice, self.shape)
        self.T = self.temperature_K * KB_HARTREE_PER_K
        self.n_electrons = float(np.sum(self.charges))
        self.refresh_ions()

    def refresh_ions(self):
        if self.positions.shape[0] and self.with_ions:
            self.vext_hat, self.alpha_sum = pot.external_potential(
                self.grid, self.positions, self.charges, self.lpp)
            self.E_ion, self.F_ion = pot.ewald(self.lattice, self.positions, self.charges)
        else:
            self.vext_hat = np.zeros(self.grid.shape, dtype=np.complex128)
            self.alpha_sum = 0.0
            self.E_ion, self.F_ion = 0.0, np.zeros((self.positions.shape[0], 3))

    def set_positions(self, positions):
        self.positions = np.asarray(positions, dtype=np.float64).reshape(-1, 3)
        self.refresh_ions()

    def uniform_phi(self):
        return np.full(self.grid.shape, np.sqrt(self.n_electrons / self.grid.volume))


@dataclasses.dataclass
class EvalResult:
    F_tot: float
    F_s: float
    TS_s: float
    E_xc: float
    E_H: float
    E_ext: float          # G != 0 part of int n v_ext
    E_alphaZ: float
    E_ion: float
    N_e: float
    mu: float
    v: np.ndarray         # total potential on the grid
    nhat: np.ndarray
    grad: np.ndarray      # projected gradient g = 2 dv phi (v - mu)
    TS_xc: float = 0.0    # T S_xc = -T dF_xc/dT (KSDT; 0 for the T-independent PZ81)

    @property
    def E_internal(self) -> float:
        """F_tot + T S_s + T S_xc: the internal energy (the XC entropy term vanishes for PZ81)."""
        return self.F_tot + self.TS_s + self.TS_xc

    def residual(self, phi) -> float:
        """sqrt(sum n (v-mu)^2 / sum n), in hartree."""
        n = phi * phi
        return float(np.sqrt(np.sum(n * (self.v - self.mu) ** 2) / np.sum(n)))


def noninteracting(system: System, n, grad_n=None):
    """Pointwise F_s terms: (f, df/dn, W = 2 df/dsigma grad n or None, T s_s)."""
    nf = np.maximum(n, fnl.DENSITY_FLOOR)
    if system.functional == "TF":
        f, dfdn, ts = fnl.tf_point(nf, system.T)
        return f, dfdn, None, ts
    sigma = np.sum(grad_n * grad_n, axis=0)
    f, dfdn, dfds, ts = fnl.gga_point(nf, sigma, system.T, system.functional, system.mu_sga)
    W = 2.0 * dfds[None] * grad_n
    return f, dfdn, W, ts


def evaluate(phi, system: System) -> EvalResult:
    g = system.grid
    phi = np.asarray(phi, dtype=np.float64)
    n = phi * phi
    N_e = g.integrate(n)
    nhat = g.fft(n)
    grad_n = g.gradient_from_hat(nhat) if system.functional != "TF" else None
    f, dfdn, W, ts = noninteracting(system, n, grad_n)
    v = dfdn.copy()
    if W is not None:
        v -= g.divergence(W)
    F_s = g.integrate(f)
    TS_s = g.integrate(ts)
    TS_xc = 0.0
    if system.xc == "PZ81":
        eps, vxc = fnl.pz81(np.maximum(n, fnl.DENSITY_FLOOR))
        E_xc = g.integrate(n * eps)
        v += vxc
    elif system.xc == "KSDT":
        fxc, vxc, tsxc = fnl.ksdt(np.maximum(n, fnl.DENSITY_FLOOR), system.T)
        E_xc = g.integrate(n * fxc)
        TS_xc = g.integrate(n * tsxc)
        v += vxc
    elif system.xc == "NONE":
        E_xc = 0.0
    else:
        raise ValueError(system.xc)
    E_H, vh_hat = pot.hartree(g, nhat)
    E_ext = g.volume * float(np.real(np.sum(np.conj(nhat) * system.vext_hat)))
    v += np.real(g.ifft(vh_hat + system.vext_hat)) + system.alpha_sum
    E_aZ = N_e * system.alpha_sum
    F_tot = F_s + E_xc + E_H + E_ext + E_aZ + system.E_ion
    mu = float(np.sum(n * v) / np.sum(n))
    grad = 2.0 * g.dv * phi * (v - mu)
    return EvalResult(F_tot=F_tot, F_s=F_s, TS_s=TS_s, E_xc=E_xc, E_H=E_H, E_ext=E_ext,
                      E_alphaZ=E_aZ, E_ion=system.E_ion, N_e=N_e, mu=mu, v=v, nhat=nhat,
                      grad=grad, TS_xc=TS_xc)


def energy_only(phi, system: System) -> float:
    return evaluate(phi, system).F_tot

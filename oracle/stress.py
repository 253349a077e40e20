"""Stress tensor and pressure of the free energy (Eqs. StressTensor, pressure,
stressTF_a, stressTF_b).

TEST INFRASTRUCTURE (oracle).  Plain FP64 sums; shares nothing with the HIP path.

Sigma_ab = (1/V) sum_nu dOmega/dh_{a nu} h_{b nu} is the derivative of Omega under a
homogeneous strain of the cell, h -> (1 + eps) h, with the ions at fixed
fractional coordinates and the density carried along with the cell (grid values
of n times V0/V, so N_e is fixed).  At the minimising density this is the total
derivative, because the density's own response does not change Omega to first
order.  P = -Tr Sigma / 3.  Each energy term gives one piece (before the 1/V):

  non-interacting + XC (local):
      delta_ab [ int (f - n df/dn) + int n (eps_xc - v_xc) - int W.grad n ] - int W_a d_b n
      with W = 2 (df/dsigma) grad n (zero for ftTF); with v_s = df/dn - div W this is
      Eq. stressTF_b (Eq. stressTF_a for ftTF) plus the LDA term
  Hartree:    -delta_ab E_H + V sum_G 4 pi |n(G)|^2 G_a G_b / G^4
  external:   -delta_ab E_ext - sum_G Re[n(G)^* sum_I u_I'(|G|) e^{-i G.R_I}] G_a G_b / |G|,
              u_I = V v_I the volume-free form factor
  alpha Z:    -delta_ab E_alphaZ        (alpha_I ~ 1/V)
  Ewald:      real 1/2 sum Z_i Z_j phi'(r) r_a r_b / r with phi(r) = erfc(a r)/r;
              reciprocal -delta_ab E_rec + (2 pi/V) sum_G w |S|^2 2 G_a G_b (1/G^2 + 1/(4 a^2));
              background -delta_ab E_bg; the self term does not depend on the cell.

The reciprocal sums use the same kept set as the energies (G != 0, no Nyquist
modes), so every piece is the exact strain derivative of the discrete energy.

Pins (tests/test_oracle_stress.py): central differences of the oracle's F_tot
under strain for TF and GGA, Gaussian and HA pseudopotentials, cubic and
triclinic cells; the uniform-gas pressure 2/3 C_TF n^(5/3) as T -> 0 and n T in
the classical limit; the form-factor derivative against central differences.
"""
from __future__ import annotations

from math import pi, sqrt

import numpy as np
from scipy.special import erfc as erfc_v

from . import functionals as fnl
from . import potentials as pot
from .energy import System, noninteracting


def form_factor_derivative(q, Z, lpp: dict):
    """d/dq of u(q) = V v_I(q), the volume-free form factor (q > 0)."""
    q = np.asarray(q, dtype=np.float64)
    if lpp["kind"] == "gauss":
        rc = lpp["rc"]
        e = np.exp(-0.25 * q * q * rc * rc)
        return 4.0 * pi * Z * e * (0.5 * rc * rc / q + 2.0 / q ** 3)
    if lpp["kind"] == "ha":
        rc, A, qc = lpp["rc"], lpp["A"], lpp["qc"]
        g = (Z - A * rc) * np.cos(q * rc) + (A / q) * np.sin(q * rc)
        dg = -(Z - A * rc) * rc * np.sin(q * rc) + A * (rc * np.cos(q * rc) / q - np.sin(q * rc) / (q * q))
        e = np.exp(-(q / qc) ** 6)
        de = -6.0 * q ** 5 / qc ** 6 * e
        return -4.0 * pi * (dg * e / q ** 2 + g * de / q ** 2 - 2.0 * g * e / q ** 3)
    raise ValueError(lpp["kind"])


def local_stress(phi, system: System):
    """V Sigma of the non-interacting and XC free energies (local terms)."""
    g = system.grid
    n = np.asarray(phi, dtype=np.float64) ** 2
    nhat = g.fft(n)
    grad_n = g.gradient_from_hat(nhat) if system.functional != "TF" else None
    f, dfdn, W, _ = noninteracting(system, n, grad_n)
    iso = g.integrate(f - n * dfdn)
    if system.xc == "PZ81":
        eps, vxc = fnl.pz81(np.maximum(n, fnl.DENSITY_FLOOR))
        iso += g.integrate(n * (eps - vxc))
    elif system.xc == "KSDT":
        # Eq. stressLSDAxc: delta_ab int (n f_xc - n v_xc)
        fxc, vxc, _ = fnl.ksdt(np.maximum(n, fnl.DENSITY_FLOOR), system.T)
        iso += g.integrate(n * (fxc - vxc))
    S = np.eye(3) * iso
    if W is not None:
        B = np.array([[g.integrate(W[a] * grad_n[b]) for b in range(3)] for a in range(3)])
        S += -np.eye(3) * np.trace(B) - B
    return S


def hartree_stress(nhat, system: System):
    g = system.grid
    sel = g.keep_nonzero
    E_H, _ = pot.hartree(g, nhat)
    w = 4.0 * pi * np.abs(nhat[sel]) ** 2 / g.G2[sel] ** 2
    Gs = [g.G[a][sel] for a in range(3)]
    S = np.array([[g.volume * float(np.sum(w * Gs[a] * Gs[b])) for b in range(3)] for a in range(3)])
    return S - np.eye(3) * E_H


def external_stress(nhat, system: System):
    g = system.grid
    sel = g.keep_nonzero
    q = np.sqrt(g.G2[sel])
    E_ext = g.volume * float(np.real(np.sum(np.conj(nhat) * system.vext_hat)))
    dS = np.zeros(q.shape, dtype=np.complex128)
    for R, Z in zip(system.positions, system.charges):
        dS += form_factor_derivative(q, Z, system.lpp) * pot.phase(g, R)[sel]
    c = np.real(np.conj(nhat[sel]) * dS) / q
    Gs = [g.G[a][sel] for a in range(3)]
    S = np.array([[-float(np.sum(c * Gs[a] * Gs[b])) for b in range(3)] for a in range(3)])
    return S - np.eye(3) * E_ext


def ewald_stress(lattice, positions, charges, split=None, accuracy=1e-15):
    """V Sigma of the Ewald energy (same splitting and cutoffs as potentials.ewald)."""
    lat = np.asarray(lattice, dtype=np.float64)
    pos = np.asarray(positions, dtype=np.float64)
    Z = np.asarray(charges, dtype=np.float64)
    V = abs(np.linalg.det(lat))
    nat = len(Z)
    if split is None:
        split = sqrt(pi) * (nat / V ** 2) ** (1.0 / 6.0)
    a = split
    c = sqrt(-np.log(accuracy))
    rcut, gcut = c / a, 2.0 * a * c
    S = np.zeros((3, 3))
    L = pot._lattice_images(lat, rcut + float(np.sum(np.linalg.norm(lat, axis=1))))
    for i in range(nat):
        d = pos[i][None, None, :] - pos[None, :, :] + L[:, None, :]
        r = np.linalg.norm(d, axis=2)
        ok = (r > 1e-12) & (r < rcut)
        rr = np.where(ok, r, 1.0)
        dphi = -erfc_v(a * rr) / rr ** 2 - 2.0 * a / sqrt(pi) * np.exp(-(a * rr) ** 2) / rr
        w = np.where(ok, 0.5 * Z[i] * Z[None, :] * dphi / rr, 0.0)
        S += np.einsum("ln,lna,lnb->ab", w, d, d)
    B = 2.0 * pi * np.linalg.inv(lat).T
    Gs = pot._lattice_images(B, gcut)
    Gs = Gs[np.linalg.norm(Gs, axis=1) > 1e-12]
    G2 = np.sum(Gs * Gs, axis=1)
    Sg = np.sum(Z[None, :] * np.exp(1j * (Gs @ pos.T)), axis=1)
    wgt = np.exp(-G2 / (4.0 * a * a)) / G2 * np.abs(Sg) ** 2
    E_rec = 2.0 * pi / V * float(np.sum(wgt))
    k = 2.0 * pi / V * wgt * 2.0 * (1.0 / G2 + 1.0 / (4.0 * a * a))
    S += np.einsum("g,ga,gb->ab", k, Gs, Gs) - np.eye(3) * E_rec
    E_bg = -pi * float(np.sum(Z)) ** 2 / (2.0 * V * a * a)
    S -= np.eye(3) * E_bg
    return S


def stress(phi, system: System):
    """Sigma (3x3, hartree/bohr^3) at amplitude phi: every piece above over V."""
    g = system.grid
    n = np.asarray(phi, dtype=np.float64) ** 2
    nhat = g.fft(n)
    S = local_stress(phi, system) + hartree_stress(nhat, system)
    if system.positions.shape[0] and system.with_ions:
        S += external_stress(nhat, system)
        S -= np.eye(3) * g.integrate(n) * system.alpha_sum
        S += ewald_stress(system.lattice, system.positions, system.charges)
    return S / g.volume


def pressure(sigma) -> float:
    """Eq. pressure: P = -Tr Sigma / 3."""
    return -float(np.trace(sigma)) / 3.0

"""Hartree solve, local pseudopotentials, structure factors and Ewald sums.

TEST INFRASTRUCTURE (oracle).  Brute-force sums, FP64.

* Hartree (Eq. E2) in reciprocal space with a neutralising background:
    E_H = (V/2) sum_{G != 0} 4 pi |n(G)|^2 / G^2,   v_H(G) = 4 pi n(G)/G^2.
* Local pseudopotential form factors v_I(q), normalised so that
  v_ext(G) = sum_I v_I(|G|) exp(-i G.R_I):
    - Gaussian-regularised Coulomb  v(r) = -Z erf(r/r_c)/r
          v(q) = -4 pi Z exp(-q^2 r_c^2/4) / (V q^2),
      G = 0 remainder alpha = pi Z r_c^2 / V (Coulomb tail removed);
    - Heine-Abarenkov (Eq. E4A)
          v(q) = -4 pi/(V q^2) [(Z - A r_c) cos(q r_c) + (A/q) sin(q r_c)] exp(-(q/q_c)^6),
      G = 0 remainder alpha = (2 pi/V)(Z r_c^2 - (2/3) A r_c^3) (q -> 0 expansion).
  The G = 0 terms give E_alphaZ = N_e sum_I alpha_I.
* Ewald energy and forces of point ions Z_I in a neutralising background
  (real + reciprocal + self + background), independent of the split parameter.

Pins (tests/test_oracle_potentials.py): Hartree energy of a Gaussian charge in
a cubic box against its closed form with the simple-cubic Madelung constant;
the Gaussian form factor against the radial Fourier integral of
-Z erf(r/r_c)/r; alpha terms against the series of the form factors; Ewald
independence of the split parameter and the one-ion simple-cubic Madelung
energy; Ewald forces by central differences.  The sign of the phase
exp(-i G.R_I): the potential of one ion is deepest on the ion, and the energy of
a Gaussian density centred at R' equals the independently summed periodic
Gaussian-Gaussian interaction at R' - R (tests/test_oracle_orientation.py).
"""
from __future__ import annotations

from math import erfc, pi, sqrt

import numpy as np
from scipy.special import erfc as erfc_v

from .grid import Grid


def hartree(grid: Grid, nhat):
    """(E_H, v_H(G)) with the G = 0 term and Nyquist planes dropped."""
    sel = grid.keep_nonzero
    vh = np.zeros(grid.shape, dtype=np.complex128)
    vh[sel] = 4.0 * pi * nhat[sel] / grid.G2[sel]
    E = 0.5 * grid.volume * float(np.sum(4.0 * pi * np.abs(nhat[sel]) ** 2 / grid.G2[sel]))
    return E, vh


def form_factor(q, Z, lpp: dict, volume: float):
    """v_I(q) for q > 0 (array)."""
    q = np.asarray(q, dtype=np.float64)
    kind = lpp["kind"]
    if kind == "gauss":
        rc = lpp["rc"]
        return -4.0 * pi * Z * np.exp(-0.25 * q * q * rc * rc) / (volume * q * q)
    if kind == "ha":
        rc, A, qc = lpp["rc"], lpp["A"], lpp["qc"]
        return (-4.0 * pi / (volume * q * q)
                * ((Z - A * rc) * np.cos(q * rc) + (A / q) * np.sin(q * rc))
                * np.exp(-(q / qc) ** 6))
    raise ValueError(kind)


def alpha_term(Z, lpp: dict, volume: float) -> float:
    """G = 0 remainder of v_I after removing -4 pi Z/(V q^2)."""
    kind = lpp["kind"]
    if kind == "gauss":
        return pi * Z * lpp["rc"] ** 2 / volume
    if kind == "ha":
        rc, A = lpp["rc"], lpp["A"]
        return 2.0 * pi / volume * (Z * rc * rc - (2.0 / 3.0) * A * rc ** 3)
    raise ValueError(kind)


def phase(grid: Grid, R):
    """exp(-i G.R) on the full grid for one position R (3,)."""
    return np.exp(-1j * np.tensordot(R, grid.G, axes=(0, 0)))


def external_potential(grid: Grid, positions, charges, lpp: dict):
    """v_ext(G) (kept G != 0) and alpha_sum = sum_I alpha_I."""
    sel = grid.keep_nonzero
    q = np.sqrt(grid.G2[sel])
    vext = np.zeros(grid.shape, dtype=np.complex128)
    alpha_sum = 0.0
    for R, Z in zip(np.asarray(positions), np.asarray(charges)):
        vext[sel] += form_factor(q, Z, lpp, grid.volume) * phase(grid, R)[sel]
        alpha_sum += alpha_term(Z, lpp, grid.volume)
    return vext, alpha_sum


# ---------------------------------------------------------------- Ewald
def _lattice_images(lattice, rmax):
    """All integer combinations L = n.lattice with |L| < rmax (+ slack)."""
    a = np.asarray(lattice)
    # number of images along each axis from the plane spacings
    b = np.linalg.inv(a).T
    nmax = [int(np.ceil(rmax * np.linalg.norm(b[k]))) + 1 for k in range(3)]
    r = [np.arange(-n, n + 1) for n in nmax]
    I, J, K = np.meshgrid(*r, indexing="ij")
    n = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    L = n @ a
    return L[np.linalg.norm(L, axis=1) < rmax]


def ewald(lattice, positions, charges, split=None, accuracy=1e-15):
    """Ewald energy and forces of point charges with a neutralising background."""
    lat = np.asarray(lattice, dtype=np.float64)
    pos = np.asarray(positions, dtype=np.float64)
    Z = np.asarray(charges, dtype=np.float64)
    V = abs(np.linalg.det(lat))
    nat = len(Z)
    if split is None:
        split = sqrt(pi) * (nat / V ** 2) ** (1.0 / 6.0)
    a = split
    c = sqrt(-np.log(accuracy))            # erfc(c) ~ accuracy
    rcut = c / a
    gcut = 2.0 * a * c
    # real space
    L = _lattice_images(lat, rcut + float(np.sum(np.linalg.norm(lat, axis=1))))
    E_real = 0.0
    F = np.zeros((nat, 3))
    for i in range(nat):
        d = pos[i][None, None, :] - pos[None, :, :] + L[:, None, :]    # (nL, nat, 3)
        r = np.linalg.norm(d, axis=2)
        ok = (r > 1e-12) & (r < rcut)
        rr = np.where(ok, r, 1.0)
        e = np.where(ok, erfc_v(a * rr) / rr, 0.0)
        E_real += 0.5 * Z[i] * float(np.sum(e * Z[None, :]))
        fmag = np.where(ok, (erfc_v(a * rr) / rr ** 2 + 2.0 * a / sqrt(pi) * np.exp(-(a * rr) ** 2) / rr) / rr, 0.0)
        F[i] += Z[i] * np.sum((fmag * Z[None, :])[:, :, None] * d, axis=(0, 1))
    # reciprocal space
    B = 2.0 * pi * np.linalg.inv(lat).T
    Gs = _lattice_images(B, gcut)
    Gs = Gs[np.linalg.norm(Gs, axis=1) > 1e-12]
    G2 = np.sum(Gs * Gs, axis=1)
    ph = Gs @ pos.T                                    # (nG, nat)
    S = np.sum(Z[None, :] * np.exp(1j * ph), axis=1)   # sum_I Z_I e^{iG.R_I}
    wgt = np.exp(-G2 / (4.0 * a * a)) / G2
    E_rec = 2.0 * pi / V * float(np.sum(wgt * np.abs(S) ** 2))
    # F_I = (4 pi/V) Z_I sum_G w G Im[e^{iG.R_I} S*(G)]
    im = np.imag(np.exp(1j * ph) * np.conj(S)[:, None])  # (nG, nat)
    F += 4.0 * pi / V * Z[:, None] * ((wgt[:, None] * im).T @ Gs)
    E_self = -a / sqrt(pi) * float(np.sum(Z * Z))
    E_bg = -pi * float(np.sum(Z)) ** 2 / (2.0 * V * a * a)
    return E_real + E_rec + E_self + E_bg, F

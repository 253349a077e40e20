"""Orientation pins of the local-pseudopotential structure-factor sum and its forces.

v_ext(G) = sum_I v_I(|G|) exp(-i G.R_I) (Eq. E4A with the Gaussian-regularised
Coulomb form factor) and the Eq. M12 force sum both carry the phase
exp(-i G.R_I).  A sign flip shared by the two would pass every
finite-difference and GPU-parity test, since both sides would then put the ion
at -R_I.  These tests place the ion and a Gaussian electron density at known,
different points and compare with what does not depend on that sign:

  * the potential of one ion has its minimum on the grid point of the ion;
  * the interaction energy of a normalised Gaussian density
        n(r) = N exp(-|r - R'|^2/s^2) / (pi^{3/2} s^3)
    with the ion's potential -Z erf(r/r_c)/r, in the periodic cell with the
    G = 0 term removed, is -Z N f_w(R' - R) with w^2 = s^2 + r_c^2 and
        f_w(d) = (4 pi/V) sum_{G != 0} exp(-G^2 w^2/4) cos(G.d) / G^2,
    evaluated here independently of the oracle by Poisson summation (a wide
    Gaussian W summed in G space plus the short-ranged difference of the two
    screened Coulomb potentials summed in real space);
  * the force on the ion is -Z N grad f_w(d), i.e. it points toward the density.
"""
import numpy as np
import pytest
from scipy.special import erf

import oracle
from oracle import forces as ofo
from oracle import potentials as opot

L_BOX = 10.0
GRID = (32, 32, 32)
RC = 0.5
Z_ION = 1.0


def periodic_gauss_pair(lattice, d, w, W=None):
    """f_w(d) for a cell with rows `lattice`, computed without the oracle.

    f_w(d) = f_W(d) + sum_L g(d + L) - pi (W^2 - w^2)/V,
    g(r) = [erf(r/w) - erf(r/W)]/r   (Fourier transform 4 pi (e^{-G^2 w^2/4} - e^{-G^2 W^2/4})/G^2),
    with W wide enough that f_W converges in a few G shells and narrow enough
    that g decays within a few lattice translations.
    """
    lat = np.asarray(lattice, dtype=np.float64)
    V = abs(np.linalg.det(lat))
    W = W if W is not None else 0.25 * min(np.linalg.norm(lat, axis=1))
    B = 2.0 * np.pi * np.linalg.inv(lat).T
    m = np.arange(-12, 13)
    M = np.stack(np.meshgrid(m, m, m, indexing="ij"), -1).reshape(-1, 3)
    M = M[np.any(M != 0, axis=1)]
    G = M @ B
    G2 = np.sum(G * G, axis=1)
    fW = 4.0 * np.pi / V * float(np.sum(np.exp(-0.25 * G2 * W * W) * np.cos(G @ d) / G2))
    n = np.arange(-4, 5)
    Nn = np.stack(np.meshgrid(n, n, n, indexing="ij"), -1).reshape(-1, 3)
    r = np.linalg.norm(d[None, :] + Nn @ lat, axis=1)
    small = r < 1e-12
    rr = np.where(small, 1.0, r)
    g = np.where(small, 2.0 / np.sqrt(np.pi) * (1.0 / w - 1.0 / W), (erf(rr / w) - erf(rr / W)) / rr)
    return fW + float(np.sum(g)) - np.pi * (W * W - w * w) / V


def gaussian_density(grid, center, s, N):
    """Periodic Gaussian density (minimum-image displacement) on the grid points."""
    pts = grid.points().reshape(3, -1).T
    lat = grid.lattice
    frac = (pts - center) @ np.linalg.inv(lat)
    frac -= np.round(frac)
    disp = frac @ lat
    r2 = np.sum(disp * disp, axis=1)
    n = N * np.exp(-r2 / (s * s)) / (np.pi ** 1.5 * s ** 3)
    return n.reshape(grid.shape)


def test_closed_form_is_independent_of_the_split():
    lat = np.eye(3) * L_BOX
    d = np.array([1.3, -0.4, 0.9])
    a = periodic_gauss_pair(lat, d, 0.9, W=2.0)
    b = periodic_gauss_pair(lat, d, 0.9, W=2.8)
    assert abs(a - b) < 1e-12 * abs(a)


def test_single_ion_potential_minimum_sits_on_the_ion():
    lat = np.eye(3) * L_BOX
    grid = oracle.grid.Grid(lat, GRID)
    j = np.array([3, 11, 26])
    R = (j / np.array(GRID)) @ lat
    vext, _ = opot.external_potential(grid, [R], [Z_ION], {"kind": "gauss", "rc": RC})
    v = np.real(grid.ifft(vext))
    assert tuple(np.unravel_index(np.argmin(v), v.shape)) == tuple(j)
    # and the potential is symmetric about the ion: v(R + e) = v(R - e)
    for e in [(1, 0, 0), (0, 2, 0), (1, 1, 3)]:
        p = tuple((j + e) % GRID)
        q = tuple((j - np.array(e)) % GRID)
        assert abs(v[p] - v[q]) < 1e-12 * abs(v[p])


@pytest.mark.parametrize("R, Rp", [((1.0, 2.0, 3.0), (2.1, 1.4, 3.5)), ((7.5, 0.7, 4.2), (6.2, 1.9, 4.9))])
def test_gaussian_density_energy_and_force_match_the_periodic_closed_form(R, Rp):
    lat = np.eye(3) * L_BOX
    s, N = 0.8, 2.0
    R, Rp = np.array(R), np.array(Rp)
    sysm = oracle.System(lat, GRID, [R], [Z_ION], 1.0e4, functional="TF")
    g = sysm.grid
    n = gaussian_density(g, Rp, s, N)
    assert abs(g.integrate(n) - N) < 1e-12
    nhat = g.fft(n)
    w = np.sqrt(s * s + RC * RC)
    d = Rp - R
    E_ref = -Z_ION * N * periodic_gauss_pair(lat, d, w)
    E_orc = g.volume * float(np.real(np.sum(np.conj(nhat) * sysm.vext_hat)))
    assert abs(E_orc - E_ref) < 1e-9 * abs(E_ref)
    # the ion at -R (a flipped phase) would give a clearly different energy
    E_flip = -Z_ION * N * periodic_gauss_pair(lat, Rp + R, w)
    assert abs(E_flip - E_ref) > 1e-3 * abs(E_ref)
    # force on the ion: -dE/dR = -Z N grad f_w(d), by central differences of the closed form
    h = 1e-4
    grad = np.array([(periodic_gauss_pair(lat, d + h * e, w) - periodic_gauss_pair(lat, d - h * e, w)) / (2 * h)
                     for e in np.eye(3)])
    F_ref = -Z_ION * N * grad
    F_orc = ofo.external_forces(sysm, nhat)[0]
    assert np.max(np.abs(F_orc - F_ref)) < 1e-7 * np.max(np.abs(F_ref))
    # attractive: the force has a positive component along R' - R
    assert float(F_orc @ d) > 0.0

"""Pins of the oracle's grid operators, Hartree, pseudopotentials and Ewald."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import erfc

from oracle import potentials as pot
from oracle.grid import Grid

MADELUNG_SC = 2.837297479480620   # simple-cubic lattice with uniform background


def test_fft_matches_brute_dft_8cubed():
    rng = np.random.default_rng(3)
    lat = np.array([[5.0, 0, 0], [0.4, 6.0, 0], [0.3, -0.2, 5.5]])
    g = Grid(lat, (8, 6, 12))
    a = rng.normal(size=g.shape)
    r = g.points().reshape(3, -1)
    G = g.G.reshape(3, -1)
    brute = np.exp(-1j * (G.T @ r)) @ a.ravel() / g.N
    assert np.allclose(g.fft(a).ravel(), brute, atol=1e-13)


def test_spectral_gradient_of_plane_wave():
    lat = np.diag([4.0, 5.0, 6.0]) + np.array([[0, 0.3, 0], [0, 0, 0], [0.2, 0, 0]])
    g = Grid(lat, (12, 12, 16))
    m = (2, -3, 1)
    Gv = m[0] * g.recip[0] + m[1] * g.recip[1] + m[2] * g.recip[2]
    r = g.points()
    ph = np.tensordot(Gv, r, axes=(0, 0))
    a = np.cos(ph)
    grad = g.gradient(a)
    for k in range(3):
        assert np.allclose(grad[k], -Gv[k] * np.sin(ph), atol=1e-11)
    div = g.divergence(np.stack([a, a, a]))
    assert np.allclose(div, -np.sum(Gv) * np.sin(ph), atol=1e-11)


def test_nyquist_modes_dropped_and_derivative_antisymmetric():
    g = Grid(np.eye(3) * 3.0, (8, 8, 8))
    rng = np.random.default_rng(1)
    a = rng.normal(size=g.shape)
    b = rng.normal(size=g.shape)
    # <b, D a> = -<D b, a>
    Da = g.gradient(a)
    Db = g.gradient(b)
    for k in range(3):
        assert abs(np.sum(b * Da[k]) + np.sum(Db[k] * a)) < 1e-10
    # a pure Nyquist field has zero gradient
    j = np.arange(8)
    nyq = np.cos(np.pi * j)[:, None, None] * np.ones(g.shape)
    assert np.max(np.abs(g.gradient(nyq))) < 1e-12


def _periodic_gaussian(g, center, Q, s, images=2):
    r = g.points()
    out = np.zeros(g.shape)
    L = g.lattice
    for i in range(-images, images + 1):
        for j in range(-images, images + 1):
            for k in range(-images, images + 1):
                c = center + i * L[0] + j * L[1] + k * L[2]
                d2 = sum((r[a] - c[a]) ** 2 for a in range(3))
                out += np.exp(-d2 / (2 * s * s))
    return Q * out / (2 * math.pi * s * s) ** 1.5


def test_hartree_energy_of_gaussian_charge():
    Lc, s, Q = 10.0, 0.4, 1.3
    g = Grid(np.eye(3) * Lc, (64, 64, 64))
    n = _periodic_gaussian(g, np.array([3.0, 4.0, 5.0]), Q, s, images=1)
    E, vh = pot.hartree(g, g.fft(n))
    V = Lc ** 3
    ref = Q * Q / (2 * math.sqrt(math.pi) * s) - MADELUNG_SC / 2 * Q * Q / Lc + 2 * math.pi * Q * Q * s * s / V
    assert E == pytest.approx(ref, rel=1e-10)


def test_gaussian_form_factor_against_radial_transform():
    Z, rc, V = 1.0, 0.5, 100.0
    lpp = {"kind": "gauss", "rc": rc}
    for q in (0.3, 1.7, 6.0):
        # short-range part Z erfc(r/rc)/r has an absolutely convergent transform
        val, _ = integrate.quad(lambda r: erfc(r / rc) * math.sin(q * r), 0, 12 * rc, limit=400)
        ref = 4 * math.pi * Z / q * val             # FT of  Z erfc(r/rc)/r
        got = V * pot.form_factor(np.array([q]), Z, lpp, V)[0] + 4 * math.pi * Z / q ** 2
        assert got == pytest.approx(ref, rel=1e-9)


@pytest.mark.parametrize("lpp", [{"kind": "gauss", "rc": 0.5},
                                 {"kind": "ha", "rc": 0.25, "A": 6.18, "qc": 29.97},
                                 {"kind": "ha", "rc": 1.15, "A": 0.1107, "qc": 3.5}])
def test_alpha_term_is_q_to_zero_limit(lpp):
    Z, V = 1.0, 50.0
    q = np.array([0.01, 0.02, 0.03])
    rem = V * pot.form_factor(q, Z, lpp, V) + 4 * math.pi * Z / q ** 2
    # rem is even in q: rem(q) = a + b q^2 + c q^4; a is the q -> 0 limit
    A = np.stack([np.ones(3), q ** 2, q ** 4], axis=1)
    lim = np.linalg.solve(A, rem)[0]
    assert V * pot.alpha_term(Z, lpp, V) == pytest.approx(lim, rel=1e-8)


def test_ha_form_factor_real_space_model():
    # Heine-Abarenkov: v(r) = -A (r < rc), -Z/r (r > rc); without the exp(-(q/qc)^6) cutoff
    Z, rc, A, V = 1.0, 0.25, 6.18, 1.0
    lpp = {"kind": "ha", "rc": rc, "A": A, "qc": 1e9}
    q = 2.3
    inner, _ = integrate.quad(lambda r: (-A + Z / r) * r * math.sin(q * r), 0, rc)
    # FT of (v + Z/r): only r < rc contributes
    ref = 4 * math.pi / q * inner
    got = V * pot.form_factor(np.array([q]), Z, lpp, V)[0] + 4 * math.pi * Z / q ** 2
    assert got == pytest.approx(ref, rel=1e-10)


def test_ewald_single_ion_madelung():
    for Lc in (4.0, 9.0):
        E, F = pot.ewald(np.eye(3) * Lc, np.zeros((1, 3)), np.array([1.0]))
        assert E == pytest.approx(-MADELUNG_SC / 2 / Lc, rel=1e-12)
        assert np.max(np.abs(F)) < 1e-12


def test_ewald_split_independence_and_forces():
    rng = np.random.default_rng(11)
    lat = np.array([[6.0, 0.2, 0], [0, 5.5, 0.3], [0.1, 0, 7.0]])
    pos = rng.random((5, 3)) @ lat
    Z = np.array([1.0, 1.0, 2.0, 1.0, 3.0])
    E1, F1 = pot.ewald(lat, pos, Z, split=0.4)
    E2, F2 = pot.ewald(lat, pos, Z, split=0.9)
    assert E1 == pytest.approx(E2, rel=1e-12)
    assert np.allclose(F1, F2, atol=1e-10)
    h = 1e-5
    for i in (0, 3):
        for a in range(3):
            p = pos.copy(); p[i, a] += h
            m = pos.copy(); m[i, a] -= h
            num = -(pot.ewald(lat, p, Z)[0] - pot.ewald(lat, m, Z)[0]) / (2 * h)
            assert num == pytest.approx(F1[i, a], abs=1e-8)

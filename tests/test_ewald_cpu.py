"""Host Ewald sum of the library (ofdft_ewald, no device needed) against the oracle.

The library's sum (minimum-image real space with sorted lattice translations,
half-sphere reciprocal space with separable phase tables, its own splitting
parameter) and the oracle's plain double loop share no code; the Ewald energy
is independent of the splitting parameter, so both must agree to rounding.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import potentials as pot
from paper_1406_0835_amd import binding as B


@pytest.fixture(scope="module", autouse=True)
def _library():
    import os
    if not os.path.exists(B.library_path()):
        from paper_1406_0835_amd import build
        build.build()


def _check(lattice, positions, charges, tol_e=1e-13, tol_f=1e-11):
    E, F = B.ewald(lattice, positions, charges)
    Eo, Fo = pot.ewald(lattice, positions, charges)
    assert abs(E - Eo) <= tol_e * abs(Eo)
    assert np.max(np.abs(F - Fo)) <= tol_f * max(1.0, np.max(np.abs(Fo)))
    # momentum conservation
    assert np.max(np.abs(F.sum(axis=0))) < 1e-10 * max(1.0, np.max(np.abs(F)))


@pytest.mark.parametrize("nat,rho,seed", [(1, 1.0, 1), (2, 1.0, 2), (16, 1.0, 3), (128, 1.0, 4), (128, 2.0, 5)])
def test_cubic_hydrogen_cells(nat, rho, seed):
    c = wl.h_cell(nat, rho, 16, 1e4, seed=900 + seed)
    _check(c.lattice, c.positions, c.charges)


def test_triclinic_cell_mixed_charges():
    rng = np.random.default_rng(11)
    lat = np.array([[6.1, 0.0, 0.0], [1.3, 5.4, 0.0], [-0.8, 0.9, 7.2]])
    pos = rng.random((9, 3)) @ lat
    Z = rng.uniform(0.5, 3.0, 9)
    _check(lat, pos, Z)


def test_single_ion_madelung():
    # one unit charge in a simple-cubic cell with background: -1.4186487 / L (Madelung)
    L = 7.3
    E, F = B.ewald(np.eye(3) * L, np.zeros((1, 3)), np.ones(1))
    assert E == pytest.approx(-1.4186487397 / L, rel=1e-9)
    assert np.max(np.abs(F)) < 1e-12


def test_translation_and_image_invariance():
    c = wl.h_cell(32, 1.5, 16, 1e4, seed=950)
    E0, F0 = B.ewald(c.lattice, c.positions, c.charges)
    shifted = c.positions + np.array([0.37, -1.2, 2.9]) + 2 * c.lattice[0] - c.lattice[2]
    E1, F1 = B.ewald(c.lattice, shifted, c.charges)
    assert E1 == pytest.approx(E0, rel=1e-13)
    assert np.max(np.abs(F1 - F0)) < 1e-11


def test_forces_are_minus_the_energy_gradient():
    c = wl.h_cell(8, 1.0, 16, 1e4, seed=951)
    _, F = B.ewald(c.lattice, c.positions, c.charges)
    h = 1e-5
    for i, k in [(0, 0), (3, 1), (7, 2)]:
        p, m = c.positions.copy(), c.positions.copy()
        p[i, k] += h
        m[i, k] -= h
        dE = (B.ewald(c.lattice, p, c.charges, forces=False)[0] - B.ewald(c.lattice, m, c.charges, forces=False)[0]) / (2 * h)
        assert -dE == pytest.approx(F[i, k], abs=1e-8)


def test_invalid_arguments_are_rejected():
    with pytest.raises(B.OFDFTError) as e:
        B.ewald(np.zeros((3, 3)), np.zeros((1, 3)), np.ones(1))
    assert e.value.code == B.E_ARG
    with pytest.raises(B.OFDFTError):
        B.ewald(np.eye(3) * 5, np.zeros((1, 3)), -np.ones(1))
    with pytest.raises(B.OFDFTError):
        B.ewald(np.eye(3) * 5, np.full((1, 3), np.nan), np.ones(1))


@pytest.mark.parametrize("case", ["cubic", "triclinic"])
def test_stress_term_matches_oracle(case):
    """The library's Ewald stress term against the oracle's strain derivative (which the
    oracle's own tests pin by finite differences of the energy under strain)."""
    from oracle import stress as st
    if case == "cubic":
        c = wl.h_cell(16, 1.0, 16, 1e4, seed=903)
        lat, pos, Z = c.lattice, c.positions, c.charges
    else:
        rng = np.random.default_rng(12)
        lat = np.array([[6.1, 0.0, 0.0], [1.3, 5.4, 0.0], [-0.8, 0.9, 7.2]])
        pos = rng.random((9, 3)) @ lat
        Z = rng.uniform(0.5, 3.0, 9)
    E, F, sig = B.ewald(lat, pos, Z, stress=True)
    ref = st.ewald_stress(lat, pos, Z) / abs(np.linalg.det(lat))
    assert np.allclose(sig, sig.T)
    assert np.max(np.abs(sig - ref)) <= 1e-11 * np.max(np.abs(ref))

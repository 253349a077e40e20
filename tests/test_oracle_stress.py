"""Pins of the oracle's stress tensor (Eqs. StressTensor, pressure, stressTF_a,
stressTF_b): central differences of F_tot under a homogeneous strain of the cell
(ions at fixed fractional coordinates, density carried with the cell), the
uniform-gas pressure in the degenerate and classical limits, and the
form-factor derivative."""
import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import functionals as fn
from oracle import stress as st
from oracle.energy import evaluate

HA = {"kind": "ha", "rc": 0.25, "A": 6.18, "qc": 29.97}
GAUSS = {"kind": "gauss", "rc": 0.5}


def _system(functional, lpp, triclinic, xc="PZ81"):
    cell = wl.h_cell(3, 1.0, (12, 12, 12), 5e4, seed=11)
    if triclinic:
        cell.lattice = np.array([[4.2, 0.0, 0.0], [0.9, 4.6, 0.0], [0.4, -0.7, 5.1]])
        cell.positions = np.random.default_rng(1).random((3, 3)) @ cell.lattice
    return oracle.System(cell.lattice, cell.grid, cell.positions, cell.charges, cell.temperature_K,
                         functional=functional, xc=xc, lpp=lpp)


def _phi(sysm, seed=3):
    g = sysm.grid
    phi = wl.trial_phi(g.shape, sysm.n_electrons / g.volume, seed=seed, contrast=0.5)
    return phi * np.sqrt(sysm.n_electrons / (g.dv * np.sum(phi * phi)))


def _strained(system, eps):
    M = np.eye(3) + eps
    out = oracle.System(system.lattice @ M.T, system.shape, system.positions @ M.T, system.charges,
                        system.temperature_K, functional=system.functional, xc=system.xc, lpp=system.lpp,
                        mu_sga=system.mu_sga)
    if not system.with_ions:
        out.with_ions = False
        out.refresh_ions()
    return out


def _fd(system, phi, a, b, h=1e-5):
    """(1/V) dF/d eps_ab by central differences (symmetric strain for a != b)."""
    V0 = system.grid.volume
    E = []
    for s in (1.0, -1.0):
        eps = np.zeros((3, 3))
        eps[a, b] += s * h
        if a != b:
            eps[b, a] += s * h
        sy = _strained(system, eps)
        E.append(evaluate(phi * np.sqrt(V0 / sy.grid.volume), sy).F_tot)
    return (E[0] - E[1]) / (2 * h) / V0 / (1.0 if a == b else 2.0)


@pytest.mark.parametrize("functional,lpp,triclinic,xc", [
    ("TF", GAUSS, False, "PZ81"), ("VT84F", GAUSS, True, "PZ81"), ("SGA", HA, True, "PZ81"),
    ("KST2", GAUSS, False, "PZ81"), ("VT84F", GAUSS, True, "KSDT"), ("TF", HA, False, "KSDT"),
])
def test_stress_is_strain_derivative_of_the_energy(functional, lpp, triclinic, xc):
    s = _system(functional, lpp, triclinic, xc=xc)
    phi = _phi(s)
    sig = st.stress(phi, s)
    assert np.allclose(sig, sig.T, atol=1e-15)
    for a, b in [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]:
        assert sig[a, b] == pytest.approx(_fd(s, phi, a, b), abs=1e-9 * np.abs(sig).max() + 1e-12), (a, b)


def test_each_term_is_a_strain_derivative():
    """A mistake confined to one piece (a sign, a dropped G_a G_b term) cannot hide
    behind the others: without ions and XC only the local and Hartree pieces remain."""
    s = _system("VT84F", GAUSS, True, xc="NONE")
    s.with_ions = False
    s.refresh_ions()
    phi = _phi(s, seed=5)
    sig = st.stress(phi, s)
    for a, b in [(0, 0), (0, 2), (1, 2)]:
        assert sig[a, b] == pytest.approx(_fd(s, phi, a, b), abs=1e-9 * np.abs(sig).max()), (a, b)


def _uniform_pressure(T_K, nbar):
    L = (4.0 / nbar) ** (1.0 / 3.0)
    s = oracle.System(np.eye(3) * L, (8, 8, 8), np.zeros((4, 3)), np.ones(4), T_K, functional="TF", xc="NONE")
    s.with_ions = False
    s.refresh_ions()
    return st.pressure(st.stress(s.uniform_phi(), s))


def test_uniform_gas_pressure_degenerate_limit():
    nbar = 0.5
    P = _uniform_pressure(10.0, nbar)          # t ~ 1e-5
    assert P == pytest.approx((2.0 / 3.0) * fn.C_TF * nbar ** (5.0 / 3.0), rel=1e-8)


def test_uniform_gas_pressure_classical_limit():
    nbar = 1e-3
    T_K = 3e8
    P = _uniform_pressure(T_K, nbar)            # t ~ 2e4: ideal gas, P = n T
    T = T_K * 3.1668115634556e-6
    assert P == pytest.approx(nbar * T, rel=1e-3)


@pytest.mark.parametrize("lpp", [GAUSS, HA])
def test_form_factor_derivative(lpp):
    q = np.linspace(0.3, 20.0, 57)
    h = 1e-6
    V = 7.0
    num = (oracle.potentials.form_factor(q + h, 1.0, lpp, V) - oracle.potentials.form_factor(q - h, 1.0, lpp, V)) / (2 * h) * V
    assert np.allclose(st.form_factor_derivative(q, 1.0, lpp), num, rtol=1e-7, atol=1e-9)

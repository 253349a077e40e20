"""Pins of the oracle's KSDT finite-T LDA XC free energy (Sec. IV A, Eqs. fit2, vxc1,
stressLSDAxc).

What the paper and the physics fix, independently of the fitted parameters:
  * small rs: Eq. fit2 reduces to the finite-T exchange, rs f_xc -> -a(t);
  * a(0) is the ground-state (Dirac) exchange, eps_x rs = -(3/(4 pi)) (9 pi/4)^(1/3);
  * a(t) for t -> infinity is the first-order exchange of the classical (Boltzmann)
    gas, f_x = -pi n/(2T) per electron, i.e. rs f_x = -(pi/t) (3/(4 pi))^(1/3) (3 pi^2)^(-2/3);
  * t -> 0: the fit tends to a ground-state LDA; it agrees with PZ81 within the
    spread of the ground-state parametrisations (here 2% of the correlation energy);
  * v_xc is the derivative of n f_xc at fixed T (Eq. vxc1), T s_xc = -T df/dT, and the
    XC stress (Eq. stressLSDAxc) is the strain derivative of the energy.
The parameter values of a(t)..e(t) themselves come from the cited publication and are
parity unpinned beyond these limits.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import fermi_dirac as fd
from oracle import functionals as fn

DIRAC = 3.0 / (4.0 * math.pi) * (9.0 * math.pi / 4.0) ** (1.0 / 3.0)   # 0.458165...


def test_small_rs_limit_is_the_finite_T_exchange():
    for t in (1e-3, 0.1, 1.0, 7.0, 300.0):
        a = fn.ksdt_coefficients(t)[0]
        for rs in (1e-18, 1e-16):   # the correction is b(t) rs^(1/2)
            assert rs * fn.ksdt_fxc(rs, t) == pytest.approx(-a, rel=1e-4)


def test_zero_temperature_exchange_is_dirac():
    a0 = fn.ksdt_coefficients(1e-8)[0]
    assert a0 == pytest.approx(DIRAC, rel=1e-6)   # the fit's leading constant is rounded to 6 digits


def test_high_temperature_exchange_is_the_classical_limit():
    for t in (1e3, 1e4):
        a = fn.ksdt_coefficients(t)[0]
        classical = math.pi / t * (3.0 / (4.0 * math.pi)) ** (1.0 / 3.0) / (3.0 * math.pi ** 2) ** (2.0 / 3.0)
        assert a == pytest.approx(classical, rel=2e-4)
    # and that limit is f_x = -pi n/(2T) per electron
    n, T = 0.01, 50.0
    t = fd.reduced_temperature(np.array([n]), T)[0]
    rs = (3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)
    a = fn.ksdt_coefficients(t)[0]
    assert -a / rs == pytest.approx(-math.pi * n / (2.0 * T), rel=2e-3)


@pytest.mark.parametrize("rs", [0.5, 1.0, 2.0, 5.0, 10.0])
def test_zero_temperature_limit_is_a_ground_state_lda(rs):
    n = 3.0 / (4.0 * math.pi * rs ** 3)
    f0 = fn.ksdt_fxc(rs, 1e-8)
    eps_pz, _ = fn.pz81(np.array([n]))
    eps_c = eps_pz[0] + DIRAC / rs
    assert abs(f0 - eps_pz[0]) <= 0.02 * abs(eps_c)


@pytest.mark.parametrize("T", [1e-3, 0.05, 1.0, 20.0])
def test_potential_and_entropy_by_finite_differences(T):
    n = np.geomspace(1e-4, 30.0, 17)
    f, v, ts = fn.ksdt(n, T)
    h = 1e-6 * n
    fp, _, _ = fn.ksdt(n + h, T)
    fm, _, _ = fn.ksdt(n - h, T)
    assert np.allclose(((n + h) * fp - (n - h) * fm) / (2 * h), v, rtol=1e-7, atol=1e-12)
    # f changes little with T at low t: a wider step (truncation ~1e-8) keeps rounding small
    dT = 1e-4 * T
    fTp, _, _ = fn.ksdt(n, T + dT)
    fTm, _, _ = fn.ksdt(n, T - dT)
    assert np.allclose(-T * (fTp - fTm) / (2 * dT), ts, rtol=1e-5, atol=1e-10)


def test_evaluation_potential_is_the_gradient_of_the_discrete_energy():
    rng = np.random.default_rng(3)
    lat = np.eye(3) * 4.0
    pos = rng.random((2, 3)) * 4.0
    s = oracle.System(lat, (12, 12, 12), pos, np.ones(2), 2e5, functional="VT84F", xc="KSDT")
    g = s.grid
    phi = np.sqrt(2.0 / g.volume * (1.0 + 0.4 * np.cos(2 * np.pi * g.points()[0] / 4.0)))
    ev = oracle.evaluate(phi, s)
    for idx in [(1, 2, 3), (7, 0, 11), (5, 5, 5)]:
        e = 1e-6 * phi[idx]
        pp, pm = phi.copy(), phi.copy()
        pp[idx] += e
        pm[idx] -= e
        num = (oracle.evaluate(pp, s).F_tot - oracle.evaluate(pm, s).F_tot) / (2 * e)
        assert num == pytest.approx(2 * g.dv * phi[idx] * ev.v[idx], rel=1e-6)
    assert ev.TS_xc != 0.0
    assert ev.E_internal == pytest.approx(ev.F_tot + ev.TS_s + ev.TS_xc, rel=1e-15)

"""Pins of the oracle's Fermi-Dirac integrals and reduced-temperature factors.

Each check compares against something other than the oracle itself:
mpmath quadrature, the Dirichlet eta function, Sommerfeld/Boltzmann
asymptotics, the T -> 0 Thomas-Fermi and T -> inf classical ideal-gas limits
(Sec. III A), and a brute-force finite-T Lindhard response for h~.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import fermi_dirac as fd

ETAS = np.array([-40.0, -5.0, -1.0, 0.0, 0.3, 2.0, 10.0, 37.0, 100.0])


def _mp_fd(j, eta):
    mp.mp.dps = 30
    eta = mp.mpf(eta)
    ue = mp.sqrt(max(eta, 0))
    pts = [0, ue / 2, ue, ue + 2, ue + 10, mp.inf]
    if j > -1:
        p = 2 * j + 1
        return 2 / mp.gamma(j + 1) * mp.quad(lambda u: u ** p / (1 + mp.exp(u * u - eta)), pts)
    g = {-1.5: lambda f: f * (1 - f),
         -2.5: lambda f: f * (1 - f) * (1 - 2 * f),
         -3.5: lambda f: f * (1 - f) * (1 - 6 * f * (1 - f))}[j]
    return 2 / mp.sqrt(mp.pi) * mp.quad(lambda u: g(1 / (1 + mp.exp(u * u - eta))), pts)


@pytest.mark.parametrize("j", fd.ORDERS)
def test_fd_against_mpmath(j):
    got = fd.fd_all(ETAS)[j]
    for e, g in zip(ETAS, got):
        ref = float(_mp_fd(j, e))
        tol = 1e-13 if j > -2 or e < 20 else 1e-10
        assert abs(g - ref) <= tol * abs(ref), (j, e, g, ref)


@pytest.mark.parametrize("j", fd.ORDERS)
def test_fd_at_zero_is_dirichlet_eta(j):
    # F_j(0) = (1 - 2^-j) zeta(j+1), valid for every order by analytic continuation
    ref = float((1 - mp.mpf(2) ** (-j)) * mp.zeta(j + 1))
    assert fd.fd(j, 0.0)[0] == pytest.approx(ref, rel=2e-15)


def test_fd_half_at_zero_value():
    assert fd.fd(0.5, 0.0)[0] == pytest.approx(0.765147024625408, rel=1e-14)
    assert fd.fd(-0.5, 0.0)[0] == pytest.approx(0.604898643421630, rel=1e-14)


@pytest.mark.parametrize("j", [1.5, 0.5, -0.5, -1.5])
def test_sommerfeld_asymptotics(j):
    for eta in (300.0, 2000.0):
        lead = eta ** (j + 1) / math.gamma(j + 2)
        c1 = math.pi ** 2 / 6 * (j + 1) * j / eta ** 2
        c2 = 7 * math.pi ** 4 / 360 * (j + 1) * j * (j - 1) * (j - 2) / eta ** 4
        ref = lead * (1 + c1 + c2)
        assert fd.fd(j, eta)[0] == pytest.approx(ref, rel=1e-11)


@pytest.mark.parametrize("j", fd.ORDERS)
def test_boltzmann_limit(j):
    eta = -30.0
    z = math.exp(eta)
    ref = z - z * z / 2 ** (j + 1) + z ** 3 / 3 ** (j + 1)
    assert fd.fd(j, eta)[0] == pytest.approx(ref, rel=1e-14)


def test_derivative_relation():
    etas = np.array([-3.0, -0.4, 0.0, 1.7, 6.0, 25.0])
    h = 1e-4
    Fp = fd.fd_all(etas + h)
    Fm = fd.fd_all(etas - h)
    F0 = fd.fd_all(etas)
    pairs = [(1.5, 0.5), (0.5, -0.5), (-0.5, -1.5), (-1.5, -2.5), (-2.5, -3.5)]
    for j, jm in pairs:
        num = (Fp[j] - Fm[j]) / (2 * h)
        assert np.allclose(num, F0[jm], rtol=2e-7, atol=1e-12 * np.max(np.abs(F0[j]))), (j, num, F0[jm])


def test_inverse_round_trip():
    y = np.logspace(-12, 8, 80)
    eta = fd.inverse_f_half(y)
    assert np.allclose(fd.fd(0.5, eta), y, rtol=5e-15, atol=0)


def test_kappa_low_temperature_limit():
    # Sommerfeld: kappa = 1 - (5 pi^2/12) t^2 + O(t^4), xi = 1 + (5 pi^2/12) t^2, zeta = (5 pi^2/6) t^2
    t = np.array([1e-3])
    f = fd.t_factors(t)
    assert f["kappa"][0] == pytest.approx(1 - 5 * math.pi ** 2 / 12 * 1e-6, abs=1e-11)
    assert f["xi"][0] == pytest.approx(1 + 5 * math.pi ** 2 / 12 * 1e-6, abs=1e-11)
    assert f["zeta"][0] == pytest.approx(5 * math.pi ** 2 / 6 * 1e-6, rel=1e-5)
    # the full value at t = 0.01 from the polylogarithm (see _kappa_polylog)
    assert fd.t_factors(np.array([0.01]))["kappa"][0] == pytest.approx(_kappa_polylog(0.01), abs=2e-10)


def test_classical_ideal_gas_limit():
    # f_s = n T (ln(n lambda^3 / 2) - 1) + quantum correction; lambda = sqrt(2 pi / T)
    T = 50.0
    n = 1e-3
    t = fd.reduced_temperature(n, T)
    f = fd.t_factors(np.array([t]))
    c_tf = 0.3 * (3 * math.pi ** 2) ** (2 / 3)
    fs = c_tf * n ** (5 / 3) * f["kappa"][0]
    lam3 = (2 * math.pi / T) ** 1.5
    y = n * lam3 / 2
    ref = n * T * (math.log(y) - 1 + y / 2 ** 2.5)
    assert fs == pytest.approx(ref, rel=1e-10)
    # kinetic energy -> (3/2) n T (1 + y/2^(5/2)) : xi -> (5/2) t (1 + y/2^(5/2))
    assert f["xi"][0] / (2.5 * t) == pytest.approx(1.0 + y / 2 ** 2.5, rel=1e-9)


def _kappa_polylog(t):
    """kappa(t) = (5/3) t (eta - F_{3/2}/F_{1/2}) (Table I, note a) with F_j(eta) =
    -Li_{j+1}(-e^eta) from mpmath's polylogarithm at 40 digits and eta from
    F_{1/2}(eta) = 4/(3 sqrt pi) t^(-3/2) (Eq. tred): independent of the oracle's quadrature."""
    mp = pytest.importorskip("mpmath")
    with mp.workdps(40):
        def F(j, eta):
            return -mp.polylog(j + 1, -mp.e ** eta)
        tt = mp.mpf(t)
        target = 4 / (3 * mp.sqrt(mp.pi)) * tt ** mp.mpf(-1.5)
        eta = mp.findroot(lambda e: F(mp.mpf(1) / 2, e) - target, 1 / tt if tt < 1 else mp.log(target))
        return float(mp.re(5 * tt / 3 * (eta - F(mp.mpf(3) / 2, eta) / F(mp.mpf(1) / 2, eta))))


@pytest.mark.parametrize("t", [0.3, 2.0, 50.0])
def test_kappa_against_polylogarithm(t):
    assert fd.t_factors(np.array([t]))["kappa"][0] == pytest.approx(_kappa_polylog(t), rel=1e-11)


def test_t_derivatives_by_finite_difference():
    t = np.array([0.03, 0.2, 1.0, 4.0])
    h = 1e-5 * t
    P = fd.t_factors(t + h)
    M = fd.t_factors(t - h)
    C = fd.t_factors(t)
    for key, dkey in (("kappa", "dkappa"), ("xi", "dxi"), ("zeta", "dzeta"), ("h", "dh"), ("dh", "d2h")):
        num = (P[key] - M[key]) / (2 * h)
        assert np.allclose(num, C[dkey], rtol=1e-6, atol=1e-9), (key, num, C[dkey])
    # zeta = -t kappa'  (Eq. xizeta)
    assert np.allclose(C["zeta"], -t * (P["kappa"] - M["kappa"]) / (2 * h), rtol=1e-7)


def test_htilde_limits_and_shape():
    lo = fd.t_factors(np.array([1e-3]))
    assert (lo["h"][0] - 1) / 1e-6 == pytest.approx(math.pi ** 2 / 3, rel=1e-4)
    hi = fd.t_factors(np.array([1e4]))
    assert hi["h"][0] == pytest.approx(3.0, rel=1e-5)
    t = np.logspace(-2, math.log10(50), 40)
    f = fd.t_factors(t)
    assert np.all(np.diff(f["h"]) > 0)
    assert np.all(f["h"] - t * f["dh"] > 0)
    # s_sigma^2 / s^2 -> 4/5 and s_tau^2/s^2 -> 1 as t -> 0
    lo = fd.t_factors(np.array([1e-3]))
    assert lo["dh"][0] * 1e-3 / lo["zeta"][0] == pytest.approx(0.8, rel=1e-4)
    assert (lo["h"][0] - 1e-3 * lo["dh"][0]) / lo["xi"][0] == pytest.approx(1.0, rel=1e-5)


def _lindhard_chi(q, mu, T):
    """Static finite-T Lindhard function by brute-force k integration (spin 2)."""
    f = lambda k: 1 / (1 + mp.exp((k * k / 2 - mu) / T))
    integrand = lambda k: k * f(k) * mp.log(abs((2 * k + q) / (2 * k - q)))
    kmax = mp.sqrt(2 * (max(mu, 0) + 60 * T))
    pts = [0, q / 2, mp.sqrt(2 * max(mu, T)), kmax]
    pts = sorted(set(pts))
    return -1 / (mp.pi ** 2 * q) * mp.quad(integrand, pts)


@pytest.mark.parametrize("mu_over_T", [4.0, 0.5, -2.0])
def test_htilde_against_finite_T_lindhard(mu_over_T):
    # The SGA free energy int (h~/72)|grad n|^2/n must reproduce the q^2 term of
    # the free-electron static response: chi(q) = -n' + (n'^2 h~ / (36 n)) q^2 + O(q^4).
    mp.mp.dps = 30
    T = mp.mpf("0.5")
    mu = mu_over_T * T
    fk = lambda k: 1 / (1 + mp.exp((k * k / 2 - mu) / T))
    kmax = mp.sqrt(2 * (max(mu, 0) + 80 * T))
    n = mp.quad(lambda k: k * k * fk(k), [0, mp.sqrt(2 * max(mu, T)), kmax]) / mp.pi ** 2
    qs = [mp.mpf("0.01"), mp.mpf("0.02"), mp.mpf("0.04")]
    chis = [_lindhard_chi(q, mu, T) for q in qs]
    # chi = c0 + c2 q^2 + c4 q^4: solve the 3x3 system
    A = mp.matrix([[1, q ** 2, q ** 4] for q in qs])
    c = mp.lu_solve(A, mp.matrix(chis))
    nprime = -c[0]
    htilde_brute = float(36 * n * c[1] / nprime ** 2)
    t = float(2 * T / (3 * mp.pi ** 2 * n) ** (mp.mpf(2) / 3))
    h = fd.t_factors(np.array([t]))["h"][0]
    assert h == pytest.approx(htilde_brute, rel=1e-5)

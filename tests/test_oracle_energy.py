"""Pins of the oracle's total-energy evaluation, minimiser and forces."""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import fermi_dirac as fd
from oracle import forces as frc
from oracle import functionals as fn
from oracle import minimize as mn

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _small_system(functional="TF", T_K=5e4, shape=(12, 12, 12), nat=2, edge=4.0, seed=5, xc="PZ81",
                  lpp=None):
    rng = np.random.default_rng(seed)
    pos = rng.random((nat, 3)) * edge
    return oracle.System(np.eye(3) * edge, shape, pos, np.ones(nat), T_K, functional=functional,
                         xc=xc, lpp=lpp or {"kind": "gauss", "rc": 0.5})


def test_paper_sample_output_identities():
    vals = {}
    with open(os.path.join(GOLDEN, "qe_sample_output.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            vals[k] = float(v)
    assert vals["Ekin"] + vals["Etot"] == pytest.approx(vals["Ekin_plus_Etot"], abs=1e-8)
    assert vals["Ekin"] + vals["EinternEl"] == pytest.approx(vals["Eint"], abs=1e-8)
    # Etot = EinternEl + (-TS): the convention E_internal = F_tot + T S
    assert vals["EinternEl"] + vals["minus_TS"] == pytest.approx(vals["Etot"], abs=1e-8)
    s = _small_system("SGA")
    ev = oracle.evaluate(s.uniform_phi() * (1 + 0.1 * wl.smooth_field(s.grid.shape, 4, 1)), s)
    assert ev.E_internal + (-ev.TS_s) == pytest.approx(ev.F_tot, rel=1e-15)


def test_jellium_uniform_density_is_stationary():
    s = _small_system("VT84F")
    s.with_ions = False
    s.refresh_ions()
    phi = s.uniform_phi()
    ev = oracle.evaluate(phi, s)
    nbar = s.n_electrons / s.grid.volume
    f, v, _ = fn.tf_point(np.array([nbar]), s.T)
    eps, vxc = fn.pz81(np.array([nbar]))
    assert ev.F_tot == pytest.approx(s.grid.volume * (f[0] + nbar * eps[0]), rel=1e-13)
    assert np.max(np.abs(ev.grad)) < 1e-14
    assert ev.mu == pytest.approx(v[0] + vxc[0], rel=1e-13)


@pytest.mark.parametrize("functional", ["TF", "SGA", "VT84F", "KST2"])
def test_potential_is_gradient_of_discrete_energy(functional):
    s = _small_system(functional)
    nbar = s.n_electrons / s.grid.volume
    phi = wl.trial_phi(s.grid.shape, nbar, seed=3, contrast=0.6)
    ev = oracle.evaluate(phi, s)
    full = 2 * s.grid.dv * phi * ev.v
    rng = np.random.default_rng(0)
    for _ in range(4):
        j = tuple(rng.integers(0, 12, 3))
        d = 1e-5 * phi[j]
        p = phi.copy(); p[j] += d
        m = phi.copy(); m[j] -= d
        num = (oracle.evaluate(p, s).F_tot - oracle.evaluate(m, s).F_tot) / (2 * d)
        assert num == pytest.approx(full[j], rel=2e-6, abs=1e-11)


@pytest.mark.parametrize("functional", ["TF", "SGA"])
def test_linear_response_of_uniform_gas(functional):
    # weak v_ext = eps cos(G.r): dn(G) = -(eps/2) / (dmu/dn + [h~ G^2/(36 n)] + 4 pi/G^2 + dv_xc/dn)
    s = _small_system(functional, T_K=3e4, shape=(16, 16, 16), edge=5.0)
    s.with_ions = False
    s.refresh_ions()
    eps = 1e-3
    m = (1, 0, 0)
    idx = tuple(mm % 16 for mm in m)
    midx = tuple((-mm) % 16 for mm in m)
    s.vext_hat = np.zeros(s.grid.shape, dtype=complex)
    s.vext_hat[idx] = eps / 2
    s.vext_hat[midx] = eps / 2
    r = mn.minimize_cg(s, tol_energy=1e-16, tol_residual=1e-11, max_iter=400)
    nbar = s.n_electrons / s.grid.volume
    dn = r.result.nhat[idx]
    t = fd.reduced_temperature(nbar, s.T)
    F = fd.fd_all(fd.eta_of_t(np.array([t])))
    dmudn = s.T * F[0.5][0] / (nbar * F[-0.5][0])
    h = 1e-6 * nbar
    dvxc = (fn.pz81(np.array([nbar + h]))[1][0] - fn.pz81(np.array([nbar - h]))[1][0]) / (2 * h)
    G2 = s.grid.G2[idx]
    kern = dmudn + 4 * math.pi / G2 + dvxc
    if functional == "SGA":
        kern += fd.t_factors(np.array([t]))["h"][0] * G2 / (36 * nbar)
    assert dn.real == pytest.approx(-(eps / 2) / kern, rel=2e-5)


def test_cg_preserves_constraint_and_decreases():
    c = wl.h_cell(4, 1.0, 16, 2e4, seed=77)
    s = oracle.System(c.lattice, c.grid, c.positions, c.charges, c.temperature_K, functional="SGA")
    norms = []
    r = mn.minimize_cg(s, tol_energy=1e-9, max_iter=60,
                       callback=lambda i, p, e: norms.append(s.grid.dv * np.sum(p * p)))
    assert r.converged
    assert np.allclose(norms, s.n_electrons, rtol=1e-13)
    assert np.all(np.diff(r.history) <= 1e-12)


def test_cg_and_tn_agree():
    c = wl.h_cell(2, 1.0, 8, 5e4, seed=78)
    s = oracle.System(c.lattice, c.grid, c.positions, c.charges, c.temperature_K, functional="VT84F")
    a = mn.minimize_cg(s, tol_energy=1e-12, tol_residual=1e-8, max_iter=500)
    b = mn.minimize_tn(s, tol_energy=1e-12, tol_residual=1e-8)
    assert a.converged and b.converged
    assert a.result.F_tot == pytest.approx(b.result.F_tot, rel=1e-11)
    assert b.iterations < a.iterations


def test_external_force_is_frozen_density_derivative():
    s = _small_system("TF", nat=3, seed=9)
    phi = wl.trial_phi(s.grid.shape, s.n_electrons / s.grid.volume, seed=4)
    nhat = s.grid.fft(phi * phi)
    F = frc.external_forces(s, nhat)
    h = 1e-5
    pos0 = s.positions.copy()
    for i, a in ((0, 0), (2, 1), (1, 2)):
        p = pos0.copy(); p[i, a] += h
        m = pos0.copy(); m[i, a] -= h
        s.positions = p
        Ep = frc.external_energy(s, nhat)
        s.positions = m
        Em = frc.external_energy(s, nhat)
        s.positions = pos0
        assert -(Ep - Em) / (2 * h) == pytest.approx(F[i, a], rel=1e-7, abs=1e-10)


def test_total_force_is_derivative_of_minimised_free_energy():
    # Eq. M12: at equilibrium the implicit density response drops out
    s = _small_system("TF", nat=2, seed=21, edge=4.0, shape=(12, 12, 12))
    tol = dict(tol_energy=1e-14, tol_residual=1e-10, max_iter=800)
    r = mn.minimize_cg(s, **tol)
    F = frc.total_forces(s, r.result.nhat)
    h = 2e-4
    pos0 = s.positions.copy()
    i, a = 0, 1
    E = []
    for sgn in (1, -1):
        p = pos0.copy(); p[i, a] += sgn * h
        s.set_positions(p)
        E.append(mn.minimize_cg(s, phi0=r.phi, **tol).result.F_tot)
    s.set_positions(pos0)
    num = -(E[0] - E[1]) / (2 * h)
    assert num == pytest.approx(F[i, a], abs=2e-6)
    assert abs(np.sum(F[:, a])) < 0.05   # egg-box effect only

"""The MD driver's host logic (no device): velocity Verlet, the Andersen thermostat,
the output block and the XYZ trajectory, on a harmonic toy surface passed in place
of the library call."""
import types

import numpy as np
import pytest

from paper_1406_0835_amd import md

K_SPRING = 0.05   # hartree/bohr^2


def _harmonic(x):
    F = 0.5 * K_SPRING * float(np.sum(x * x))
    rep = types.SimpleNamespace(iterations=1, evaluations=1, E_internal=F, TS_s=0.0, E_xc=0.0)
    return F, -K_SPRING * x, rep


def test_nve_conserves_energy():
    nat = 8
    m = np.full(nat, md.H_MASS_ME)
    x0 = np.random.default_rng(1).normal(0, 0.3, (nat, 3))
    v0 = md.maxwell_boltzmann(nat, 3e4, md.H_MASS_ME, seed=2)
    period = 2 * np.pi * np.sqrt(md.H_MASS_ME / K_SPRING)
    recs = md.velocity_verlet(None, x0, v0, np.ones(nat), m, period / 200, 400, step=_harmonic)
    e = np.array([r.F_total + r.kinetic for r in recs])
    assert np.ptp(e) < 1e-3 * abs(e.mean())


def test_nve_positions_follow_the_closed_form_of_the_harmonic_map():
    # velocity Verlet in a harmonic well: x_n = x_0 cos(na) + (dt v_0 / sin a) sin(na),
    # cos a = 1 - (w dt)^2 / 2 (the discrete map's exact solution)
    nat, dt = 6, 12.0
    m = np.full(nat, md.H_MASS_ME)
    rng = np.random.default_rng(3)
    x0 = rng.normal(0, 0.3, (nat, 3))
    v0 = rng.normal(0, 1e-3, (nat, 3))
    seen = []
    md.velocity_verlet(None, x0, v0, np.ones(nat), m, dt, 120, step=_harmonic,
                       callback=lambda rec, x, v, f: seen.append((rec.step, x.copy())))
    a = np.arccos(1.0 - 0.5 * (K_SPRING / md.H_MASS_ME) * dt * dt)
    for k, x in seen:
        ref = x0 * np.cos(k * a) + (dt * v0 / np.sin(a)) * np.sin(k * a)
        assert np.max(np.abs(x - ref)) < 1e-12, k


def test_andersen_thermostat_reaches_the_target_temperature():
    nat = 64
    m = np.full(nat, md.H_MASS_ME)
    period = 2 * np.pi * np.sqrt(md.H_MASS_ME / K_SPRING)
    dt = period / 50
    T = 2e4
    th = md.Thermostat(T_K=T, nu=0.2 / dt, seed=7)
    recs = md.velocity_verlet(None, np.zeros((nat, 3)), np.zeros((nat, 3)), np.ones(nat), m, dt, 3000,
                              thermostat=th, step=_harmonic)
    Tm = np.mean([r.T_ion for r in recs[500:]])
    assert Tm == pytest.approx(T, rel=0.05)
    # a zero collision rate leaves the dynamics microcanonical
    v = np.ones((nat, 3))
    assert md.andersen(v, m, T, 0.0, dt, np.random.default_rng(0)) == 0 and np.all(v == 1.0)


def test_output_block_identities():
    rec = md.MDRecord(3, F_total=-10.0, kinetic=0.5, iterations=4, evaluations=9, wall_ms=1.0,
                      E_internal=-9.0, TS=1.0, E_xc=-2.0, T_ion=1000.0, pressure=0.01)
    text = md.output_block(rec)
    vals = {l.split("=")[0].strip(): float(l.split("=")[1].split()[0]) for l in text.splitlines() if "=" in l}
    assert vals["Ekin+Etot"] == pytest.approx(vals["Ekin"] + vals["Etot"])
    assert vals["Eint"] == pytest.approx(vals["Ekin"] + vals["EinternEl"])
    assert vals["EinternEl"] + vals["-TS"] == pytest.approx(vals["Etot"])
    assert vals["P"] == pytest.approx(0.01)


def test_xyz_trajectory(tmp_path):
    pos = np.arange(6, dtype=float).reshape(2, 3)
    path = tmp_path / "md.xyz"
    md.write_xyz(str(path), [(0, pos, -1.0), (1, pos + 1, -1.5)], ["H", "H"])
    lines = path.read_text().splitlines()
    assert lines[0] == "2" and lines[4] == "2"
    assert float(lines[3].split()[1]) == pytest.approx(3 * md.BOHR_ANGSTROM)

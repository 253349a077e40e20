"""GPU stress tensor and pressure (ofdft_stress, the pressure output of
ofdft_free_energy_and_forces) against the oracle's stress (Eqs. StressTensor,
pressure, stressTF_a, stressTF_b; pinned by strain finite differences in
tests/test_oracle_stress.py), both at the GPU's converged density.  FP64: 1e-9 of
the largest component; mixed: 1e-5."""
import ctypes

import numpy as np
import pytest

import workloads as wl
from oracle import stress as st
from paper_1406_0835_amd import binding as B

from _gpu_common import make_pair

pytestmark = pytest.mark.gpu

HA = {"kind": "ha", "rc": 0.25, "A": 6.18, "qc": 29.97}


def _cell(shape, triclinic, nat=4, seed=820):
    cell = wl.h_cell(nat, 1.0, shape, 5e4, seed=seed)
    if triclinic:
        cell.lattice = np.array([[4.2, 0.0, 0.0], [0.9, 4.6, 0.0], [0.4, -0.7, 5.1]])
        cell.positions = np.random.default_rng(seed).random((nat, 3)) @ cell.lattice
    return cell


@pytest.mark.parametrize("functional,precision,shape,triclinic,lpp,xc", [
    ("TF", "fp64", (16, 16, 16), False, None, "PZ81"),
    ("VT84F", "fp64", (16, 16, 16), False, None, "PZ81"),
    ("SGA", "fp64", (12, 16, 12), True, HA, "PZ81"),
    ("VT84F", "fp64", (24, 24, 24), True, None, "PZ81"),
    ("VT84F", "mixed", (32, 32, 32), False, None, "PZ81"),
    ("TF", "mixed", (24, 24, 24), True, None, "PZ81"),
    ("VT84F", "fp64", (16, 16, 16), True, None, "KSDT"),
    ("TF", "fp64", (16, 16, 16), False, HA, "KSDT"),
    ("VT84F", "mixed", (24, 24, 24), False, None, "KSDT"),
])
def test_stress_matches_oracle(functional, precision, shape, triclinic, lpp, xc):
    cell = _cell(shape, triclinic)
    ctx, sysm = make_pair(cell, functional, precision=precision, lpp=lpp, xc=xc,
                          tol_energy=1e-10 if precision == "fp64" else 1e-8)
    ctx.minimize_density()
    sig = ctx.stress()
    ref = st.stress(ctx.get_density(), sysm)
    tol = 1e-9 if precision == "fp64" else 1e-5
    assert np.allclose(sig, sig.T, rtol=0, atol=1e-15 * np.max(np.abs(sig)) + 1e-18)
    assert np.max(np.abs(sig - ref)) <= tol * np.max(np.abs(ref)), (sig, ref)
    # the pressure output of free_energy_and_forces is -Tr/3 of the same tensor
    lib = B.load_library()
    P = ctypes.c_double()
    F = ctypes.c_double()
    rc = lib.ofdft_free_energy_and_forces(ctx._h, ctypes.byref(F), None, None, ctypes.byref(P))
    assert rc == 0
    assert P.value == pytest.approx(st.pressure(ref), rel=tol, abs=tol * np.max(np.abs(ref)))


def test_stress_needs_a_converged_density():
    cell = _cell((12, 12, 12), False)
    ctx, _ = make_pair(cell, "TF")
    with pytest.raises(B.OFDFTError) as e:
        ctx.stress()
    assert e.value.code == B.E_STATE


def test_stress_is_the_strain_derivative_of_the_converged_energy():
    """Pressure from the tensor against -dF/dV of full minimisations at three volumes
    (the density relaxes at each volume, so this checks the Hellmann-Feynman reading
    as well as the sums)."""
    cell = _cell((16, 16, 16), False, nat=3, seed=821)
    F = []
    h = 2e-4
    for s in (-h, 0.0, h):
        c = wl.h_cell(3, 1.0, (16, 16, 16), 5e4, seed=821)
        c.lattice = cell.lattice * (1.0 + s)
        c.positions = cell.positions * (1.0 + s)
        ctx, _ = make_pair(c, "VT84F", tol_energy=1e-12)
        F.append(ctx.minimize_density().F_total)
        if s == 0.0:
            P = ctx.pressure()
    V0 = abs(np.linalg.det(cell.lattice))
    dFdV = (F[2] - F[0]) / (V0 * ((1 + h) ** 3 - (1 - h) ** 3))
    assert P == pytest.approx(-dFdV, rel=1e-5)


def test_nvt_md_steps_with_pressure_and_output_block(tmp_path):
    """A few Andersen-NVT steps through the library with the pressure in each record,
    the paper's output block and an md.xyz trajectory."""
    from paper_1406_0835_amd import md
    cell = _cell((16, 16, 16), False, nat=4, seed=822)
    ctx, _ = make_pair(cell, "VT84F", tol_energy=1e-9)
    m = np.full(cell.nat, md.H_MASS_ME)
    v0 = md.maxwell_boltzmann(cell.nat, 5e4, md.H_MASS_ME, seed=3)
    frames = []
    recs = md.velocity_verlet(ctx, cell.positions, v0, cell.charges, m, 0.2 * md.FS_AU, 3,
                              thermostat=md.Thermostat(5e4, 0.01, seed=4), pressure=True,
                              callback=lambda r, x, v, f: frames.append((r.step, x.copy(), r.F_total)))
    assert all(np.isfinite(r.pressure) for r in recs)
    assert recs[-1].E_internal == pytest.approx(recs[-1].F_total + recs[-1].TS, rel=1e-12)
    assert "EinternEl" in md.output_block(recs[-1])
    md.write_xyz(str(tmp_path / "md.xyz"), frames, ["H"] * cell.nat)
    assert (tmp_path / "md.xyz").read_text().count("step") == 3

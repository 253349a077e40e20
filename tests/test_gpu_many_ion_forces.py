"""Forces of cells with many ions (Eq. M12).  From 256 ions up the library sums the
external-potential force with one thread per ion; that kernel is checked against the
G-parallel kernel on the same converged state (only the summation order differs) and,
at the library's converged FP64 density, against the oracle's forces."""
import numpy as np
import pytest

import workloads as wl
from oracle import forces as frc

from _gpu_common import make_ctx, oracle_system

pytestmark = pytest.mark.gpu


def _cell(kind):
    if kind == "gauss":   # 300 ions: one full tile of 256 and a ragged one
        return wl.h_cell(300, 1.0, 32, 2e4, seed=1401), None
    cell = wl.fcc_al_cell(4, 64)   # 256 ions, displaced from the lattice sites
    rng = np.random.Generator(np.random.PCG64(1402))
    cell.positions = cell.positions + rng.normal(0.0, 0.1, cell.positions.shape)
    return cell, wl.AL_HA_LPP


def _forces(cell, lpp, precision, mode, monkeypatch):
    monkeypatch.setenv("OFDFT_ION_FORCES", mode)
    ctx = make_ctx(cell, "TF", precision=precision, lpp=lpp, tol_energy=1e-10 if precision == "fp64" else 1e-7)
    monkeypatch.delenv("OFDFT_ION_FORCES")
    ctx.minimize_density()
    _, _, f = ctx.free_energy_and_forces()
    phi = ctx.get_density()
    ctx.close()
    return f, phi


@pytest.mark.parametrize("kind", ["gauss", "ha"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_per_ion_kernel_matches_g_parallel_kernel(kind, precision, monkeypatch):
    cell, lpp = _cell(kind)
    f_ion, phi_ion = _forces(cell, lpp, precision, "1", monkeypatch)
    f_g, phi_g = _forces(cell, lpp, precision, "0", monkeypatch)
    assert np.array_equal(phi_ion, phi_g)
    scale = max(1.0, float(np.max(np.abs(f_g))))
    assert np.max(np.abs(f_ion - f_g)) <= (1e-11 if precision == "fp64" else 1e-5) * scale


@pytest.mark.parametrize("kind", ["gauss", "ha"])
def test_per_ion_forces_match_oracle(kind, monkeypatch):
    cell, lpp = _cell(kind)
    f, phi = _forces(cell, lpp, "fp64", "1", monkeypatch)
    s = oracle_system(cell, "TF", lpp=lpp)
    fo = frc.total_forces(s, s.grid.fft(phi * phi))
    assert np.max(np.abs(f - fo)) <= 1e-9 * max(1.0, float(np.max(np.abs(fo))))

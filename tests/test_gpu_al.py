"""fcc aluminium with the Heine-Abarenkov Al pseudopotential (Eq. E4A, the paper's
static scaling workload at 2.70 g/cm^3 and 100 K): one evaluation against the
oracle, and at the converged density the symmetries of the perfect lattice (zero
forces, an isotropic stress tensor) in FP64 and mixed precision."""
import numpy as np
import pytest

import oracle
import workloads as wl

from _gpu_common import make_pair, normalized_phi, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_al_evaluation_matches_oracle(precision, tol):
    cell = wl.fcc_al_cell(1, 24)
    ctx, sysm = make_pair(cell, "VT84F", precision=precision, lpp=wl.AL_HA_LPP)
    phi = normalized_phi(sysm, seed=31, contrast=0.4)
    ctx.set_density(phi)
    rep, v = ctx.eval(potential=True)
    ev = oracle.evaluate(phi, sysm)
    for a, b in [("F_total", "F_tot"), ("F_s", "F_s"), ("E_H", "E_H"), ("E_ext", "E_ext"), ("E_xc", "E_xc"),
                 ("E_ion", "E_ion"), ("mu", "mu")]:
        assert abs(getattr(rep, a) - getattr(ev, b)) <= tol * max(abs(getattr(ev, b)), 1e-3 * abs(ev.F_tot)), a
    assert np.sqrt(np.mean((v - ev.v) ** 2)) / np.sqrt(np.mean(ev.v ** 2)) <= 10 * tol


def test_al_lattice_symmetries_at_the_minimum():
    cell = wl.fcc_al_cell(2, 32)
    F = {}
    for precision in ("fp64", "mixed"):
        ctx, _ = make_pair(cell, "VT84F", precision=precision, lpp=wl.AL_HA_LPP,
                           tol_energy=1e-10 if precision == "fp64" else 1e-8, cg_precond=8.0)
        rep = ctx.minimize_density()
        F[precision] = rep.F_total
        _, _, f = ctx.free_energy_and_forces()
        assert np.max(np.abs(f)) < (1e-6 if precision == "fp64" else 1e-4)
        sig = ctx.stress()
        d = np.diag(sig)
        assert np.max(np.abs(d - d.mean())) <= (1e-8 if precision == "fp64" else 1e-5) * abs(d.mean())
        assert np.max(np.abs(sig - np.diag(d))) <= (1e-8 if precision == "fp64" else 1e-5) * abs(d.mean())
    assert rel(F["mixed"], F["fp64"]) <= 1e-6

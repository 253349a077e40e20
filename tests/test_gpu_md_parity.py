"""Born-Oppenheimer MD through the library against the oracle (Sec. VI B; the interface of
Sec. V D): the same velocity-Verlet steps, one driven by the C ABI (set_ions,
minimize_density with the warm start, free_energy_and_forces), the other by the oracle's
velocity_verlet with oracle minimisations and Eq. M12 forces.  Both minimise to a residual of
1e-10 hartree, so their forces agree to ~1e-10 hartree/bohr and a position error grows by
about dt^2/M times that per step (dt = 0.2 fs, M = the proton mass).  FP64: positions within
1e-9 bohr, E_cons = sum M v^2/2 + F_tot within 1e-10 relative, at every step."""
import numpy as np
import pytest

import workloads as wl
from oracle import forces as frc
from oracle import md as omd
from oracle import minimize as mn
from paper_1406_0835_amd import md

from _gpu_common import make_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("functional", ["TF", "VT84F"])
def test_nve_trajectory_matches_oracle(functional):
    cell = wl.h_cell(4, 1.0, (16, 16, 16), 5e4, seed=990)
    ctx, sysm = make_pair(cell, functional, tol_energy=1e-13, tol_residual=1e-10,
                          cg_precond=8.0 if functional != "TF" else 0.0)
    masses = np.full(cell.nat, md.H_MASS_ME)
    assert md.H_MASS_ME == pytest.approx(omd.H_MASS_ME, rel=1e-15)
    v0 = md.maxwell_boltzmann(cell.nat, 5e4, md.H_MASS_ME, seed=991)
    dt = 0.2 * md.FS_AU
    # each oracle step is a CPU minimisation to 1e-10 hartree: the gradient-corrected case
    # keeps to two steps (about a minute of host time), the ftTF case takes four
    n_steps = 4 if functional == "TF" else 2
    recs = []
    md.velocity_verlet(ctx, cell.positions, v0, cell.charges, masses, dt, n_steps,
                       callback=lambda rec, x, v, f: recs.append((x.copy(), v.copy(), rec.F_total + rec.kinetic)))
    state = {"phi": None}

    def energy_forces(x):
        sysm.set_positions(x)
        r = mn.minimize_cg(sysm, phi0=state["phi"], tol_energy=1e-13, tol_residual=1e-10, max_iter=4000)
        assert r.converged
        state["phi"] = r.phi
        return r.result.F_tot, frc.total_forces(sysm, r.result.nhat)

    frames = omd.velocity_verlet(cell.positions, v0, masses, dt, n_steps, energy_forces)
    assert len(frames) == n_steps + 1 and len(recs) == n_steps
    for k, (x, v, e_cons) in enumerate(recs, start=1):
        fr = frames[k]
        assert np.max(np.abs(x - fr.positions)) < 1e-9, (k, np.max(np.abs(x - fr.positions)))
        assert np.max(np.abs(v - fr.velocities)) < 1e-9 / dt, k
        e_ref = fr.F_tot + fr.kinetic
        assert abs(e_cons - e_ref) <= 1e-10 * abs(e_ref), (k, e_cons, e_ref)

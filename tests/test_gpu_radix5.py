"""Grids with a factor 5 (radix-5 Stockham stages) and lengths above 256: the sizes of the
paper's largest fcc-Al cells (Sec. VI A: 32 000 ions, 20^3 conventional cells, and 62 500
ions, 25^3 cells, on 320^3 and 400^3 grids at 16 points per cell edge).

Small grids run every pass (plane passes for square (i2, i3) planes up to 128, row, x2 and
x1 passes otherwise) against the FP64 oracle point by point; lengths 320 and 400 sit on one
axis at a time so the oracle stays small.  At full size a density with the period of one
conventional cell makes the supercell's evaluation exactly n_rep^3 times the single cell's,
so the oracle's one-cell evaluation checks the 32 000- and 62 500-ion evaluations, and the
tiled symmetric one-cell minimum is the supercell's minimum (zero forces, isotropic stress)."""
import numpy as np
import pytest

import oracle
import workloads as wl

from _gpu_common import (assert_potential, fcc_al_symmetric_minimum, make_ctx, make_pair, normalized_phi,
                         oracle_system, rel)
from paper_1406_0835_amd import binding as B

pytestmark = pytest.mark.gpu

COMPONENTS = [("F_total", "F_tot"), ("F_s", "F_s"), ("TS_s", "TS_s"), ("E_xc", "E_xc"), ("E_H", "E_H"),
              ("E_ext", "E_ext"), ("E_alphaZ", "E_alphaZ"), ("E_ion", "E_ion"), ("N_e", "N_e"), ("mu", "mu")]
AL_FP64_V_TOL = 1e-9   # the oracle's own rounding at t ~ 7e-4 (see test_gpu_al.py)


# The mixed path's FP32 potential error grows as the grid spacing shrinks (the gradient and
# divergence terms weight the spectrum by G^2: RMS 1.7e-6 of the RMS potential at h = 0.16 bohr,
# 8e-6 at 0.08, 2.2e-5 at 0.04, measured on radix-2, -3 and -5 grids alike), so every axis keeps
# the spacing of the workloads instead of a cubic cell squeezed onto a long axis.


@pytest.mark.parametrize("shape", [
    (20, 20, 20), (20, 40, 40), (12, 80, 80), (40, 20, 80), (80, 40, 20), (8, 160, 12), (8, 8, 320),
    (400, 8, 8), (8, 400, 8), (8, 192, 40),
])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_radix5_and_long_axes_match_oracle(shape, precision):
    cell = wl.h_cell_spaced(shape, seed=1300 + sum(shape))
    ctx, sysm = make_pair(cell, "VT84F", precision=precision)
    phi = normalized_phi(sysm, seed=13, contrast=0.6)
    ctx.set_density(phi)
    rep, v = ctx.eval(potential=True)
    ev = oracle.evaluate(phi, sysm)
    tol = 1e-10 if precision == "fp64" else 1e-6
    # mixed: the FP32 grid arithmetic resolves energies to a fraction of the scale of the terms
    # (here F_tot ~ 0.08 and E_ext ~ 3e-4 beside terms of order 1), so each energy is held to
    # tol times the sum of the terms' magnitudes; N_e and mu to their own size
    S = sum(abs(getattr(ev, k)) for k in ("F_s", "E_xc", "E_H", "E_ext", "E_alphaZ", "E_ion"))
    for a, b in COMPONENTS:
        got, ref = getattr(rep, a), getattr(ev, b)
        own = max(abs(ref), 1e-3 * abs(ev.F_tot))
        scale = own if (precision == "fp64" or a in ("N_e", "mu")) else S
        assert abs(got - ref) <= tol * scale, (shape, a, got, ref)
    assert_potential(v, ev.v, precision)


def test_radix5_minimisation_and_forces_match_oracle():
    from oracle import forces as frc
    from oracle import minimize as mn
    cell = wl.h_cell(5, 1.0, (20, 40, 40), 5e4, seed=1390)
    ctx, sysm = make_pair(cell, "VT84F", tol_energy=1e-12, tol_residual=1e-8, cg_precond=8.0)
    rep = ctx.minimize_density()
    F, _, f = ctx.free_energy_and_forces()
    r = mn.minimize_cg(sysm, tol_energy=1e-12, tol_residual=1e-8, max_iter=3000)
    assert rep.converged and rel(F, r.result.F_tot) < 1e-10
    assert np.max(np.abs(f - frc.total_forces(sysm, r.result.nhat))) < 1e-7


def test_grid_sizes_outside_the_supported_set_are_refused():
    for bad in (10, 36, 100, 480, 512):
        ctx = B.Context(functional="VT84F")
        with pytest.raises(B.OFDFTError) as e:
            ctx.set_cell(np.eye(3) * 8.0, (bad, 16, 16))
        assert e.value.code == B.E_GRID
        ctx.close()


@pytest.mark.parametrize("n_rep", [20, 25])
def test_large_fcc_al_cells_tiled_evaluation_and_symmetric_minimum(n_rep):
    """32 000 ions on 320^3 and 62 500 ions on 400^3, FP64."""
    one = wl.fcc_al_cell(1, 16)
    s1 = oracle_system(one, "VT84F", lpp=wl.AL_HA_LPP)
    phi1 = normalized_phi(s1, seed=43, contrast=0.4)
    ev = oracle.evaluate(phi1, s1)
    cell = wl.fcc_al_cell(n_rep, 16 * n_rep)
    k = n_rep ** 3
    ctx = make_ctx(cell, "VT84F", precision="fp64", lpp=wl.AL_HA_LPP, tol_energy=1e-10 * cell.nat, cg_precond=8.0)
    ctx.set_density(np.tile(phi1, (n_rep,) * 3))
    rep, v = ctx.eval(potential=True)
    print(n_rep, "tiled evaluation", rep.F_total / k, ev.F_tot, flush=True)
    for a, b in [("F_total", "F_tot"), ("F_s", "F_s"), ("E_xc", "E_xc"), ("E_H", "E_H"), ("E_ext", "E_ext"),
                 ("E_ion", "E_ion")]:
        assert abs(getattr(rep, a) / k - getattr(ev, b)) <= 1e-10 * max(abs(getattr(ev, b)), 1e-3 * abs(ev.F_tot)), a
    assert abs(rep.mu - ev.mu) <= 1e-10 * abs(ev.mu)
    assert_potential(v, np.tile(ev.v, (n_rep,) * 3), "fp64", fp64_tol=AL_FP64_V_TOL)
    del v
    rep1, phi_sym, s_one = fcc_al_symmetric_minimum()
    ctx.set_density(np.tile(phi_sym, (n_rep,) * 3))
    rep = ctx.minimize_density(check=False)
    print(n_rep, "tiled symmetric start", ctx.last_rc, rep.iterations, rep.evaluations, rep.F_total / cell.nat,
          rep1.F_total / one.nat, flush=True)
    assert ctx.last_rc == B.OK
    assert rel(rep.F_total / cell.nat, rep1.F_total / one.nat) <= 1e-10
    _, _, f = ctx.free_energy_and_forces()
    sig = ctx.stress()
    ctx.close()
    d = np.diag(sig)
    print(n_rep, np.max(np.abs(f)), np.diag(sig), np.diag(s_one), flush=True)
    assert f.shape == (cell.nat, 3) and np.max(np.abs(f)) < 1e-6
    assert np.max(np.abs(sig - s_one)) <= 1e-8 * abs(d.mean())

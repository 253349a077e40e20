"""Shared helpers of the GPU tests: build a library context and the matching oracle system."""
import numpy as np

import oracle
import workloads as wl
from paper_1406_0835_amd import binding as B


def make_ctx(cell, functional="TF", precision="fp64", minimizer="cg", xc="PZ81", lpp=None, tol_energy=1e-10,
             tol_residual=0.0, max_iter=2000, mu_sga=5.0 / 27.0, cg_precond=0.0):
    lpp = lpp or {"kind": "gauss", "rc": 0.5}
    kw = dict(functional=functional, precision=precision, minimizer=minimizer, xc=xc.lower(),
              lpp_rc=lpp["rc"], tol_energy=tol_energy, tol_residual=tol_residual, max_iter=max_iter,
              cg_precond=cg_precond,
              mu_sga=mu_sga)
    if lpp["kind"] == "ha":
        kw.update(lpp="ha", lpp_A=lpp["A"], lpp_qc=lpp["qc"])
    ctx = B.Context(**kw)
    ctx.set_cell(cell.lattice, cell.grid)
    ctx.set_ions(cell.positions, cell.charges)
    ctx.set_temperature(cell.temperature_K)
    return ctx


def fcc_al_symmetric_minimum(precision="fp64", rounds=80):
    """The minimum of one conventional fcc-Al cell (4 ions, 16^3, VT84F, HA LPP, 100 K) over
    densities with the lattice's symmetry: CG runs of at most 25 iterations, each followed by
    the projection onto symmetric amplitudes (wl.fcc_symmetrize), until F changes by less
    than 1e-14 relative.  Returns the report, the amplitude and the stress (after a last,
    converged CG run from the projected density).  Unconstrained runs leave the symmetric
    densities at the ion-site points, where the 100 K density vanishes and F is not convex."""
    cell = wl.fcc_al_cell(1, 16)
    c = make_ctx(cell, "VT84F", precision=precision, lpp=wl.AL_HA_LPP, tol_energy=1e-14, max_iter=25,
                 cg_precond=8.0)
    F_prev = None
    for _ in range(rounds):
        c.minimize_density(check=False)
        c.set_density(wl.fcc_symmetrize(c.get_density()))
        rep = c.eval()
        if F_prev is not None and abs(rep.F_total - F_prev) <= 1e-14 * abs(F_prev):
            break
        F_prev = rep.F_total
    phi = c.get_density()
    c.minimize_density()
    sig = c.stress()
    c.close()
    return rep, phi, sig


def oracle_system(cell, functional="TF", xc="PZ81", lpp=None, mu_sga=5.0 / 27.0):
    lpp = lpp or {"kind": "gauss", "rc": 0.5}
    return oracle.System(cell.lattice, cell.grid, cell.positions, cell.charges, cell.temperature_K,
                         functional=functional, xc=xc.upper() if xc.upper() != "NONE" else "NONE", lpp=lpp,
                         mu_sga=mu_sga)


def make_pair(cell, functional="TF", precision="fp64", minimizer="cg", xc="PZ81", lpp=None, tol_energy=1e-10,
              tol_residual=0.0, max_iter=2000, mu_sga=5.0 / 27.0, cg_precond=0.0):
    ctx = make_ctx(cell, functional, precision, minimizer, xc, lpp, tol_energy, tol_residual, max_iter, mu_sga,
                   cg_precond)
    return ctx, oracle_system(cell, functional, xc, lpp, mu_sga)


def normalized_phi(sysm, seed, contrast=0.5):
    g = sysm.grid
    phi = wl.trial_phi(g.shape, sysm.n_electrons / g.volume, seed=seed, contrast=contrast)
    return phi * np.sqrt(sysm.n_electrons / (g.dv * np.sum(phi * phi)))


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def assert_pointwise(v, v_ref, tol):
    """|v - v_ref| <= tol * max|v_ref| at every grid point (reports the worst point)."""
    v = np.asarray(v)
    v_ref = np.asarray(v_ref)
    assert v.shape == v_ref.shape, (v.shape, v_ref.shape)
    diff = np.abs(v - v_ref)
    scale = float(np.max(np.abs(v_ref)))
    worst = int(np.argmax(diff))
    err = float(diff.flat[worst]) / scale
    assert err <= tol, (f"max |v - v_ref| = {err:.3e} of max|v_ref| at flat index {worst} "
                        f"(v = {v.flat[worst]!r}, v_ref = {v_ref.flat[worst]!r}); tolerance {tol:.1e}")


# Potential tolerances.  FP64: every point within 1e-10 of max|v_ref|.  Mixed (FP32 FFTs and
# gradient terms): the RMS error within 1e-5 of the RMS, and every point within 5e-5 of
# max|v_ref|.  The pointwise bound is ~800 FP32 roundings (u = 6e-8): the three-pass FFTs
# add ~log2(N) roundings of the largest term at every point, and the divergence of W and
# df/dn cancel to a few per cent of their size at the worst points.
def assert_potential(v, v_ref, precision, fp64_tol=1e-10):
    if precision == "fp64":
        assert_pointwise(v, v_ref, fp64_tol)
    else:
        assert_pointwise(v, v_ref, 5e-5)
        rms = float(np.sqrt(np.mean((np.asarray(v) - v_ref) ** 2)) / np.sqrt(np.mean(np.asarray(v_ref) ** 2)))
        assert rms <= 1e-5, f"RMS error {rms:.3e} of the RMS potential; tolerance 1e-5"

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

#!/usr/bin/env python3
"""Write converged reference results of the CPU oracle for the GPU parity tests.

Calls only oracle/ (and the seeded input generators in workloads/).  Targets:
  c1   16 H, 1.0 g/cm^3, 32^3, 10 kK, ftTF + PZ81, Gaussian LPP rc = 0.5
  c2   128 H, 2.0 g/cm^3, 64^3, VT84F + PZ81, T = 2 kK, 50 kK, 1 MK
Each file holds F_tot and its components, mu, and the forces at the minimum,
with the oracle minimised until |dF| < 1e-12 Ha twice and the density-weighted
potential residual is below the stated value.
  c3eval_<functional>_<T>   1024 H, 4.0 g/cm^3, 128^3: one evaluation at the
       seeded benchmark phi (no minimisation): energy components and the
       potential at 4096 seeded sample points.
  al1_sym   fcc Al, one conventional cell (4 ions, 2.7 g/cm^3, 16^3, 100 K), VT84F
       + PZ81, HA local pseudopotential: the minimum over densities with the
       lattice's symmetry (the amplitude and the gradient projected after every
       CG step onto functions invariant under the fcc translations and the
       inversion through an ion).  Unconstrained runs leave this subspace at the
       four ion-site grid points, where the 100 K density vanishes and F is not
       convex in phi; the projection removes that freedom.

Usage: python tests/golden/make_golden.py c1 [c2_2000 c2_50000 c2_1000000] [c3eval_VT84F_100000] [al1_sym]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as wl  # noqa: E402
from oracle import forces as frc  # noqa: E402
from oracle import minimize as mn  # noqa: E402


C3_SAMPLE_SEED = 1406_77


def run_c3eval(name):
    _, functional, T = name.split("_")
    cell = wl.gga_128_cell(float(T))
    sysm = oracle.System(cell.lattice, cell.grid, cell.positions, cell.charges, cell.temperature_K,
                         functional=functional)
    nbar = cell.nat / sysm.grid.volume
    phi = wl.trial_phi(cell.grid, nbar, seed=wl.SEED_BASE + 2, contrast=0.6)
    phi *= np.sqrt(sysm.n_electrons / (sysm.grid.dv * np.sum(phi * phi)))
    t0 = time.time()
    ev = oracle.evaluate(phi, sysm)
    rng = np.random.Generator(np.random.PCG64(C3_SAMPLE_SEED))
    idx = rng.integers(0, sysm.grid.N, size=4096)
    out = {
        "target": name, "functional": functional, "temperature_K": cell.temperature_K,
        "grid": list(cell.grid), "nat": cell.nat, "seed": cell.seed, "phi_seed": wl.SEED_BASE + 2,
        "phi_contrast": 0.6, "sample_seed": C3_SAMPLE_SEED,
        "F_tot": ev.F_tot, "F_s": ev.F_s, "TS_s": ev.TS_s, "E_xc": ev.E_xc, "E_H": ev.E_H, "E_ext": ev.E_ext,
        "E_alphaZ": ev.E_alphaZ, "E_ion": ev.E_ion, "mu": ev.mu, "N_e": ev.N_e,
        "v_rms": float(np.sqrt(np.mean(ev.v ** 2))),
        "sample_index": idx.tolist(), "v_sample": ev.v.ravel()[idx].tolist(), "seconds": time.time() - t0,
        "source": "oracle.energy.evaluate",
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(out, fh)
    print("wrote", name, out["F_tot"], out["seconds"])


def run_al1_sym(name):
    cell = wl.fcc_al_cell(1, 16)
    sysm = oracle.System(cell.lattice, cell.grid, cell.positions, cell.charges, cell.temperature_K,
                         functional="VT84F", lpp=wl.AL_HA_LPP)

    def project(i, phi, ev):
        phi[...] = wl.fcc_symmetrize(phi)
        ev.grad[...] = wl.fcc_symmetrize(ev.grad)

    t0 = time.time()
    r = mn.minimize_cg(sysm, tol_energy=1e-14, tol_residual=1e-8, max_iter=2000, callback=project)
    ev = oracle.evaluate(r.phi, sysm)
    F = frc.total_forces(sysm, ev.nhat)
    out = {
        "target": name, "functional": "VT84F", "lpp": "HA", "temperature_K": cell.temperature_K,
        "grid": list(cell.grid), "nat": cell.nat, "rho_gcc": cell.rho_gcc,
        "converged": bool(r.converged), "iterations": r.iterations, "residual": ev.residual(r.phi),
        "F_tot": ev.F_tot, "F_per_ion": ev.F_tot / cell.nat, "F_s": ev.F_s, "E_xc": ev.E_xc, "E_H": ev.E_H,
        "E_ext": ev.E_ext, "E_ion": ev.E_ion, "mu": ev.mu, "max_abs_force": float(np.max(np.abs(F))),
        "seconds": time.time() - t0,
        "source": "oracle.minimize.minimize_cg (projected onto fcc-symmetric amplitudes) + oracle.forces",
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", name, out["F_per_ion"], out["residual"], out["seconds"])


def run(name):
    if name.startswith("c3eval_"):
        return run_c3eval(name)
    if name == "al1_sym":
        return run_al1_sym(name)
    if name == "c1":
        cell = wl.small_tf_cell()
        functional = "TF"
    elif name.startswith("c2_"):
        cell = wl.gga_64_cell(float(name[3:]))
        functional = "VT84F"
    else:
        raise SystemExit(f"unknown target {name}")
    sysm = oracle.System(cell.lattice, cell.grid, cell.positions, cell.charges, cell.temperature_K,
                         functional=functional)
    t0 = time.time()
    tol_res = 1e-8
    r = mn.minimize_cg(sysm, tol_energy=1e-12, tol_residual=tol_res, max_iter=3000,
                       callback=lambda i, p, e: print(name, i, e.F_tot, e.residual(p), flush=True)
                       if i % 20 == 0 else None)
    ev = r.result
    F = frc.total_forces(sysm, ev.nhat)
    out = {
        "target": name, "functional": functional, "temperature_K": cell.temperature_K,
        "grid": list(cell.grid), "nat": cell.nat, "seed": cell.seed, "rho_gcc": cell.rho_gcc,
        "converged": bool(r.converged), "iterations": r.iterations, "evaluations": r.evaluations,
        "residual": ev.residual(r.phi), "F_tot": ev.F_tot, "F_s": ev.F_s, "TS_s": ev.TS_s, "E_xc": ev.E_xc,
        "E_H": ev.E_H, "E_ext": ev.E_ext, "E_alphaZ": ev.E_alphaZ, "E_ion": ev.E_ion, "mu": ev.mu,
        "E_internal": ev.E_internal, "forces": F.tolist(), "seconds": time.time() - t0,
        "source": "oracle.minimize.minimize_cg + oracle.forces.total_forces",
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", name, out["F_tot"], out["residual"], out["seconds"])


if __name__ == "__main__":
    for n in sys.argv[1:]:
        run(n)

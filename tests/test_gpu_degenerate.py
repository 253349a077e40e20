"""Degenerate densities through the C ABI against the FP64 oracle (Sec. III A/B: the functionals
at zero gradient and at the density floor).

* A uniform amplitude: grad n = 0 at every point, so s = 0 and every enhancement factor takes
  its s -> 0 value (the small-x branch of Eq. VT84F); the G = 0 term is excluded from the
  Hartree and pseudopotential sums, so E_H vanishes up to the FFT's rounding.  At s = 0 every
  GGA of Table I reduces to ftTF, so the seven functionals give one free energy and one
  potential.
* An empty slab: phi = 0 exactly on four i1 planes, so n is held at the density floor there
  and the reduced gradient of the spectral grad n is huge next to the slab.  ftTF and the
  enhancement factors that stay bounded at large s (KST2, TW, APBEF) give O(1) energies; the
  forms that grow with s^2 (SGA, VWTF, VT84F) give energies of order 1e11 Ha from the floored
  points, the same on both sides.
Tolerances are those of the evaluation parity tests: FP64 1e-10 relative per component and
1e-10 of max|v| at every point; mixed 1e-6 and the mixed potential bounds."""
import numpy as np
import pytest

import oracle
import workloads as wl

from _gpu_common import assert_potential, make_pair

pytestmark = pytest.mark.gpu

FUNCTIONALS = ["TF", "SGA", "VT84F", "KST2", "VWTF", "TW", "APBEF"]
COMPONENTS = [("F_total", "F_tot"), ("F_s", "F_s"), ("TS_s", "TS_s"), ("E_xc", "E_xc"), ("E_H", "E_H"),
              ("E_ext", "E_ext"), ("N_e", "N_e"), ("mu", "mu")]


def _cell():
    return wl.h_cell(3, 1.0, (12, 12, 12), 3e4, seed=611)


def _uniform(sysm):
    g = sysm.grid
    return np.full(g.shape, np.sqrt(sysm.n_electrons / g.volume))


def _slab(sysm):
    g = sysm.grid
    f = wl.smooth_field(g.shape, 8, seed=612)
    phi = np.sqrt(sysm.n_electrons / g.volume * (1.0 + 0.5 * f))
    phi[4:8] = 0.0
    return phi * np.sqrt(sysm.n_electrons / (g.dv * np.sum(phi * phi)))


def _check(ctx, sysm, phi, precision):
    ctx.set_density(phi)
    rep, v = ctx.eval(potential=True)
    ev = oracle.evaluate(phi, sysm)
    tol = 1e-10 if precision == "fp64" else 1e-6
    for a, b in COMPONENTS:
        got, ref = getattr(rep, a), getattr(ev, b)
        scale = max(abs(ref), 1e-3 * abs(ev.F_tot))
        assert np.isfinite(got) and abs(got - ref) <= tol * scale, (a, got, ref)
    assert np.all(np.isfinite(v))
    assert_potential(v, ev.v, precision)
    return rep, v


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_uniform_density_matches_oracle_and_every_gga_reduces_to_fttf(precision):
    cell = _cell()
    results = []
    for fn in FUNCTIONALS:
        ctx, sysm = make_pair(cell, fn, precision=precision)
        rep, v = _check(ctx, sysm, _uniform(sysm), precision)
        assert abs(rep.E_H) <= 1e-12 * abs(rep.F_total)   # rounding residue of the FFT of a constant
        results.append((rep.F_total, v))
        ctx.close()
    F0, v0 = results[0]
    tol = 1e-12 if precision == "fp64" else 1e-6
    for fn, (F, v) in zip(FUNCTIONALS[1:], results[1:]):
        assert abs(F - F0) <= tol * abs(F0), (fn, F, F0)
        assert np.max(np.abs(v - v0)) <= tol * np.max(np.abs(v0)), fn


@pytest.mark.parametrize("precision,functional", [(p, f) for p in ("fp64", "mixed") for f in FUNCTIONALS
                                                  if p == "fp64" or f in ("TF", "KST2", "TW", "APBEF")])
def test_empty_slab_matches_oracle(precision, functional):
    ctx, sysm = make_pair(_cell(), functional, precision=precision)
    rep, _ = _check(ctx, sysm, _slab(sysm), precision)
    if functional in ("SGA", "VWTF", "VT84F"):
        assert rep.F_total > 1e9   # the floored points dominate, as in the oracle
    ctx.close()

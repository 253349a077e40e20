"""GPU evaluation parity: the HIP path (through the C ABI) against the FP64 oracle.

One F[n] + gradient evaluation at the same seeded phi: every energy component
and the potential on every grid point.  FP64 path: 1e-10 relative, and at every
grid point |v - v_oracle| <= 1e-10 max|v_oracle|.  Mixed path (FP32 FFTs and
gradient terms, FP64 Fermi-Dirac inversion and sums): 1e-6 relative in F_tot,
the potential's RMS error within 1e-5 of its RMS and every point within 5e-5 of
max|v_oracle| (the bounds of _gpu_common.assert_potential).
"""
import numpy as np
import pytest

import oracle
import workloads as wl

from _gpu_common import assert_potential, make_pair, normalized_phi, rel

pytestmark = pytest.mark.gpu

COMPONENTS = [("F_total", "F_tot"), ("F_s", "F_s"), ("TS_s", "TS_s"), ("E_xc", "E_xc"), ("E_H", "E_H"),
              ("E_ext", "E_ext"), ("E_alphaZ", "E_alphaZ"), ("E_ion", "E_ion"), ("N_e", "N_e"), ("mu", "mu")]


def _compare(ctx, sysm, phi, tol_e, precision="fp64"):
    ctx.set_density(phi)
    rep, v = ctx.eval(potential=True)
    ev = oracle.evaluate(phi, sysm)
    for a, b in COMPONENTS:
        got, ref = getattr(rep, a), getattr(ev, b)
        scale = max(abs(ref), 1e-3 * abs(ev.F_tot))
        assert abs(got - ref) <= tol_e * scale, (a, got, ref)
    assert_potential(v, ev.v, precision)
    return rep, ev, v


CASES = [
    ("TF", (12, 12, 12), 2), ("TF", (16, 24, 8), 3), ("SGA", (16, 16, 16), 3), ("VT84F", (12, 16, 24), 4),
    ("KST2", (16, 16, 16), 2), ("VWTF", (12, 12, 12), 2), ("TW", (8, 8, 8), 2), ("APBEF", (12, 12, 12), 2),
]


@pytest.mark.parametrize("functional,shape,nat", CASES)
def test_eval_fp64_matches_oracle(functional, shape, nat):
    cell = wl.h_cell(nat, 1.0, shape, 3e4, seed=500 + nat)
    ctx, sysm = make_pair(cell, functional)
    phi = normalized_phi(sysm, seed=nat)
    _compare(ctx, sysm, phi, 1e-10)


@pytest.mark.parametrize("T_K", [2e3, 5e4, 1e6, 4e6])
def test_eval_fp64_temperature_range(T_K):
    cell = wl.h_cell(4, 2.0, (16, 16, 16), T_K, seed=600)
    ctx, sysm = make_pair(cell, "VT84F")
    phi = normalized_phi(sysm, seed=7, contrast=0.8)
    _compare(ctx, sysm, phi, 1e-10)


def test_eval_fp64_triclinic_cell_and_ha_pseudopotential():
    cell = wl.h_cell(3, 1.0, (12, 16, 12), 5e4, seed=601)
    cell.lattice = np.array([[4.2, 0.0, 0.0], [0.9, 4.6, 0.0], [0.4, -0.7, 5.1]])
    cell.positions = np.random.default_rng(1).random((3, 3)) @ cell.lattice
    lpp = {"kind": "ha", "rc": 0.25, "A": 6.18, "qc": 29.97}
    ctx, sysm = make_pair(cell, "SGA", lpp=lpp)
    _compare(ctx, sysm, normalized_phi(sysm, seed=3), 1e-10)


def test_eval_without_xc():
    cell = wl.h_cell(2, 1.0, (12, 12, 12), 1e5, seed=602)
    ctx, sysm = make_pair(cell, "VT84F", xc="NONE")
    _compare(ctx, sysm, normalized_phi(sysm, seed=5), 1e-10)


@pytest.mark.parametrize("functional,T_K,precision", [
    ("TF", 1e4, "fp64"), ("VT84F", 2e3, "fp64"), ("VT84F", 5e4, "fp64"), ("SGA", 1e6, "fp64"),
    ("VT84F", 4e6, "fp64"), ("VT84F", 5e4, "mixed"), ("TF", 1e6, "mixed"),
])
def test_eval_ksdt_matches_oracle(functional, T_K, precision):
    """The finite-T LDA XC of Sec. IV A (Eq. fit2, potential Eq. vxc1) in place of PZ81:
    energies, T S_xc, the internal energy and the potential at every point."""
    # the mixed path's 1e-6 is relative to F: its cell (16 H on 32^3) has a free energy that
    # is not a near cancellation of its terms, unlike the small FP64 cell (F ~ 1e-3 Ha)
    cell = (wl.h_cell(4, 1.0, (16, 16, 16), T_K, seed=610) if precision == "fp64"
            else wl.h_cell(16, 1.0, (32, 32, 32), T_K, seed=603))
    ctx, sysm = make_pair(cell, functional, precision=precision, xc="KSDT")
    phi = normalized_phi(sysm, seed=13, contrast=0.7)
    tol = 1e-10 if precision == "fp64" else 1e-6
    rep, ev, _ = _compare(ctx, sysm, phi, tol, precision)
    assert ev.TS_xc != 0.0
    assert abs(rep.TS_xc - ev.TS_xc) <= tol * max(abs(ev.TS_xc), 1e-3 * abs(ev.F_tot))
    # E_internal = F + T S_s + T S_xc carries F's absolute error; scale it as F's
    assert abs(rep.E_internal - ev.E_internal) <= tol * max(abs(ev.E_internal), abs(ev.F_tot))


def test_ksdt_minimisation_matches_oracle():
    """Converged FP64 density with KSDT (ftTF, 8 H on 16^3 at 10 kK) against the oracle's CG."""
    from oracle import minimize as om
    cell = wl.h_cell(8, 1.0, (16, 16, 16), 1e4, seed=611)
    ctx, sysm = make_pair(cell, "TF", xc="KSDT", tol_energy=1e-12, tol_residual=1e-9)
    rep = ctx.minimize_density()
    res = om.minimize_cg(sysm, tol_energy=1e-12, tol_residual=1e-9)
    assert rep.converged and res.converged
    assert rel(rep.F_total, res.result.F_tot) <= 1e-10
    assert rel(rep.E_internal, res.result.E_internal) <= 1e-10
    _, _, f = ctx.free_energy_and_forces()
    from oracle import forces as ofo
    f_ref = ofo.total_forces(sysm, res.result.nhat)
    assert np.max(np.abs(f - f_ref)) <= 1e-7


@pytest.mark.parametrize("functional", ["TF", "VT84F", "SGA"])
def test_eval_mixed_precision(functional):
    cell = wl.h_cell(16, 1.0, (32, 32, 32), 5e4, seed=603)
    ctx, sysm = make_pair(cell, functional, precision="mixed")
    _compare(ctx, sysm, normalized_phi(sysm, seed=9), 1e-6, "mixed")


def test_eval_is_deterministic():
    cell = wl.h_cell(4, 1.0, (16, 16, 16), 5e4, seed=604)
    ctx, sysm = make_pair(cell, "VT84F")
    ctx.set_density(normalized_phi(sysm, seed=2))
    r1, v1 = ctx.eval(potential=True)
    r2, v2 = ctx.eval(potential=True)
    assert r1.F_total == r2.F_total
    assert np.array_equal(v1, v2)


@pytest.mark.parametrize("precision,functional", [("fp64", "VT84F"), ("mixed", "VT84F"), ("fp64", "TF")])
def test_fft_tiles_do_not_change_results(precision, functional):
    """Every tile choice (rows/columns per workgroup of the three FFT passes, including
    tiles with 1, 2, 4 and 8 staged elements per thread) gives the same evaluation; the
    oracle pins the default tiles."""
    cell = wl.h_cell(6, 2.0, (32, 32, 32), 5e4, seed=605)
    ctx, sysm = make_pair(cell, functional, precision=precision)
    phi = normalized_phi(sysm, seed=11)
    ctx.set_density(phi)
    tol_e, tol_v = (1e-10, 1e-10) if precision == "fp64" else (1e-6, 1e-5)
    ev = oracle.evaluate(phi, sysm)
    rep0, v0 = ctx.eval(potential=True)
    assert rel(rep0.F_total, ev.F_tot) <= tol_e
    for tiles in [(2, 1, 1), (4, 2, 2), (8, 8, 8), (16, 16, 32), (32, 32, 64)]:
        ctx.set_tiles(tiles)
        rep, v = ctx.eval(potential=True)
        assert rel(rep.F_total, rep0.F_total) <= (1e-13 if precision == "fp64" else 1e-6), tiles
        assert np.max(np.abs(v - v0)) <= (1e-12 if precision == "fp64" else 1e-5) * np.max(np.abs(v0)), tiles
    tiles = ctx.autotune(2)
    rep, v = ctx.eval(potential=True)
    assert rel(rep.F_total, ev.F_tot) <= tol_e, tiles
    assert_potential(v, ev.v, precision)


@pytest.mark.parametrize("precision,functional,shape", [
    ("fp64", "VT84F", (16, 24, 24)), ("mixed", "VT84F", (12, 48, 48)), ("fp64", "TF", (8, 32, 32)),
    ("mixed", "SGA", (8, 96, 96)), ("mixed", "VT84F", (8, 128, 128)), ("fp64", "VT84F", (8, 128, 128)),
])
def test_plane_passes_match_row_passes(precision, functional, shape, monkeypatch):
    """Square (i2, i3) planes up to 128 run the x3 and x2 transforms as one plane pass
    per i1; with it switched off (row passes and a separate x2 pass) the evaluation, a
    line-search trial and the forces agree, and the oracle pins the plane path."""
    fp64 = precision == "fp64"
    # mixed: the two paths round differently, so they agree only to the mixed path's own error,
    # which on a cubic 4-atom cell squeezed onto 8 x 128 x 128 points (0.034 bohr along two axes)
    # reaches 2e-4 of max|v| (the G^2 weight of the gradient terms); its cells keep 0.15 bohr
    cell = wl.h_cell(4, 1.0, shape, 5e4, seed=606) if fp64 else wl.h_cell_spaced(shape, seed=606)
    # FP64 minimises to a residual target: two energy-stopped runs whose paths differ in
    # rounding stop up to ~1e-9 apart, a convergence difference and not a pass difference
    stop = dict(tol_energy=1e-12, tol_residual=1e-8) if fp64 else {}
    ctx, sysm = make_pair(cell, functional, precision=precision, **stop)
    monkeypatch.setenv("OFDFT_PLANE_PASSES", "0")
    ctx_row, _ = make_pair(cell, functional, precision=precision, **stop)
    monkeypatch.delenv("OFDFT_PLANE_PASSES")
    phi = normalized_phi(sysm, seed=12, contrast=0.6)
    tol_f, tol_v = (1e-12, 1e-11) if precision == "fp64" else (1e-6, 1e-5)
    ctx.set_density(phi)
    ctx_row.set_density(phi)
    rep, v = ctx.eval(potential=True)
    rep_r, v_r = ctx_row.eval(potential=True)
    for a, _ in COMPONENTS:
        got, ref = getattr(rep, a), getattr(rep_r, a)
        assert abs(got - ref) <= tol_f * max(abs(ref), 1e-3 * abs(rep_r.F_total)), (a, got, ref)
    assert np.max(np.abs(v - v_r)) <= tol_v * np.max(np.abs(v_r))
    if shape[1] <= 48:
        ev = oracle.evaluate(phi, sysm)
        assert rel(rep.F_total, ev.F_tot) <= (1e-10 if precision == "fp64" else 1e-6)
        assert_potential(v, ev.v, precision)
    # a minimisation (line-search trials, preconditioned directions) and the forces
    r1 = ctx.minimize_density()
    r2 = ctx_row.minimize_density()
    assert abs(r1.F_total - r2.F_total) <= (1e-11 if fp64 else 1e-5) * abs(r2.F_total)
    _, _, f1 = ctx.free_energy_and_forces()
    _, _, f2 = ctx_row.free_energy_and_forces()
    if fp64:
        assert np.max(np.abs(f1 - f2)) <= 1e-7
    else:
        # each mixed run carries its own force error of up to the mixed tolerance (1e-4
        # hartree/bohr): both are held to the FP64 minimum of the same cell
        ref, _ = make_pair(cell, functional, precision="fp64", tol_energy=1e-12, tol_residual=1e-8)
        ref.minimize_density()
        _, _, f64 = ref.free_energy_and_forces()
        assert np.max(np.abs(f1 - f64)) <= 1e-4
        assert np.max(np.abs(f2 - f64)) <= 1e-4


@pytest.mark.parametrize("functional,xc,shape,rho,T_K", [
    ("VT84F", "PZ81", (16, 32, 32), 4.0, 1e5), ("SGA", "NONE", (12, 32, 32), 2.0, 1e6),
    ("VT84F", "PZ81", (12, 64, 64), 2.0, 1e5), ("KST2", "PZ81", (8, 64, 64), 1.0, 5e4),
    ("VT84F", "NONE", (8, 128, 128), 1.0, 5e4), ("VT84F", "PZ81", (16, 128, 128), 2.0, 1e5),
])
def test_fused_gradient_pass_matches_separate_passes(functional, xc, shape, rho, T_K, monkeypatch):
    """Mixed precision on square planes of 32, 64 and 128 points runs the inverse gradient
    transforms and the pointwise functional as one plane pass (x2 split four ways over i2 mod 4),
    the final pass on the same split and the density pass split by the parity of k3; with them
    switched off (OFDFT_FUSED_GGA=0: whole-plane passes and the separate pointwise kernel) the
    evaluation agrees to the mixed path's rounding, and the oracle pins the split path on every
    grid point, including plane counts that are not multiples of 8 and the no-XC form.  The
    mixed path's 1e-6 is relative to F, so the cells are ones whose F is not a near
    cancellation of its terms (|F| at least half the largest component)."""
    cell = wl.h_cell_spaced(shape, seed=607, rho_gcc=rho, temperature_K=T_K)
    ctx, sysm = make_pair(cell, functional, precision="mixed", xc=xc)
    monkeypatch.setenv("OFDFT_FUSED_GGA", "0")
    ctx_sep, _ = make_pair(cell, functional, precision="mixed", xc=xc)
    monkeypatch.delenv("OFDFT_FUSED_GGA")
    phi = normalized_phi(sysm, seed=13, contrast=0.6)
    ctx.set_density(phi)
    ctx_sep.set_density(phi)
    rep, v = ctx.eval(potential=True)
    rep_s, v_s = ctx_sep.eval(potential=True)
    for a, _ in COMPONENTS:
        got, ref = getattr(rep, a), getattr(rep_s, a)
        assert abs(got - ref) <= 1e-6 * max(abs(ref), 1e-3 * abs(rep_s.F_total)), (a, got, ref)
    assert np.max(np.abs(v - v_s)) <= 1e-5 * np.max(np.abs(v_s))
    # against the oracle: what the fused pass forms (the free-energy density sums and, through
    # them, F and mu; the potential at every point).  E_H and E_ext come from the x1 pass before
    # it, unchanged, and are held to the separate passes above.
    ev = oracle.evaluate(phi, sysm)
    for a, b in [("F_total", "F_tot"), ("F_s", "F_s"), ("TS_s", "TS_s"), ("E_xc", "E_xc"), ("mu", "mu")]:
        got, ref = getattr(rep, a), getattr(ev, b)
        assert abs(got - ref) <= 1e-6 * max(abs(ref), 1e-3 * abs(ev.F_tot)), (a, got, ref)
    assert_potential(v, ev.v, "mixed")
    # bitwise repeatable: fixed block order of every sum
    rep2, v2 = ctx.eval(potential=True)
    assert rep2.F_total == rep.F_total and np.array_equal(v2, v)
    ctx.close()
    ctx_sep.close()

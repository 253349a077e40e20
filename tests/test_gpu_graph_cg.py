"""The HIP-graph CG (options.graph_cg = 1: every decision of an iteration on the device, the
iteration replayed as one captured graph) against the FP64 oracle, against the host-driven
CG, in a batch of heterogeneous cells driven by one host thread, and on its failure paths.
Converged results only: FP64 within 1e-10 in F and 1e-7 Ha/bohr in the forces, mixed within
1e-6 and 1e-4 (the iteration paths of the two minimisers differ)."""
import numpy as np
import pytest

import workloads as wl
from oracle import forces as frc
from oracle import minimize as mn
from paper_1406_0835_amd import binding as B

from _gpu_common import make_pair, oracle_system, rel

pytestmark = pytest.mark.gpu


def _graph_pair(cell, functional, precision="fp64", **kw):
    sysm = oracle_system(cell, functional, xc=kw.get("xc", "PZ81"))
    opts = dict(functional=functional, precision=precision, xc=kw.get("xc", "PZ81").lower(),
                tol_energy=kw.get("tol_energy", 1e-10), tol_residual=kw.get("tol_residual", 0.0),
                max_iter=kw.get("max_iter", 2000), cg_precond=kw.get("cg_precond", 0.0), graph_cg=1)
    g = B.Context(**opts)
    g.set_cell(cell.lattice, cell.grid)
    g.set_ions(cell.positions, cell.charges)
    g.set_temperature(cell.temperature_K)
    return g, sysm


@pytest.mark.parametrize("functional,precision,precond,shape", [
    ("TF", "fp64", 0.0, (16, 16, 16)), ("VT84F", "fp64", 8.0, (16, 16, 16)), ("SGA", "fp64", 0.0, (12, 16, 12)),
    ("VT84F", "mixed", 8.0, (24, 24, 24)),
])
def test_graph_cg_matches_oracle(functional, precision, precond, shape):
    cell = wl.h_cell(4, 1.0, shape, 5e4, seed=960)
    fp64 = precision == "fp64"
    ctx, sysm = _graph_pair(cell, functional, precision, tol_energy=1e-12 if fp64 else 1e-9,
                            tol_residual=1e-9 if fp64 else 0.0, cg_precond=precond)
    rep = ctx.minimize_density()
    F, _, f = ctx.free_energy_and_forces()
    r = mn.minimize_cg(sysm, tol_energy=1e-12, tol_residual=1e-9, max_iter=3000)
    assert rep.converged and rep.iterations > 0
    assert rel(F, r.result.F_tot) < (1e-10 if fp64 else 1e-6)
    assert np.max(np.abs(f - frc.total_forces(sysm, r.result.nhat))) < (1e-7 if fp64 else 1e-4)
    assert rep.N_e == pytest.approx(sysm.n_electrons, rel=1e-12)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_cg_reaches_the_host_cg_minimum(precision):
    """The 128-H, 64^3 VT84F cell at 50 kK (the MD workload's size): both minimisers stop at
    the same free energy."""
    cell = wl.gga_64_cell(5e4)
    fp64 = precision == "fp64"
    tol = 1e-10 if fp64 else 1e-8
    host, _ = make_pair(cell, "VT84F", precision=precision, tol_energy=tol, cg_precond=8.0)
    rh = host.minimize_density()
    graph, _ = _graph_pair(cell, "VT84F", precision, tol_energy=tol, cg_precond=8.0)
    rg = graph.minimize_density()
    print(precision, "host", rh.iterations, rh.evaluations, "graph", rg.iterations, rg.evaluations, flush=True)
    assert rel(rg.F_total, rh.F_total) < (1e-9 if fp64 else 1e-6)
    _, _, fh = host.free_energy_and_forces()
    _, _, fg = graph.free_energy_and_forces()
    if fp64:
        assert np.max(np.abs(fg - fh)) < 1e-6
    else:
        # each mixed result carries its own error of up to the 1e-4 mixed force tolerance:
        # both are compared with the FP64 minimum
        ref, _ = make_pair(cell, "VT84F", precision="fp64", tol_energy=1e-10, cg_precond=8.0)
        ref.minimize_density()
        _, _, f64 = ref.free_energy_and_forces()
        print("mixed force error host", np.max(np.abs(fh - f64)), "graph", np.max(np.abs(fg - f64)), flush=True)
        assert np.max(np.abs(fh - f64)) < 1e-4
        assert np.max(np.abs(fg - f64)) < 1e-4
    # a warm start from the converged density stays there
    rg2 = graph.minimize_density()
    assert rg2.converged and rel(rg2.F_total, rg.F_total) < (1e-9 if fp64 else 1e-6)


def test_graph_batch_matches_oracle_cell_by_cell():
    """Six cells of different grids, ion counts, densities and temperatures minimised together
    by one host thread (each cell's captured iteration on its own stream): each cell's
    converged F and forces against the oracle's minimisation of that cell."""
    specs = [(3, 1.0, (16, 16, 16), 2e3), (5, 2.0, (16, 16, 16), 5e4), (2, 0.6, (12, 12, 12), 1e6),
             (6, 3.0, (24, 24, 24), 1e5), (4, 1.5, (16, 24, 16), 4e6), (3, 0.8, (12, 16, 12), 1e4)]
    ctxs, systems = [], []
    for k, (nat, rho, grid, T) in enumerate(specs):
        cell = wl.h_cell(nat, rho, grid, T, seed=970 + k)
        fn = "VT84F" if k % 2 == 0 else "TF"
        c, s = _graph_pair(cell, fn, "fp64", tol_energy=1e-12, tol_residual=1e-9, cg_precond=8.0 if fn != "TF" else 0.0)
        ctxs.append(c)
        systems.append(s)
    reps = B.batch_minimize(ctxs)
    for c, s, rep in zip(ctxs, systems, reps):
        assert rep.converged
        F, _, f = c.free_energy_and_forces()
        r = mn.minimize_cg(s, tol_energy=1e-12, tol_residual=1e-9, max_iter=3000)
        assert rel(F, r.result.F_tot) < 1e-10, (c.shape, F, r.result.F_tot)
        assert np.max(np.abs(f - frc.total_forces(s, r.result.nhat))) < 1e-7


def test_graph_batch_equals_one_after_another():
    cells = wl.batch_cells(8, grids=(16, 24, 32))
    def build():
        out = []
        for cell in cells:
            c, _ = _graph_pair(cell, "VT84F", "mixed", tol_energy=1e-8, cg_precond=8.0)
            out.append(c)
        return out
    batch = build()
    reps = B.batch_minimize(batch)
    seq = build()
    for c, rb in zip(seq, reps):
        rs = c.minimize_density()
        # the same captured iteration on the same inputs: the same path and result
        assert rs.F_total == rb.F_total and rs.iterations == rb.iterations


def test_graph_cg_max_iter_and_nonfinite_recovery(monkeypatch):
    cell = wl.h_cell(16, 1.0, 32, 5e4, seed=980)
    ctx, _ = _graph_pair(cell, "VT84F", "fp64", tol_energy=1e-10, max_iter=3, cg_precond=8.0)
    F0 = ctx.eval().F_total
    rep = ctx.minimize_density(check=False)
    assert ctx.last_rc == B.E_NOT_CONVERGED and rep.iterations == 3 and rep.F_total < F0
    ref, _ = _graph_pair(cell, "VT84F", "fp64", tol_energy=1e-10, cg_precond=8.0)
    F_ref = ref.minimize_density().F_total
    monkeypatch.setenv("OFDFT_TEST_NONFINITE", "2")
    one, _ = _graph_pair(cell, "VT84F", "fp64", tol_energy=1e-10, cg_precond=8.0)
    monkeypatch.setenv("OFDFT_TEST_NONFINITE", "-1")
    every, _ = _graph_pair(cell, "VT84F", "fp64", tol_energy=1e-10, cg_precond=8.0)
    monkeypatch.delenv("OFDFT_TEST_NONFINITE")
    r1 = one.minimize_density()
    assert r1.converged and rel(r1.F_total, F_ref) < 1e-9
    F0 = every.eval().F_total
    r2 = every.minimize_density(check=False)
    assert every.last_rc == B.E_NONFINITE and r2.F_total == pytest.approx(F0, rel=1e-13)


def test_c4_batch_of_64_cells_against_fp64_cell_by_cell():
    """The C4 workload itself: 64 heterogeneous cells (16-256 H, grids 32^3-96^3, 0.5-5 g/cm^3,
    2 kK-4 MK) minimised together in mixed precision with the graph CG, each against the FP64
    host-driven minimisation of the same cell (the 6-cell batch above is checked against the
    oracle).  Mixed and FP64 stop at 1e-8 Ha on different paths; the mixed path resolves F to
    about 1e-6 of the terms' magnitudes (measured worst cell 3.7e-6 relative)."""
    cells = wl.batch_cells(64)

    def ctx_for(cell, precision, graph):
        c = B.Context(functional="VT84F", precision=precision, tol_energy=1e-8, max_iter=2000, graph_cg=graph)
        c.set_cell(cell.lattice, cell.grid)
        c.set_ions(cell.positions, cell.charges)
        c.set_temperature(cell.temperature_K)
        return c

    batch = [ctx_for(c, "mixed", 1) for c in cells]
    reps = B.batch_minimize(batch)
    worst = 0.0
    for cell, ctx, rep in zip(cells, batch, reps):
        assert rep.converged, cell.grid
        ref = ctx_for(cell, "fp64", 0)
        F64 = ref.minimize_density().F_total
        ref.close()
        worst = max(worst, rel(rep.F_total, F64))
        ctx.close()
    print("worst relative F difference", worst, flush=True)
    assert worst < 1e-5

"""Checks of the seeded synthetic input generators (no method arithmetic)."""
import numpy as np
import pytest

import workloads as wl


def test_cell_edges_from_density():
    # 16 H at 1.0 g/cm^3 and 1024 H at 4.0 g/cm^3 (edge values of the hydrogen workloads)
    assert wl.cubic_edge_bohr(16, 1.0) == pytest.approx(5.6537, abs=2e-4)
    assert wl.cubic_edge_bohr(128, 2.0) == pytest.approx(8.9747, abs=2e-4)
    assert wl.cubic_edge_bohr(1024, 4.0) == pytest.approx(14.2465, abs=2e-4)
    # the paper's 128 H at 0.983 g/cm^3 has r_s = 1.40 bohr (Sec. VI B)
    L = wl.cubic_edge_bohr(128, 0.983)
    rs = (3 * L ** 3 / (4 * np.pi * 128)) ** (1 / 3)
    assert rs == pytest.approx(1.40, abs=0.005)


def test_minimum_image_separation_and_determinism():
    c1 = wl.gga_64_cell()
    c2 = wl.gga_64_cell()
    assert np.array_equal(c1.positions, c2.positions)
    L = c1.edge
    d = c1.positions[:, None, :] - c1.positions[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d ** 2).sum(-1)) + np.eye(c1.nat) * 1e9
    assert r.min() >= 0.8
    assert np.all((c1.positions >= 0) & (c1.positions < L))


def test_batch_draws_within_ranges():
    cells = wl.batch_cells(64)
    assert len(cells) == 64
    for c in cells:
        assert 16 <= c.nat <= 256
        assert c.grid[0] in (32, 48, 64, 96) and c.grid[0] == c.grid[1] == c.grid[2]
        assert 0.5 <= c.rho_gcc <= 5.0
        assert 2e3 <= c.temperature_K <= 4e6
    assert len({c.seed for c in cells}) == 64


def test_trial_phi_positive_and_smooth():
    phi = wl.trial_phi((16, 16, 16), 0.1, seed=3, contrast=0.6)
    assert phi.min() > 0
    n = phi ** 2
    assert n.mean() == pytest.approx(0.1, rel=0.3)

"""Pins of the oracle's velocity-Verlet integrator (the MD of Sec. VI B; E_cons as printed in
Sec. V D), on model surfaces whose discrete dynamics are known independently of the code:

* a harmonic well: the velocity-Verlet positions obey x_{n+1} - 2 x_n + x_{n-1} = -(w dt)^2 x_n,
  so x_n = x_0 cos(n a) + (dt v_0 / sin a) sin(n a) with cos a = 1 - (w dt)^2 / 2, exactly;
* time reversal: n steps, velocities reversed, n steps return to the start;
* a pair potential (forces of equal size and opposite sign): the total momentum stays at its
  initial value, and E_cons = sum M v^2/2 + E is conserved to O(dt^2).
A dropped half-kick, a wrong sign or a mass in the wrong place fails the first pin."""
import numpy as np
import pytest

from oracle import md as omd


def _harmonic(k):
    def ef(x):
        return 0.5 * k * float(np.sum(x * x)), -k * x
    return ef


def test_harmonic_well_follows_the_closed_form_of_the_discrete_map():
    k, M, dt, n = 0.07, 1837.0, 9.0, 150
    w = np.sqrt(k / M)
    rng = np.random.default_rng(11)
    x0 = rng.normal(0.0, 0.3, (5, 3))
    v0 = rng.normal(0.0, 1e-3, (5, 3))
    frames = omd.velocity_verlet(x0, v0, np.full(5, M), dt, n, _harmonic(k))
    a = np.arccos(1.0 - 0.5 * (w * dt) ** 2)
    for fr in frames[1:]:
        ref = x0 * np.cos(fr.step * a) + (dt * v0 / np.sin(a)) * np.sin(fr.step * a)
        assert np.max(np.abs(fr.positions - ref)) < 1e-12, fr.step
    # the velocity of the map: v_n = (x_{n+1} - x_{n-1}) / (2 dt), exactly, for this integrator
    for j in range(1, n):
        vc = (frames[j + 1].positions - frames[j - 1].positions) / (2.0 * dt)
        assert np.max(np.abs(frames[j].velocities - vc)) < 1e-14


def _pair(eps=0.02, r0=1.6):
    """A Morse pair potential summed over all pairs of a small cluster."""
    def ef(x):
        E, F = 0.0, np.zeros_like(x)
        for i in range(len(x)):
            for j in range(i + 1, len(x)):
                d = x[i] - x[j]
                r = np.linalg.norm(d)
                e = np.exp(-1.3 * (r - r0))
                E += eps * (1.0 - e) ** 2
                dEdr = 2.0 * eps * (1.0 - e) * 1.3 * e
                F[i] -= dEdr * d / r
                F[j] += dEdr * d / r
        return E, F
    return ef


def _cluster():
    x0 = np.array([[0.0, 0.0, 0.0], [1.7, 0.1, 0.0], [0.2, 1.6, -0.1], [-0.1, 0.3, 1.5]])
    rng = np.random.default_rng(5)
    M = np.array([1837.0, 1837.0, 3674.0, 1837.0])
    v0 = rng.normal(0.0, 2e-3, (4, 3))
    return x0, v0, M


def test_time_reversal_returns_to_the_start():
    x0, v0, M = _cluster()
    dt, n = 8.0, 120
    fwd = omd.velocity_verlet(x0, v0, M, dt, n, _pair())
    back = omd.velocity_verlet(fwd[-1].positions, -fwd[-1].velocities, M, dt, n, _pair())
    assert np.max(np.abs(back[-1].positions - x0)) < 1e-10
    assert np.max(np.abs(back[-1].velocities + v0)) < 1e-12


def test_momentum_is_conserved_and_energy_error_is_second_order():
    x0, v0, M = _cluster()
    p0 = np.sum(M[:, None] * v0, axis=0)
    spans = []
    for dt in (16.0, 8.0):
        frames = omd.velocity_verlet(x0, v0, M, dt, int(1600 / dt), _pair())
        for fr in frames:
            assert np.max(np.abs(np.sum(M[:, None] * fr.velocities, axis=0) - p0)) < 1e-13
        e = np.array([fr.F_tot + fr.kinetic for fr in frames])
        spans.append(np.ptp(e))
        assert fr.kinetic == pytest.approx(0.5 * np.sum(M[:, None] * fr.velocities ** 2), rel=1e-14)
    # halving dt divides the energy error by about four
    assert 3.0 < spans[0] / spans[1] < 5.0, spans

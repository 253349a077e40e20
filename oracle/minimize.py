"""Direct minimisation of F_tot[phi^2] on the electron-count sphere.

TEST INFRASTRUCTURE (oracle).

The paper minimises the total free energy directly under the constraint that
the integral of the density is constant, with the nonlinear conjugate-gradient
and truncated-Newton optimisers of PROFESS (Sec. I, Sec. II).  Their details
are in a reference that is not reproduced here, so this module takes the
following reading (several iteration paths are correct; only the converged
results are compared):

* variable phi with n = phi^2 and the sphere dv * sum phi^2 = N_e;
* projected gradient g = 2 dv phi (v - mu), mu = int n v / N_e (Eq. E10);
* a step along a tangent direction d (d . phi = 0) is a rotation on the sphere
      phi(theta) = cos(theta) phi + sin(theta) |phi| d/|d|,
  which keeps sum phi^2 fixed exactly;
* the line search uses dF/dtheta = g(theta) . dphi/dtheta, a first trial step,
  then safeguarded secant/bisection on dF/dtheta until
  |dF/dtheta| <= 0.1 |dF/dtheta(0)| with sufficient decrease (or, once the
  change of F is at its rounding level 1e-14 |F|, with no increase beyond it);
* CG: Polak-Ribiere with restart (beta = max(0, .)), direction projected
  orthogonal to phi;
* TN: Newton-CG in the tangent space on the Lagrangian Hessian
      H v = P[(grad F(phi + e v) - grad F(phi - e v))/(2 e)] - 2 dv mu v,
  grad F = 2 dv phi v_pot the unconstrained gradient, P the tangent
  projector; inner tolerance min(0.5, sqrt|g|)|g|, at most 20 inner steps,
  stop on negative curvature;
* stop when |F_k - F_{k-1}| < tol_energy on two consecutive iterations and,
  if tol_residual > 0, sqrt(sum n (v-mu)^2 / sum n) < tol_residual.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

from .energy import EvalResult, System, evaluate


@dataclasses.dataclass
class MinResult:
    phi: np.ndarray
    result: EvalResult
    iterations: int
    evaluations: int
    converged: bool
    history: list


def _dot(a, b) -> float:
    return float(np.sum(a * b))


def _rotate(phi, dhat, r, theta):
    return math.cos(theta) * phi + math.sin(theta) * r * dhat


def _line_search(phi, F0, dF0, dhat, r, system, theta1, counter, max_trials=12):
    """Returns (theta, phi_new, eval_new) with F decreased, or None."""
    lo, Flo, dlo = 0.0, F0, dF0
    hi = None
    Fhi = dhi = None
    best = None
    theta = theta1
    for _ in range(max_trials):
        p = _rotate(phi, dhat, r, theta)
        ev = evaluate(p, system)
        counter[0] += 1
        dp = -math.sin(theta) * phi + math.cos(theta) * r * dhat
        dth = _dot(ev.grad, dp)
        if ev.F_tot <= F0 and (best is None or ev.F_tot < best[2].F_tot):
            best = (theta, p, ev)
        armijo = ev.F_tot <= F0 + 1e-4 * theta * dF0
        # at the rounding floor of F the decrease test cannot resolve progress;
        # then the slope condition alone decides (approximate Wolfe)
        flat = ev.F_tot <= F0 + 1e-14 * abs(F0)
        if (armijo or flat) and abs(dth) <= 0.1 * abs(dF0):
            return theta, p, ev
        if dth > 0 or not armijo:
            hi, Fhi, dhi = theta, ev.F_tot, dth
        else:
            lo, Flo, dlo = theta, ev.F_tot, dth
        if hi is None:
            # no bracket yet: secant on dF/dtheta through (0, dF0), (theta, dth),
            # kept within [1.5 theta, 4 theta]
            new = 2.0 * theta if dth <= dF0 else theta - dth * theta / (dth - dF0)
            theta = min(max(new, 1.5 * theta), 4.0 * theta)
        else:
            if dhi is not None and dhi > dlo and dth > 0:
                new = lo - dlo * (hi - lo) / (dhi - dlo)
            else:
                new = 0.5 * (lo + hi)
            w = hi - lo
            theta = min(max(new, lo + 0.1 * w), hi - 0.1 * w)
    return best


def _first_step(F0, F_prev, dF0):
    if F_prev is not None and dF0 < 0 and F_prev > F0:
        th = 2.0 * (F_prev - F0) / (-dF0)
        return float(min(max(th, 1e-6), 0.3))
    return 0.05


def minimize_cg(system: System, phi0=None, tol_energy: float = 1e-8,
                tol_residual: float = 0.0, max_iter: int = 2000,
                callback: Optional[Callable] = None) -> MinResult:
    phi = system.uniform_phi() if phi0 is None else np.array(phi0, dtype=np.float64)
    norm2 = system.n_electrons / system.grid.dv
    phi *= math.sqrt(norm2 / _dot(phi, phi))
    counter = [0]
    ev = evaluate(phi, system)
    counter[0] += 1
    g = ev.grad
    d = -g
    g_prev = None
    F_prev = None
    small = 0
    history = [ev.F_tot]
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        if g_prev is not None:
            beta = max(0.0, _dot(g, g - g_prev) / _dot(g_prev, g_prev))
            d = -g + beta * d
        d = d - (_dot(d, phi) / norm2) * phi
        if _dot(d, g) >= 0.0:
            d = -g
        dn = math.sqrt(_dot(d, d))
        if dn == 0.0:
            converged = True
            break
        dhat = d / dn
        r = math.sqrt(norm2)
        dF0 = r * _dot(g, dhat)
        ls = _line_search(phi, ev.F_tot, dF0, dhat, r, system,
                          _first_step(ev.F_tot, F_prev, dF0), counter)
        if ls is None:
            converged = small >= 1 or (tol_residual > 0 and ev.residual(phi) < tol_residual)
            break
        _, phi_new, ev_new = ls
        phi_new *= math.sqrt(norm2 / _dot(phi_new, phi_new))
        dF = ev.F_tot - ev_new.F_tot
        F_prev = ev.F_tot
        g_prev = g
        phi, ev = phi_new, ev_new
        g = ev.grad
        history.append(ev.F_tot)
        if callback:
            callback(it, phi, ev)
        small = small + 1 if abs(dF) < tol_energy else 0
        if small >= 2 and (tol_residual <= 0 or ev.residual(phi) < tol_residual):
            converged = True
            break
    return MinResult(phi=phi, result=ev, iterations=it, evaluations=counter[0],
                     converged=converged, history=history)


def _full_gradient(phi, system):
    ev = evaluate(phi, system)
    return 2.0 * system.grid.dv * phi * ev.v


def minimize_tn(system: System, phi0=None, tol_energy: float = 1e-8,
                tol_residual: float = 0.0, max_iter: int = 200, max_inner: int = 20,
                callback: Optional[Callable] = None) -> MinResult:
    phi = system.uniform_phi() if phi0 is None else np.array(phi0, dtype=np.float64)
    norm2 = system.n_electrons / system.grid.dv
    phi *= math.sqrt(norm2 / _dot(phi, phi))
    dv = system.grid.dv
    counter = [0]
    ev = evaluate(phi, system)
    counter[0] += 1
    history = [ev.F_tot]
    small = 0
    converged = False
    F_prev = None
    it = 0

    def proj(x):
        return x - (_dot(x, phi) / norm2) * phi

    for it in range(1, max_iter + 1):
        g = ev.grad
        gnorm = math.sqrt(_dot(g, g))
        if gnorm == 0.0:
            converged = True
            break
        # inner CG on H p = -g in the tangent space
        tol_in = min(0.5, math.sqrt(gnorm)) * gnorm
        p = np.zeros_like(phi)
        res = -g.copy()
        s = res.copy()
        rr = _dot(res, res)
        phinorm = math.sqrt(norm2)
        for k in range(max_inner):
            snorm = math.sqrt(_dot(s, s))
            eps = 1e-6 * phinorm / snorm
            gp = _full_gradient(phi + eps * s, system)
            gm = _full_gradient(phi - eps * s, system)
            counter[0] += 2
            Hs = proj((gp - gm) / (2.0 * eps)) - 2.0 * dv * ev.mu * s
            curv = _dot(s, Hs)
            if curv <= 0.0:
                if k == 0:
                    p = -g.copy()
                break
            a = rr / curv
            p += a * s
            res -= a * Hs
            rr_new = _dot(res, res)
            if math.sqrt(rr_new) < tol_in:
                break
            s = res + (rr_new / rr) * s
            rr = rr_new
        d = proj(p)
        if _dot(d, g) >= 0.0:
            d = -g
        dn = math.sqrt(_dot(d, d))
        dhat = d / dn
        r = math.sqrt(norm2)
        dF0 = r * _dot(g, dhat)
        # the Newton step length corresponds to theta ~ |d|/r
        theta1 = min(max(dn / r, 1e-8), 0.5)
        ls = _line_search(phi, ev.F_tot, dF0, dhat, r, system, theta1, counter)
        if ls is None:
            converged = small >= 1 or (tol_residual > 0 and ev.residual(phi) < tol_residual)
            break
        _, phi_new, ev_new = ls
        phi_new *= math.sqrt(norm2 / _dot(phi_new, phi_new))
        dF = ev.F_tot - ev_new.F_tot
        phi, ev = phi_new, ev_new
        history.append(ev.F_tot)
        if callback:
            callback(it, phi, ev)
        small = small + 1 if abs(dF) < tol_energy else 0
        if small >= 2 and (tol_residual <= 0 or ev.residual(phi) < tol_residual):
            converged = True
            break
    return MinResult(phi=phi, result=ev, iterations=it, evaluations=counter[0],
                     converged=converged, history=history)

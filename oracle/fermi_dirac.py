"""Fermi-Dirac integrals, their inverse, and the finite-T reduced-temperature factors.

TEST INFRASTRUCTURE (oracle).  Plain FP64 quadrature; slow by design.

What is computed (arXiv:1406.0835, Sec. III A and B, Table I footnote a):

* Normalised Fermi-Dirac integrals
      F_j(eta) = 1/Gamma(j+1) * Int_0^inf x^j / (1 + exp(x - eta)) dx,
  for j = 3/2, 1/2, -1/2, and the lower orders through F_{j-1} = dF_j/deta,
  i.e. F_{-3/2}, F_{-5/2}, F_{-7/2} are eta-derivatives of F_{-1/2} taken under
  the integral.  With x = u^2 the x^{-1/2} end-point singularity disappears:
      F_j = 2/Gamma(j+1) Int_0^inf u^{2j+1} f du,  f = 1/(1+exp(u^2-eta)),
  and d f/d eta = f(1-f), d^2 f = f(1-f)(1-2f), d^3 f = f(1-f)(1-6f(1-f)).
  Quadrature: composite Gauss-Legendre in u on panels that are uniform in x
  over the window [max(eta-44,0), max(eta,0)+44] (width <= 3.7 in units of kT,
  so the Fermi-function poles at x = eta +- i pi are far from every panel),
  plus one Gauss-Legendre panel on [0, sqrt(eta-44)] where f = 1 to e^-44.

* Reduced temperature t = T/T_F = 2T/(3 pi^2 n)^(2/3)        (Eq. tred).
  The uniform-gas density fixes eta by F_{1/2}(eta) = 4/(3 sqrt(pi)) t^(-3/2)
  (the paper's y = I_{1/2}(eta) = (2/3) t^(-3/2) with unnormalised I_nu).
  The inverse is a Newton iteration on ln F_{1/2}, which is concave and
  increasing in eta, so the iterates converge monotonically.

* kappa(t) = (5/3) t f(y), f(y) = eta - (2/3) I_{3/2}/I_{1/2} (Table I, note a)
           = (5/3) t (eta - R),   R = F_{3/2}/F_{1/2};
  xi = kappa - t kappa',  zeta = -t kappa'                    (Eq. xizeta),
  which reduce to xi = (5/2) t R and zeta = xi - kappa.  Derivatives follow
  from d eta/dt = -(3/2) F_{1/2}/(t F_{-1/2}).

* h~(t): the gradient coefficient of the finite-T second-order gradient
  expansion, h = h~/72 in the notation of Table I.  It is the q^2 term of the
  finite-T static Lindhard response: chi(q) = -n' + (q^2/12) n'' + O(q^4)
  with n' = dn/dmu, whence the SGA free energy int (h~/72)|grad n|^2/n with
      h~ = 3 n n''/n'^2 = 3 F_{1/2} F_{-3/2} / F_{-1/2}^2 .
  Its t-derivatives use F_{-5/2}, F_{-7/2}.

Pins (tests/test_oracle_fermi_dirac.py): mpmath 30-digit quadrature at sample
eta; the Dirichlet-eta values F_j(0) = (1 - 2^-j) zeta(j+1); Sommerfeld and
Boltzmann asymptotics; dF_j/deta = F_{j-1} by finite differences; round trip of
the inverse; kappa -> 1 - (5 pi^2/12) t^2 (T -> 0) and the classical ideal gas
(T -> inf); zeta = -t kappa' by finite differences; h~(0) = 1, h~(inf) = 3,
h~ = 1 + (pi^2/3) t^2; h~ against a brute-force finite-T Lindhard function.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from math import gamma, pi, sqrt

import numpy as np

_NPANEL = 24
_NGL = 16
_NGL_LOW = 24
_HALF_WINDOW = 44.0
_GL_X, _GL_W = np.polynomial.legendre.leggauss(_NGL)
_GLL_X, _GLL_W = np.polynomial.legendre.leggauss(_NGL_LOW)
_CHUNK = 2048
_THREADS = int(os.environ.get("OFDFT_ORACLE_THREADS", os.cpu_count() or 1))
_POOL = ThreadPoolExecutor(max_workers=_THREADS) if _THREADS > 1 else None


def _over_chunks(fn, size):
    """Run fn(start, stop) over independent chunks (numpy releases the GIL)."""
    spans = [(s, min(s + _CHUNK, size)) for s in range(0, size, _CHUNK)]
    if _POOL is None or len(spans) < 2:
        for a, b in spans:
            fn(a, b)
    else:
        list(_POOL.map(lambda ab: fn(*ab), spans))

ORDERS = (1.5, 0.5, -0.5, -1.5, -2.5, -3.5)

# prefactors 2/Gamma(j+1) for the direct orders
_C32 = 2.0 / gamma(2.5)
_C12 = 2.0 / gamma(1.5)
_CM12 = 2.0 / gamma(0.5)

Y_PREFACTOR = 4.0 / (3.0 * sqrt(pi))   # F_{1/2}(eta) = Y_PREFACTOR * t^(-3/2)


def _nodes(eta: np.ndarray):
    """Quadrature nodes u (m, K) and weights for each eta (m,)."""
    m = eta.shape[0]
    xa = np.maximum(eta - _HALF_WINDOW, 0.0)
    xb = np.maximum(eta, 0.0) + _HALF_WINDOW
    frac = np.arange(_NPANEL + 1) / _NPANEL
    ue = np.sqrt(xa[:, None] + (xb - xa)[:, None] * frac[None, :])
    half = 0.5 * (ue[:, 1:] - ue[:, :-1])
    mid = 0.5 * (ue[:, 1:] + ue[:, :-1])
    u = (mid[:, :, None] + half[:, :, None] * _GL_X[None, None, :]).reshape(m, -1)
    w = (half[:, :, None] * _GL_W[None, None, :]).reshape(m, -1)
    ua = np.sqrt(xa)
    ul = 0.5 * ua[:, None] * (1.0 + _GLL_X[None, :])
    wl = 0.5 * ua[:, None] * _GLL_W[None, :]
    return np.concatenate([u, ul], axis=1), np.concatenate([w, wl], axis=1)


def _fermi(u: np.ndarray, eta: np.ndarray):
    """f = 1/(1+e^z) and g = 1-f, z = u^2 - eta, both without cancellation."""
    z = np.clip(u * u - eta[:, None], -700.0, 700.0)
    ez = np.exp(z)
    f = 1.0 / (1.0 + ez)
    g = ez / (1.0 + ez)
    return f, g


def fd_all(eta) -> dict:
    """All six orders {1.5, 0.5, -0.5, -1.5, -2.5, -3.5} of F_j at eta (array)."""
    eta = np.atleast_1d(np.asarray(eta, dtype=np.float64))
    shape = eta.shape
    flat = eta.ravel()
    out = {j: np.empty(flat.shape) for j in ORDERS}

    def work(a, b):
        e = flat[a:b]
        u, w = _nodes(e)
        f, g = _fermi(u, e)
        u2 = u * u
        fg = f * g
        out[1.5][a:b] = _C32 * np.sum(w * u2 * u2 * f, axis=1)
        out[0.5][a:b] = _C12 * np.sum(w * u2 * f, axis=1)
        out[-0.5][a:b] = _CM12 * np.sum(w * f, axis=1)
        out[-1.5][a:b] = _CM12 * np.sum(w * fg, axis=1)
        out[-2.5][a:b] = _CM12 * np.sum(w * fg * (g - f), axis=1)
        out[-3.5][a:b] = _CM12 * np.sum(w * fg * (1.0 - 6.0 * fg), axis=1)

    _over_chunks(work, flat.size)
    return {j: v.reshape(shape) for j, v in out.items()}


def fd_half_and_minus_half(eta: np.ndarray):
    """F_{1/2} and F_{-1/2} only (used inside the Newton inverse)."""
    f12 = np.empty(eta.shape)
    fm12 = np.empty(eta.shape)

    def work(a, b):
        e = eta[a:b]
        u, w = _nodes(e)
        f, _ = _fermi(u, e)
        f12[a:b] = _C12 * np.sum(w * u * u * f, axis=1)
        fm12[a:b] = _CM12 * np.sum(w * f, axis=1)

    _over_chunks(work, eta.size)
    return f12, fm12


def fd(j: float, eta):
    """Single order F_j(eta)."""
    return fd_all(eta)[j]


def inverse_f_half(y, max_iter: int = 100) -> np.ndarray:
    """eta solving F_{1/2}(eta) = y (y > 0), by Newton on ln F_{1/2}.

    Iterates until the step is below 1e-9 max(1,|eta|), then takes one more
    (quadratic convergence brings it to rounding level).
    """
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    shape = y.shape
    yf = y.ravel()
    if np.any(~(yf > 0)):
        raise ValueError("F_{1/2}^{-1} needs y > 0")
    # start: two-term Boltzmann inversion for small y, two-term Sommerfeld
    # inversion for large y (only a starting point for Newton)
    e0 = (0.75 * sqrt(pi) * yf) ** (2.0 / 3.0)
    eta = np.where(yf < 1.5, np.log(yf) + yf / 2.0 ** 1.5,
                   e0 * (1.0 - pi * pi / (12.0 * e0 * e0)))
    ly = np.log(yf)
    active = np.arange(yf.size)
    final = np.zeros(yf.size, dtype=bool)
    for _ in range(max_iter):
        if active.size == 0:
            break
        e = eta[active]
        f12, fm12 = fd_half_and_minus_half(e)
        step = (np.log(f12) - ly[active]) * f12 / fm12
        eta[active] = e - step
        was_final = final[active]
        small = np.abs(step) <= 1e-9 * np.maximum(1.0, np.abs(e))
        final[active[small]] = True
        active = active[~was_final]
    if active.size:
        raise RuntimeError("F_{1/2} inverse did not converge")
    return eta.reshape(shape)


def reduced_temperature(n, T_ha):
    """t = T/T_F = 2 T / (3 pi^2 n)^(2/3)   (Eq. tred)."""
    n = np.asarray(n, dtype=np.float64)
    return 2.0 * T_ha / (3.0 * pi * pi * n) ** (2.0 / 3.0)


def eta_of_t(t) -> np.ndarray:
    """eta(t) from F_{1/2}(eta) = 4/(3 sqrt pi) t^(-3/2)."""
    t = np.asarray(t, dtype=np.float64)
    return inverse_f_half(Y_PREFACTOR * t ** -1.5)


def t_factors(t) -> dict:
    """kappa, xi, zeta, h~ and their t-derivatives at reduced temperature t.

    Keys: eta, kappa, dkappa, xi, dxi, zeta, dzeta, h, dh, d2h  (d = d/dt).
    """
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    eta = eta_of_t(t)
    F = fd_all(eta)
    f32, f12, fm12, fm32, fm52, fm72 = (F[1.5], F[0.5], F[-0.5], F[-1.5], F[-2.5], F[-3.5])
    R = f32 / f12
    kappa = (5.0 / 3.0) * t * (eta - R)
    xi = 2.5 * t * R
    zeta = xi - kappa
    deta = -1.5 * f12 / (t * fm12)                   # d eta / dt
    dkappa = -zeta / t                               # from zeta = -t kappa'
    dR = deta * (1.0 - f32 * fm12 / (f12 * f12))     # dR/dt
    dxi = 2.5 * (R + t * dR)
    dzeta = dxi - dkappa
    # h~ = 3 F12 Fm32 / Fm12^2 and its eta-derivatives
    h = 3.0 * f12 * fm32 / (fm12 * fm12)
    a = fm32 / fm12
    b = f12 * fm52 / (fm12 * fm12)
    c = -2.0 * f12 * fm32 * fm32 / fm12 ** 3
    dh_deta = 3.0 * (a + b + c)
    da = fm52 / fm12 - fm32 * fm32 / (fm12 * fm12)
    db = (fm12 * fm52 + f12 * fm72) / (fm12 * fm12) - 2.0 * f12 * fm52 * fm32 / fm12 ** 3
    dc = (-2.0 * fm32 * fm32 / (fm12 * fm12) - 4.0 * f12 * fm32 * fm52 / fm12 ** 3
          + 6.0 * f12 * fm32 ** 3 / fm12 ** 4)
    d2h_deta2 = 3.0 * (da + db + dc)
    # d2 eta/dt2 from d eta/dt = -(3/2) F12 / (t Fm12)
    d2eta = -1.5 * (deta * (1.0 - f12 * fm32 / (fm12 * fm12)) / t - f12 / (t * t * fm12))
    dh = dh_deta * deta
    d2h = d2h_deta2 * deta * deta + dh_deta * d2eta
    return dict(eta=eta, kappa=kappa, dkappa=dkappa, xi=xi, dxi=dxi, zeta=zeta,
                dzeta=dzeta, h=h, dh=dh, d2h=d2h, F=F)

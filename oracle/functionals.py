"""Pointwise free-energy densities and their partial derivatives.

TEST INFRASTRUCTURE (oracle).  Plain FP64 numpy, arrays of grid values.

Non-interacting free energy (arXiv:1406.0835 Sec. III):
  * tau_0 = c_TF n^(5/3), c_TF = (3/10)(3 pi^2)^(2/3)           (Eq. tauTFdefn)
  * ftTF:  f = tau_0 kappa(t)                                    (Eqs. TF, fTF)
           v = d tau_0/dn kappa + tau_0 kappa' dt/dn             (Eq. vTF)
  * GGA:   f = tau_0 xi F_tau(s_tau) - tau_0 zeta F_sigma(s_sigma)  (Eq. FGGA)
           with s = |grad n| / (2 (3 pi^2)^(1/3) n^(4/3))          (Eq. s_0defn)
           s_tau^2 = s^2 (h~ - t h~')/xi, s_sigma^2 = s^2 t h~'/zeta (Eq. s_s)
           and the partial derivatives entering Eq. vftGGA:
             df/dn at fixed sigma = |grad n|^2, and df/dsigma,
           so that v = df/dn - div(2 df/dsigma grad n).
           Every term of the entropic line of Eq. vftGGA carries the minus
           sign of Eq. FGGA (direct differentiation of Eq. FGGA).
  * enhancement factors, written in x = s^2:
           VT84F (Eq. VT84F, m = 8, n = 4, mu = 2.778, alpha = 1.2965),
           KST2 form 1 + C1 x/(1 + a1 x) (Eq. KST2F) with the KST2, APBEF
           and TW constants, SGA/VWTF 1 + mu x (Eq. SGA-F, mu = 5/27 or 5/3);
           F_sigma(x) = 2 - F_tau(x) for all of them.
  * T S_s density = tau_0 zeta F_sigma(s_sigma) (tau_0 zeta for ftTF).

Exchange-correlation: ground-state spin-unpolarised LDA in the Perdew-Zunger
1981 parametrisation (the paper's "PZ" XC, Sec. IV first paragraph, Sec. VI):
  eps_x = -(3/4)(3/pi)^(1/3) n^(1/3);
  eps_c = gamma/(1 + beta1 sqrt(rs) + beta2 rs)           (rs >= 1)
        = A ln rs + B + C rs ln rs + D rs                  (rs < 1)
  with gamma=-0.1423, beta1=1.0529, beta2=0.3334, A=0.0311, B=-0.048
  (Phys. Rev. B 23, 5048 (1981), unpolarised) and C, D fixed by continuity
  of eps_c and its derivative at rs = 1 (C = 0.0020192, D = -0.0116321; the
  published C = 0.0020, D = -0.0116 are these rounded);
  v_xc = eps_xc - (rs/3) d eps_xc/d rs.

Pins (tests/test_oracle_functionals.py): ftTF potential equals T*eta (uniform
gas chemical potential); SGA equals f_TF + (h~/72)|grad n|^2/n; VWTF at t -> 0
equals TF + von Weizsaecker; VT84F (F-1)/s^2 -> 5/27 and F -> 5/3 s^2 + 1/s^2;
df/dn and df/dsigma against central finite differences; the KST2-form factors'
small-s slope C1 and large-s bound 1 + C1/a1 (1.804 for APBEF); exchange closed
form; PZ81 continuity of eps_c and its slope at rs = 1; v_xc by finite differences.

Parity unpinned: the PZ81 correlation constants themselves (gamma, beta1, beta2,
A, B, and C, D).  They come from the cited publication, not from the paper, and
no test here reproduces them from something independent; the continuity-fixed
C, D differ from the published rounded values by 1.9e-5 and -3.2e-5, which moves
eps_c by -2.3e-5 to -3.2e-5 hartree per electron for rs in [0.5, 1).
"""
from __future__ import annotations

from math import pi

import numpy as np

from . import fermi_dirac as fdm

C_TF = 0.3 * (3.0 * pi * pi) ** (2.0 / 3.0)
S2_DENOM = 4.0 * (3.0 * pi * pi) ** (2.0 / 3.0)      # s^2 = sigma / (S2_DENOM n^(8/3))
DENSITY_FLOOR = 1.0e-12

VT84F_MU = 2.778
VT84F_ALPHA = 1.2965
KST2_CONSTANTS = {"KST2": (2.03087, 0.29424),
                  "APBEF": (0.23889, 0.23889 / 0.804),
                  "TW": (0.2319, 0.2748)}
MU_SGA = 5.0 / 27.0
MU_VWTF = 5.0 / 3.0

GGA_FUNCTIONALS = ("SGA", "VWTF", "VT84F", "KST2", "APBEF", "TW")
FUNCTIONALS = ("TF",) + GGA_FUNCTIONALS


# ---------------------------------------------------------------- enhancement factors
def enh_vt84f(x):
    """VT84F F(x) and dF/dx, x = s^2 (Eq. VT84F with m = 8, n = 4)."""
    x = np.asarray(x, dtype=np.float64)
    mu, al = VT84F_MU, VT84F_ALPHA
    ex = np.exp(-al * x)
    t1 = -mu * x * ex / (1.0 + mu * x)
    dt1 = -mu * ex * (1.0 - al * x - al * mu * x * x) / (1.0 + mu * x) ** 2
    # q = 1 - exp(-alpha x^2); term = q (1/x - 1)
    q = -np.expm1(-al * x * x)
    small = x < 1.0e-4
    xs = np.where(small, 1.0, x)
    q_over_x = np.where(small, al * x - 0.5 * al * al * x ** 3, q / xs)
    q_over_x2 = np.where(small, al - 0.5 * al * al * x * x, q / (xs * xs))
    t2 = q_over_x - q
    dt2 = 2.0 * al * np.exp(-al * x * x) * (1.0 - x) - q_over_x2
    F = 1.0 + t1 + t2 + (5.0 / 3.0) * x
    dF = dt1 + dt2 + 5.0 / 3.0
    return F, dF


def enh_kst2_form(x, c1, a1):
    """1 + C1 x/(1 + a1 x) and its x-derivative (Eq. KST2F)."""
    x = np.asarray(x, dtype=np.float64)
    den = 1.0 + a1 * x
    return 1.0 + c1 * x / den, c1 / (den * den)


def enh_sga(x, mu):
    """1 + mu x (Eq. SGA-F)."""
    x = np.asarray(x, dtype=np.float64)
    return 1.0 + mu * x, np.full_like(x, mu)


def enhancement(name: str, mu_sga: float = MU_SGA):
    if name == "VT84F":
        return enh_vt84f
    if name in KST2_CONSTANTS:
        c1, a1 = KST2_CONSTANTS[name]
        return lambda x: enh_kst2_form(x, c1, a1)
    if name == "SGA":
        return lambda x: enh_sga(x, mu_sga)
    if name == "VWTF":
        return lambda x: enh_sga(x, MU_VWTF)
    raise ValueError(f"unknown GGA functional {name}")


# ---------------------------------------------------------------- non-interacting
def tf_point(n, T_ha, factors=None):
    """ftTF: returns (f, df/dn, T s_s) at density n (already floored)."""
    n = np.asarray(n, dtype=np.float64)
    t = fdm.reduced_temperature(n, T_ha)
    tf = factors if factors is not None else fdm.t_factors(t)
    A = C_TF * n ** (5.0 / 3.0)
    dA = (5.0 / 3.0) * A / n
    dtdn = -(2.0 / 3.0) * t / n
    f = A * tf["kappa"]
    v = dA * tf["kappa"] + A * tf["dkappa"] * dtdn          # Eq. vTF
    ts = A * tf["zeta"]
    return f, v, ts


def gga_point(n, sigma, T_ha, name: str, mu_sga: float = MU_SGA, factors=None):
    """Generic finite-T GGA (Eq. FGGA) with the enhancement factor `name`.

    Returns (f, df/dn|_sigma, df/dsigma, T s_s); sigma = |grad n|^2.
    """
    n = np.asarray(n, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    enh = enhancement(name, mu_sga)
    t = fdm.reduced_temperature(n, T_ha)
    tf = factors if factors is not None else fdm.t_factors(t)
    xi, dxi, zeta, dzeta = tf["xi"], tf["dxi"], tf["zeta"], tf["dzeta"]
    h, dh, d2h = tf["h"], tf["dh"], tf["d2h"]
    A = C_TF * n ** (5.0 / 3.0)
    inv_den = 1.0 / (S2_DENOM * n ** (8.0 / 3.0))           # ds^2/dsigma
    s2 = sigma * inv_den
    p_tau = (h - t * dh) / xi
    p_sig = t * dh / zeta
    dp_tau = (-t * d2h * xi - (h - t * dh) * dxi) / (xi * xi)
    dp_sig = ((dh + t * d2h) * zeta - t * dh * dzeta) / (zeta * zeta)
    x_tau = s2 * p_tau
    x_sig = s2 * p_sig
    F_tau, dF_tau = enh(x_tau)
    G, dG = enh(x_sig)
    F_sig = 2.0 - G
    dF_sig = -dG
    f = A * (xi * F_tau - zeta * F_sig)
    dtdn = -(2.0 / 3.0) * t / n
    ds2dn = -(8.0 / 3.0) * s2 / n
    dfdn = ((5.0 / 3.0) * f / n
            + A * (dxi * F_tau - dzeta * F_sig) * dtdn
            + A * xi * dF_tau * (ds2dn * p_tau + s2 * dp_tau * dtdn)
            - A * zeta * dF_sig * (ds2dn * p_sig + s2 * dp_sig * dtdn))
    dfds = A * (xi * dF_tau * p_tau - zeta * dF_sig * p_sig) * inv_den
    ts = A * zeta * F_sig
    return f, dfdn, dfds, ts


# ---------------------------------------------------------------- XC (PZ81)
PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B = 0.0311, -0.048
# C and D from continuity of eps_c and d eps_c/d rs at rs = 1 (their published
# values 0.0020 and -0.0116 are these, rounded; with the rounded values eps_c
# jumps by 3e-5 hartree at rs = 1 and F_tot is discontinuous in n)
_DEN1 = 1.0 + PZ_BETA1 + PZ_BETA2
PZ_D = PZ_GAMMA / _DEN1 - PZ_B
PZ_C = -PZ_GAMMA * (0.5 * PZ_BETA1 + PZ_BETA2) / _DEN1 ** 2 - PZ_A - PZ_D
EX_COEF = -0.75 * (3.0 / pi) ** (1.0 / 3.0)


def pz81(n):
    """Returns (eps_xc, v_xc) per electron for the unpolarised PZ81 LDA."""
    n = np.asarray(n, dtype=np.float64)
    rs = (3.0 / (4.0 * pi * n)) ** (1.0 / 3.0)
    ex = EX_COEF * n ** (1.0 / 3.0)
    vx = (4.0 / 3.0) * ex
    hi = rs >= 1.0
    rsh = np.where(hi, rs, 1.0)
    sq = np.sqrt(rsh)
    den = 1.0 + PZ_BETA1 * sq + PZ_BETA2 * rsh
    ec_hi = PZ_GAMMA / den
    dec_hi = -PZ_GAMMA * (0.5 * PZ_BETA1 / sq + PZ_BETA2) / (den * den)
    rsl = np.where(hi, 0.5, rs)
    lnr = np.log(rsl)
    ec_lo = PZ_A * lnr + PZ_B + PZ_C * rsl * lnr + PZ_D * rsl
    dec_lo = PZ_A / rsl + PZ_C * (lnr + 1.0) + PZ_D
    ec = np.where(hi, ec_hi, ec_lo)
    dec = np.where(hi, dec_hi, dec_lo)
    vc = ec - (rs / 3.0) * dec
    return ex + ec, vx + vc


# ---------------------------------------------------------------- KSDT finite-T LDA XC
# Sec. IV A, Eq. fit2, spin-unpolarised (omega_u = 1):
#   f_xc(rs, t) = -(1/rs) (a(t) + b(t) rs^(1/2) + c(t) rs) / (1 + d(t) rs^(1/2) + e(t) rs),
# rs = (3/(4 pi n))^(1/3), t from Eq. tred.  The functions a(t)..e(t) and their parameters
# are those of the publication the paper cites for the fit (Karasiev, Sjostrom, Dufty,
# Trickey, Phys. Rev. Lett. 112, 076403 (2014), unpolarised set):
#   a(t) = 0.610887 tanh(1/t) (0.75 + 3.04363 t^2 - 0.09227 t^3 + 1.7035 t^4)
#                              / (1 + 8.31051 t^2 + 5.1105 t^4)
#   b(t) = tanh(1/sqrt t) (b1 + b2 t^2 + b3 t^4) / (1 + b4 t^2 + b5 t^4)
#   c(t) = (c1 + c2 exp(-c3/t)) e(t)
#   d(t) = tanh(1/sqrt t) (d1 + d2 t^2 + d3 t^4) / (1 + d4 t^2 + d5 t^4)
#   e(t) = tanh(1/t) (e1 + e2 t^2 + e3 t^4) / (1 + e4 t^2 + e5 t^4)
KSDT_A = (0.610887, 0.75, 3.04363, -0.09227, 1.7035, 8.31051, 5.1105)
KSDT_B = (0.283997, 48.932154, 0.370919, 61.095357, 0.871837)
KSDT_C = (0.870089, 0.193077, 2.414644)
KSDT_D = (0.579824, 94.537454, 97.839603, 59.939999, 24.388037)
KSDT_E = (0.212036, 16.731249, 28.485792, 34.028876, 17.235515)


def ksdt_coefficients(t):
    """a(t), b(t), c(t), d(t), e(t) of Eq. fit2 (t real or complex)."""
    A0, A1, A2, A3, A4, A5, A6 = KSDT_A
    t2 = t * t
    t4 = t2 * t2
    a = A0 * np.tanh(1.0 / t) * (A1 + A2 * t2 + A3 * t2 * t + A4 * t4) / (1.0 + A5 * t2 + A6 * t4)
    rt = np.sqrt(t)
    b = np.tanh(1.0 / rt) * (KSDT_B[0] + KSDT_B[1] * t2 + KSDT_B[2] * t4) / (1.0 + KSDT_B[3] * t2 + KSDT_B[4] * t4)
    e = np.tanh(1.0 / t) * (KSDT_E[0] + KSDT_E[1] * t2 + KSDT_E[2] * t4) / (1.0 + KSDT_E[3] * t2 + KSDT_E[4] * t4)
    c = (KSDT_C[0] + KSDT_C[1] * np.exp(-KSDT_C[2] / t)) * e
    d = np.tanh(1.0 / rt) * (KSDT_D[0] + KSDT_D[1] * t2 + KSDT_D[2] * t4) / (1.0 + KSDT_D[3] * t2 + KSDT_D[4] * t4)
    return a, b, c, d, e


def ksdt_fxc(rs, t):
    """XC free energy per electron f_xc(rs, t), Eq. fit2 (unpolarised)."""
    a, b, c, d, e = ksdt_coefficients(t)
    q = np.sqrt(rs)
    return -(a + b * q + c * rs) / (rs * (1.0 + d * q + e * rs))


def _complex_step(fun, x, y, wrt):
    """d fun(x, y)/d(x or y) by the complex step fun(x + i h)/h (exact to rounding)."""
    h = 1e-30 * np.maximum(np.abs(x if wrt == 0 else y), 1.0)
    if wrt == 0:
        return np.imag(fun(x + 1j * h, y)) / h
    return np.imag(fun(x, y + 1j * h)) / h


def ksdt(n, T_ha):
    """(f_xc, v_xc, T s_xc) per electron for KSDT at density n and temperature T (hartree).

    v_xc follows Eq. vxc1: f + n (df/drs drs/dn + df/dt dt/dn) with drs/dn = -rs/(3n) and
    dt/dn = -2t/(3n).  T s_xc = -T df/dT at fixed n = -t df/dt (t is proportional to T), so
    the XC internal energy per electron is f_xc + T s_xc."""
    n = np.asarray(n, dtype=np.float64)
    rs = (3.0 / (4.0 * pi * n)) ** (1.0 / 3.0)
    t = fdm.reduced_temperature(n, T_ha)
    f = ksdt_fxc(rs, t)
    df_drs = _complex_step(ksdt_fxc, rs, t, 0)
    df_dt = _complex_step(ksdt_fxc, rs, t, 1)
    v = f - (rs / 3.0) * df_drs - (2.0 * t / 3.0) * df_dt
    return f, v, -t * df_dt


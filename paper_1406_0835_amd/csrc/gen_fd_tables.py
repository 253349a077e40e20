#!/usr/bin/env python3
"""Generate fd_tables.h: Chebyshev tables for the device Fermi-Dirac kernels.

The device evaluates, for a degeneracy parameter eta, the six normalised
Fermi-Dirac integrals F_j(eta) = -Li_{j+1}(-exp(eta)),
j = 3/2, 1/2, -1/2, -3/2, -5/2, -7/2 (the orders needed by the finite-T
Thomas-Fermi factor kappa(t) and the gradient coefficient h~(t) and their
t-derivatives, arXiv:1406.0835 Sec. III A/B), and a starting value for the
inverse of F_{1/2}.  Reference values come from mpmath's polylogarithm at 40
digits; the tables are Chebyshev interpolants at first-kind nodes.

Regions for F_j (same degree everywhere, so a wavefront runs one loop):
  region 0          eta < ETA_LO : x from z = e^eta on [0, e^ETA_LO], F_j = z * P(x)
  regions 1..NB     eta in [B[r-1], B[r]) : x linear in eta, F_j = P(x)
  region NB+1       eta >= ETA_HI : x from w = 1/eta on [0, 1/ETA_HI], F_j = eta^(j+1) P(x)
Inverse guess: eta(l), l = ln y, Chebyshev on [L_LO, L_HI] pieces; outside,
two-term series inversions (Boltzmann for small y, Sommerfeld for large y).

Usage: python gen_fd_tables.py > fd_tables.h   (prints a max-error report to stderr)
"""
import sys

import mpmath as mp
import numpy as np

mp.mp.dps = 40
ORDERS = [1.5, 0.5, -0.5, -1.5, -2.5, -3.5]
NC = 22                     # Chebyshev coefficients per function and region
ETA_LO = -2.0
BREAKS = [-2.0, 0.0, 2.0, 4.5, 8.0, 14.0, 24.0, 40.0]
ETA_HI = BREAKS[-1]
NG = 20                     # coefficients of the inverse guess pieces
L_BREAKS = [-7.0, -3.5, -1.0, 1.0, 2.5, 4.0, 5.5, 7.0]


def fd_mp(j, eta):
    return -mp.re(mp.polylog(j + 1, -mp.exp(mp.mpf(eta))))


def cheb_nodes(n):
    return [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / n) for k in range(n)]


def cheb_coeffs(values):
    """Coefficients c_k of sum c_k T_k from values at first-kind nodes (mp arithmetic)."""
    n = len(values)
    th = [mp.pi * (i + mp.mpf(1) / 2) / n for i in range(n)]
    c = []
    for m in range(n):
        acc = mp.fsum(mp.mpf(values[i]) * mp.cos(m * th[i]) for i in range(n))
        c.append(2 * acc / n)
    c[0] /= 2
    return np.array([float(v) for v in c])


def cheb_eval(c, x):
    return np.polynomial.chebyshev.chebval(x, c)


def region_map(r, eta):
    """(x, prefactor exponent info) for region r at eta (float or mpf)."""
    nb = len(BREAKS) - 1
    if r == 0:
        z = mp.exp(eta)
        return 2 * z / mp.exp(ETA_LO) - 1
    if r <= nb:
        a, b = BREAKS[r - 1], BREAKS[r]
        return (2 * mp.mpf(eta) - a - b) / (b - a)
    w = 1 / mp.mpf(eta)
    return 2 * w * ETA_HI - 1


def region_eta(r, x):
    nb = len(BREAKS) - 1
    x = mp.mpf(x)
    if r == 0:
        z = (x + 1) / 2 * mp.exp(ETA_LO)
        return mp.log(z)
    if r <= nb:
        a, b = BREAKS[r - 1], BREAKS[r]
        return ((b - a) * x + a + b) / 2
    w = (x + 1) / (2 * ETA_HI)
    return 1 / w


def scaled(r, j, eta):
    """The function tabulated in region r: F_j / prefactor."""
    nb = len(BREAKS) - 1
    F = fd_mp(j, eta)
    if r == 0:
        return F / mp.exp(eta)
    if r <= nb:
        return F
    return F / mp.power(eta, j + 1)


def build_fd_tables():
    nb = len(BREAKS) - 1
    nreg = nb + 2
    coef = np.zeros((nreg, len(ORDERS), NC))
    xs = cheb_nodes(NC)
    for r in range(nreg):
        etas = [region_eta(r, x) for x in xs]
        for jj, j in enumerate(ORDERS):
            vals = [scaled(r, j, e) for e in etas]
            coef[r, jj] = cheb_coeffs(vals)
    return coef


def report_fd(coef):
    nb = len(BREAKS) - 1
    worst = {}
    for r in range(nb + 2):
        xs = np.linspace(-0.999, 0.999, 61)
        for jj, j in enumerate(ORDERS):
            errs = []
            scale = 0.0
            for x in xs:
                e = region_eta(r, x)
                ref = scaled(r, j, e)
                got = cheb_eval(coef[r, jj], float(x))
                scale = max(scale, abs(float(ref)))
                errs.append(abs(got - float(ref)))
            worst[(r, j)] = max(errs) / scale
    for (r, j), e in sorted(worst.items()):
        print(f"region {r} order {j:+.1f}: max |err|/max|f| = {e:.2e}", file=sys.stderr)
    return max(worst.values())


def eta_of_l(l):
    y = mp.exp(mp.mpf(l))
    return mp.findroot(lambda e: fd_mp(0.5, e) - y, guess_series(float(l)))


def guess_series(l):
    y = np.exp(l)
    if y < 1.5:
        return float(np.log(y + y * y / 2 ** 1.5))
    e0 = (0.75 * np.sqrt(np.pi) * y) ** (2 / 3)
    return float(e0 * (1 - np.pi ** 2 / (12 * e0 * e0)))


def build_guess():
    npc = len(L_BREAKS) - 1
    coef = np.zeros((npc, NG))
    xs = cheb_nodes(NG)
    for p in range(npc):
        a, b = L_BREAKS[p], L_BREAKS[p + 1]
        vals = [eta_of_l(((b - a) * mp.mpf(x) + a + b) / 2) for x in xs]
        coef[p] = cheb_coeffs(vals)
    return coef


def report_guess(coef):
    worst = 0.0
    for p in range(len(L_BREAKS) - 1):
        a, b = L_BREAKS[p], L_BREAKS[p + 1]
        for x in np.linspace(-1, 1, 41):
            l = ((b - a) * x + a + b) / 2
            ref = float(eta_of_l(l))
            got = cheb_eval(coef[p], x)
            worst = max(worst, abs(got - ref) / max(1.0, abs(ref)))
    print(f"inverse guess: max |err|/max(1,|eta|) = {worst:.2e}", file=sys.stderr)
    return worst


def fmt(a):
    return ",\n".join("  " + ", ".join(f"{v:.17e}" for v in row) for row in a.reshape(-1, 4 if a.size % 4 == 0 else 1))


def main():
    coef = build_fd_tables()
    e1 = report_fd(coef)
    g = build_guess()
    e2 = report_guess(g)
    nb = len(BREAKS) - 1
    out = []
    out.append("// Generated by gen_fd_tables.py (mpmath polylogarithm, 40 digits). Do not edit.")
    out.append(f"// max scaled error of the F_j tables {e1:.2e}; of the inverse guess {e2:.2e}")
    out.append("#pragma once")
    out.append(f"#define OFDFT_FD_NC {NC}")
    out.append(f"#define OFDFT_FD_NB {nb}")
    out.append(f"#define OFDFT_FD_NREG {nb + 2}")
    out.append(f"#define OFDFT_FD_ETA_LO ({ETA_LO!r})")
    out.append(f"#define OFDFT_FD_ETA_HI ({ETA_HI!r})")
    out.append(f"#define OFDFT_GUESS_NC {NG}")
    out.append(f"#define OFDFT_GUESS_NP {len(L_BREAKS) - 1}")
    out.append("static constexpr double kFdBreaks[OFDFT_FD_NB + 1] = {" + ", ".join(repr(b) for b in BREAKS) + "};")
    out.append("static constexpr double kGuessBreaks[OFDFT_GUESS_NP + 1] = {" + ", ".join(repr(b) for b in L_BREAKS) + "};")
    out.append("// [region][order 3/2,1/2,-1/2,-3/2,-5/2,-7/2][coefficient]")
    flat = coef.reshape(-1)
    out.append("static const double kFdCheb[OFDFT_FD_NREG * 6 * OFDFT_FD_NC] = {")
    out.append(",\n".join("  " + ", ".join(f"{v:.17e}" for v in flat[i:i + 4]) for i in range(0, flat.size, 4)))
    out.append("};")
    gf = g.reshape(-1)
    out.append("static const double kGuessCheb[OFDFT_GUESS_NP * OFDFT_GUESS_NC] = {")
    out.append(",\n".join("  " + ", ".join(f"{v:.17e}" for v in gf[i:i + 4]) for i in range(0, gf.size, 4)))
    out.append("};")
    print("\n".join(out))


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Generate t_tables.h: FP64 Chebyshev expansions in ln t of the t-dependent
factors of the finite-T Thomas-Fermi and GGA free energies.

Every factor that depends on the reduced temperature t = T/T_F alone
(arXiv:1406.0835 Eqs. fTF, tred, vTF, xizeta, s_s, vftGGA and Table I) is
tabulated here, so the device evaluates one shared Chebyshev recurrence per
grid point instead of inverting F_{1/2} and evaluating six Fermi-Dirac
integrals.  Reference values come from mpmath at 60 digits:
  * eta from F_{1/2}(eta) = 4/(3 sqrt(pi)) t^(-3/2), F_j(eta) = -Li_{j+1}(-e^eta)
  * R = F_{3/2}/F_{1/2}; kappa = (5/3) t (eta - R); xi = (5/2) t R; zeta = xi - kappa
  * h~ = 3 F_{1/2} F_{-3/2} / F_{-1/2}^2 and its t-derivatives (chain rule in eta)
  * P_tau = (h~ - t h~')/xi, P_sigma = t h~'/zeta  (s_tau^2 = s^2 P_tau, s_sigma^2 = s^2 P_sigma)
Tabulated functions of l = ln t (t-derivatives multiplied by t):
  GGA: xi, zeta, t xi', t zeta', P_tau, P_sigma, t P_tau', t P_sigma'
  TF : kappa, zeta, t eta
Pieces overlap: piece j covers [L_LO + j H, L_LO + j H + W] with W = 2 H, so
any set of l values whose spread is at most H lies inside one piece (the
piece of the smallest value), and a wavefront of neighbouring grid points is
served by one piece with wave-uniform coefficients.  Each piece holds NC
first-kind Chebyshev coefficients per function.  Outside [L_LO, L_HI] the
device clamps l.

Usage: python gen_t_tables.py > t_tables.h   (error report on stderr)
"""
import os
import sys

import mpmath as mp

mp.mp.dps = 60
L_LO, L_HI, H, NC = -16.0, 24.0, 0.5, 22
W = 2 * H
TOL = {"xi": 2e-15, "zeta": 4e-15, "t_dxi": 2e-14, "t_dzeta": 2e-14, "p_tau": 2e-14, "p_sig": 2e-14,
       "t_dp_tau": 1e-13, "t_dp_sig": 1e-13, "kappa": 2e-15, "t_eta": 4e-15}
GGA_NAMES = ["xi", "zeta", "t_dxi", "t_dzeta", "p_tau", "p_sig", "t_dp_tau", "t_dp_sig"]
TF_NAMES = ["kappa", "zeta", "t_eta"]


def fd(j, eta):
    return -mp.re(mp.polylog(j + 1, -mp.exp(eta)))


def eta_of_t(t):
    y = 4 / (3 * mp.sqrt(mp.pi)) * t ** mp.mpf(-1.5)
    if y < 1:
        e = mp.log(y)
    else:
        e = (3 * mp.sqrt(mp.pi) * y / 4) ** (mp.mpf(2) / 3)
    for _ in range(200):
        f12 = fd(0.5, e)
        step = (f12 - y) / fd(-0.5, e)
        e -= step
        if abs(step) < mp.mpf(10) ** (-50) * max(1, abs(e)):
            break
    return e, y


def factors(l):
    t = mp.exp(mp.mpf(l))
    eta, y = eta_of_t(t)
    f32, f12, fm12, fm32, fm52, fm72 = (fd(j, eta) for j in (1.5, 0.5, -0.5, -1.5, -2.5, -3.5))
    R = f32 / f12
    kappa = mp.mpf(5) / 3 * t * (eta - R)
    xi = mp.mpf(5) / 2 * t * R
    zeta = xi - kappa
    deta = -mp.mpf(3) / 2 * f12 / (t * fm12)
    dR = deta * (1 - f32 * fm12 / f12 ** 2)
    dxi = mp.mpf(5) / 2 * (R + t * dR)
    dkappa = -zeta / t
    dzeta = dxi - dkappa
    h = 3 * f12 * fm32 / fm12 ** 2
    a = fm32 / fm12
    b = f12 * fm52 / fm12 ** 2
    c = -2 * f12 * fm32 ** 2 / fm12 ** 3
    h1 = 3 * (a + b + c)
    da = fm52 / fm12 - fm32 ** 2 / fm12 ** 2
    db = (fm12 * fm52 + f12 * fm72) / fm12 ** 2 - 2 * f12 * fm52 * fm32 / fm12 ** 3
    dc = -2 * fm32 ** 2 / fm12 ** 2 - 4 * f12 * fm32 * fm52 / fm12 ** 3 + 6 * f12 * fm32 ** 3 / fm12 ** 4
    h2 = 3 * (da + db + dc)
    d2eta = -mp.mpf(3) / 2 * (deta * (1 - f12 * fm32 / fm12 ** 2) / t - f12 / (t * t * fm12))
    dh = h1 * deta
    d2h = h2 * deta ** 2 + h1 * d2eta
    p_tau = (h - t * dh) / xi
    p_sig = t * dh / zeta
    dp_tau = (-t * d2h * xi - (h - t * dh) * dxi) / xi ** 2
    dp_sig = ((dh + t * d2h) * zeta - t * dh * dzeta) / zeta ** 2
    gga = [xi, zeta, t * dxi, t * dzeta, p_tau, p_sig, t * dp_tau, t * dp_sig]
    tf = [kappa, zeta, t * eta]
    return gga, tf


def piece_l(a, b, x):
    return ((b - a) * mp.mpf(x) + a + b) / 2


def cheb_coeffs(vals):
    n = len(vals)
    th = [mp.pi * (i + mp.mpf(1) / 2) / n for i in range(n)]
    out = []
    for m in range(n):
        out.append(2 * mp.fsum(vals[i] * mp.cos(m * th[i]) for i in range(n)) / n)
    out[0] /= 2
    return out


def cheb_eval(c, x):
    x = float(x)
    b1 = b2 = 0.0
    for k in range(len(c) - 1, 0, -1):
        b1, b2 = 2 * x * b1 - b2 + c[k], b1
    return x * b1 - b2 + c[0]


def fit_piece(a, b, nodes):
    vals = [factors(piece_l(a, b, x)) for x in nodes]
    gga = [[float(v) for v in cheb_coeffs([vv[0][f] for vv in vals])] for f in range(len(GGA_NAMES))]
    tf = [[float(v) for v in cheb_coeffs([vv[1][f] for vv in vals])] for f in range(len(TF_NAMES))]
    xs = [mp.mpf(-1) + mp.mpf(2) * i / 16 for i in range(17)]
    ref = [factors(piece_l(a, b, x)) for x in xs]
    errs = {}
    for f, n in enumerate(GGA_NAMES):
        scale = max(abs(float(r[0][f])) for r in ref)
        errs[n] = max(abs(cheb_eval(gga[f], x) - float(r[0][f])) for x, r in zip(xs, ref)) / scale
    for f, n in enumerate(TF_NAMES):
        scale = max(abs(float(r[1][f])) for r in ref)
        errs[n] = max(abs(cheb_eval(tf[f], x) - float(r[1][f])) for x, r in zip(xs, ref)) / scale
    return gga, tf, errs


def build_piece(j):
    nodes = [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / NC) for k in range(NC)]
    a = L_LO + j * H
    gga, tf, errs = fit_piece(a, a + W, nodes)
    bad = [n for n, e in errs.items() if e > TOL[n]]
    flag = (" ABOVE TOLERANCE: " + ", ".join(bad)) if bad else ""
    print(f"piece {j} [{a}, {a + W}] max err {max(errs.values()):.1e}{flag}", file=sys.stderr, flush=True)
    return gga, tf, errs


def main():
    import multiprocessing as mpr
    npieces = int(round((L_HI - L_LO) / H))
    with mpr.Pool(int(os.environ.get("GEN_PROCS", "6"))) as pool:
        pieces = pool.map(build_piece, range(npieces), chunksize=1)
    worst = {n: max(p[2][n] for p in pieces) for n in GGA_NAMES + TF_NAMES}
    for n, e in worst.items():
        print(f"{n}: max |err| / max|f| per piece = {e:.2e}", file=sys.stderr)
    out = ["// Generated by gen_t_tables.py (mpmath, 60 digits). Do not edit.",
           "// max error / piece scale: " + ", ".join(f"{n} {e:.1e}" for n, e in worst.items()),
           "#pragma once",
           f"#define OFDFT_T_LLO ({L_LO!r})",
           f"#define OFDFT_T_LHI ({L_HI!r})",
           f"#define OFDFT_T_H ({H!r})",
           f"#define OFDFT_T_W ({W!r})",
           f"#define OFDFT_T_NP {npieces}",
           f"#define OFDFT_T_NC {NC}",
           "// [piece][function][coefficient]; piece j spans l in [LLO + j H, LLO + j H + W]",
           "// GGA functions: " + ", ".join(GGA_NAMES),
           f"static const double kTGga[OFDFT_T_NP * {len(GGA_NAMES)} * OFDFT_T_NC] = {{"]
    flat = [v for p in pieces for f in range(len(GGA_NAMES)) for v in p[0][f]]
    out += ["  " + ", ".join(f"{v:.17e}" for v in flat[i:i + 4]) + "," for i in range(0, len(flat), 4)]
    out.append("};")
    out.append("// TF functions: " + ", ".join(TF_NAMES))
    out.append(f"static const double kTTf[OFDFT_T_NP * {len(TF_NAMES)} * OFDFT_T_NC] = {{")
    flat = [v for p in pieces for f in range(len(TF_NAMES)) for v in p[1][f]]
    out += ["  " + ", ".join(f"{v:.17e}" for v in flat[i:i + 4]) + "," for i in range(0, len(flat), 4)]
    out.append("};")
    print("\n".join(out))


if __name__ == "__main__":
    main()

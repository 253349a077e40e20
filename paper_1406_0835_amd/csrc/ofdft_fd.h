// Device Fermi-Dirac integrals, reduced-temperature factors and pointwise
// free-energy densities (arXiv:1406.0835 Sec. III A/B, Table I; PZ XC Sec. IV).
//
// Precision split: everything that depends on t alone (the inverse of F_{1/2},
// kappa, xi, zeta, h~ and their t-derivatives) is computed in FP64 in both the
// FP64 and the mixed path; the gradient-dependent assembly runs in R.
#pragma once
#include <hip/hip_runtime.h>

#include "fd_tables.h"

namespace ofdft {

__constant__ double c_fd_cheb[OFDFT_FD_NREG * 6 * OFDFT_FD_NC];
__constant__ double c_guess_cheb[OFDFT_GUESS_NP * OFDFT_GUESS_NC];

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kYPref = 0.75225277806367504925;     // 4/(3 sqrt(pi)): F_{1/2}(eta) = kYPref t^-3/2
constexpr double kCTF = 2.87123400018819181594;       // (3/10)(3 pi^2)^(2/3)
constexpr double kS2Den = 38.2831200025092242125;     // 4 (3 pi^2)^(2/3)
constexpr double kThreePi2 = 29.6088132032680740;     // 3 pi^2
constexpr double kDensityFloor = 1.0e-12;

// The six normalised FD integrals F_j(eta), j = 3/2, 1/2, -1/2, -3/2, -5/2, -7/2.
struct FD6 {
  double f32, f12, fm12, fm32, fm52, fm72;
};

// Six Chebyshev series at one x with a shared T_k recurrence.
__device__ __forceinline__ void cheb6(const double* __restrict__ c, double x, double* s) {
#pragma unroll
  for (int j = 0; j < 6; ++j) s[j] = c[j * OFDFT_FD_NC] + c[j * OFDFT_FD_NC + 1] * x;
  double t0 = 1.0, t1 = x;
  const double x2 = 2.0 * x;
#pragma unroll 4
  for (int k = 2; k < OFDFT_FD_NC; ++k) {
    const double t2 = x2 * t1 - t0;
#pragma unroll
    for (int j = 0; j < 6; ++j) s[j] = fma(c[j * OFDFT_FD_NC + k], t2, s[j]);
    t0 = t1;
    t1 = t2;
  }
}

__device__ __forceinline__ FD6 fd6(double eta) {
  int r;
  double x;
  if (eta < OFDFT_FD_ETA_LO) {
    r = 0;
    x = 2.0 * exp(eta - OFDFT_FD_ETA_LO) - 1.0;
  } else if (eta >= OFDFT_FD_ETA_HI) {
    r = OFDFT_FD_NB + 1;
    x = 2.0 * OFDFT_FD_ETA_HI / eta - 1.0;
  } else {
    r = 1;
#pragma unroll
    for (int b = 1; b < OFDFT_FD_NB; ++b) r += (eta >= kFdBreaks[b]) ? 1 : 0;
    const double a = kFdBreaks[r - 1], bb = kFdBreaks[r];
    x = (2.0 * eta - a - bb) / (bb - a);
  }
  double s[6];
  // Neighbouring grid points usually share a region: then the region index is
  // wave-uniform and the coefficients come through scalar loads.
  const int r0 = __builtin_amdgcn_readfirstlane(r);
  if (__all(r == r0)) {
    cheb6(c_fd_cheb + r0 * 6 * OFDFT_FD_NC, x, s);
  } else {
    cheb6(c_fd_cheb + r * 6 * OFDFT_FD_NC, x, s);
  }
  FD6 F;
  if (r == 0) {
    const double z = exp(eta);
    F = {s[0] * z, s[1] * z, s[2] * z, s[3] * z, s[4] * z, s[5] * z};
  } else if (r == OFDFT_FD_NB + 1) {
    const double se = sqrt(eta), ie = 1.0 / eta;
    const double p12 = se, p32 = eta * se, p52 = eta * eta * se;
    const double pm12 = 1.0 / se, pm32 = pm12 * ie, pm52 = pm32 * ie;
    F = {s[0] * p52, s[1] * p32, s[2] * p12, s[3] * pm12, s[4] * pm32, s[5] * pm52};
  } else {
    F = {s[0], s[1], s[2], s[3], s[4], s[5]};
  }
  return F;
}

// Starting value for eta with F_{1/2}(eta) = y: series inversions outside the
// tabulated range of ln y, a Chebyshev piece inside.
__device__ __forceinline__ double eta_guess(double y) {
  const double l = log(y);
  if (l < kGuessBreaks[0]) {
    // F_{1/2} = z - z^2/2^{3/2} + z^3/3^{3/2} - ...  =>  z = y + y^2/2^{3/2} + b y^3
    const double z = y + y * y * (0.35355339059327376220 + y * 0.05754991027012474);
    return log(z);
  }
  if (l >= kGuessBreaks[OFDFT_GUESS_NP]) {
    // Sommerfeld: y = (4/(3 sqrt pi)) eta^{3/2} (1 + pi^2/(8 eta^2) + 7 pi^4/(640 eta^4))
    const double e0 = cbrt(y / kYPref);
    const double e00 = e0 * e0;
    double e = e00;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double ie2 = 1.0 / (e * e);
      const double corr = 1.0 + ie2 * (1.2337005501361698 + ie2 * 1.0654866825427722);
      e = e00 / cbrt(corr * corr);
    }
    return e;
  }
  int p = 0;
#pragma unroll
  for (int b = 1; b < OFDFT_GUESS_NP; ++b) p += (l >= kGuessBreaks[b]) ? 1 : 0;
  const double a = kGuessBreaks[p], bb = kGuessBreaks[p + 1];
  const double x = (2.0 * l - a - bb) / (bb - a);
  const double* c = c_guess_cheb + p * OFDFT_GUESS_NC;
  // Clenshaw
  double b1 = 0.0, b2 = 0.0;
  for (int k = OFDFT_GUESS_NC - 1; k >= 1; --k) {
    const double b0 = fma(2.0 * x, b1, c[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fma(x, b1, c[0] - b2);
}

// Reduced-temperature factors and their t-derivatives.
struct TFac {
  double eta, kappa, dkappa, xi, dxi, zeta, dzeta, h, dh, d2h;
};

// full = false computes only eta, kappa, zeta (ftTF needs no more).
template <bool FULL>
__device__ __forceinline__ TFac t_factors(double t) {
  const double y = kYPref / (t * sqrt(t));
  const double e0 = eta_guess(y);
  FD6 F = fd6(e0);
  // one Newton step on F_{1/2}(eta) = y, then a first-order Taylor shift of
  // every order to the corrected eta (the shift is below 1e-9)
  const double d = (y - F.f12) / F.fm12;
  const double eta = e0 + d;
  F.f32 = fma(F.f12, d, F.f32);
  F.f12 = y;
  F.fm12 = fma(F.fm32, d, F.fm12);
  F.fm32 = fma(F.fm52, d, F.fm32);
  F.fm52 = fma(F.fm72, d, F.fm52);
  TFac o;
  const double R = F.f32 / F.f12;
  o.eta = eta;
  o.kappa = (5.0 / 3.0) * t * (eta - R);
  o.xi = 2.5 * t * R;
  o.zeta = o.xi - o.kappa;
  o.dkappa = -o.zeta / t;
  if constexpr (FULL) {
    const double deta = -1.5 * F.f12 / (t * F.fm12);
    const double q = F.f32 * F.fm12 / (F.f12 * F.f12);
    o.dxi = 2.5 * (R + t * deta * (1.0 - q));
    o.dzeta = o.dxi + o.zeta / t;
    // h~ = 3 F12 Fm32 / Fm12^2 and eta-derivatives
    const double im = 1.0 / F.fm12;
    const double a = F.fm32 * im;             // Fm32/Fm12
    const double bq = F.f12 * im;             // F12/Fm12
    o.h = 3.0 * bq * a;
    const double h1 = 3.0 * (a + bq * F.fm52 * im - 2.0 * bq * a * a);
    const double da = F.fm52 * im - a * a;
    const double db = F.fm52 * im + bq * F.fm72 * im - 2.0 * bq * F.fm52 * im * a;
    const double dc = -2.0 * a * a - 4.0 * bq * a * F.fm52 * im + 6.0 * bq * a * a * a;
    const double h2 = 3.0 * (da + db + dc);
    const double d2eta = -1.5 * (deta * (1.0 - bq * a) / t - bq / (t * t));
    o.dh = h1 * deta;
    o.d2h = h2 * deta * deta + h1 * d2eta;
  } else {
    o.dxi = o.dzeta = o.h = o.dh = o.d2h = 0.0;
  }
  return o;
}

// ---------------------------------------------------------------- enhancement factors
// Functional ids (match the C ABI).
enum { F_TF = 0, F_SGA = 1, F_VWTF = 2, F_VT84F = 3, F_KST2 = 4, F_TW = 5, F_APBEF = 6 };

struct EnhParams {
  int kind;      // 0: 1 + mu x ; 1: 1 + c1 x/(1 + a1 x) ; 2: VT84F
  double c1, a1; // mu for kind 0
};

// F(x) and dF/dx with x = s^2 (Eqs. VT84F, KST2F, SGA-F).
template <typename R>
__device__ __forceinline__ void enhancement(const EnhParams& p, R x, R& F, R& dF) {
  if (p.kind == 0) {
    F = R(1) + R(p.c1) * x;
    dF = R(p.c1);
  } else if (p.kind == 1) {
    const R den = R(1) + R(p.a1) * x;
    F = R(1) + R(p.c1) * x / den;
    dF = R(p.c1) / (den * den);
  } else {
    const R mu = R(2.778), al = R(1.2965);
    const R ex = exp(-al * x);
    const R den = R(1) + mu * x;
    const R t1 = -mu * x * ex / den;
    const R dt1 = -mu * ex * (R(1) - al * x - al * mu * x * x) / (den * den);
    // (1 - exp(-al x^2)) (1/x - 1), with its small-x series
    R q, qx, qx2;
    if (x < R(1e-4)) {
      qx = al * x - R(0.5) * al * al * x * x * x;
      qx2 = al - R(0.5) * al * al * x * x;
      q = qx * x;
    } else {
      q = -expm1(-al * x * x);
      qx = q / x;
      qx2 = qx / x;
    }
    F = R(1) + t1 + (qx - q) + R(5.0 / 3.0) * x;
    dF = dt1 + R(2) * al * exp(-al * x * x) * (R(1) - x) - qx2 + R(5.0 / 3.0);
  }
}

// ---------------------------------------------------------------- PZ81 LDA XC
// eps_xc and v_xc of the unpolarised Perdew-Zunger (1981) parametrisation.
// The high-density C and D follow from continuity of eps_c and its slope at
// rs = 1 (the published 0.0020 and -0.0116 are these values rounded).
constexpr double kPzGamma = -0.1423, kPzB1 = 1.0529, kPzB2 = 0.3334, kPzA = 0.0311, kPzB = -0.048;
constexpr double kPzDen1 = 1.0 + kPzB1 + kPzB2;
constexpr double kPzD = kPzGamma / kPzDen1 - kPzB;
constexpr double kPzC = -kPzGamma * (0.5 * kPzB1 + kPzB2) / (kPzDen1 * kPzDen1) - kPzA - kPzD;

template <typename R>
__device__ __forceinline__ void pz81(R n, R& eps, R& v) {
  const R rs = cbrt(R(0.75) / (R(kPi) * n));
  const R ex = R(-0.45816529328314287) / rs;
  R ec, dec;
  if (rs >= R(1)) {
    const R sq = sqrt(rs);
    const R den = R(1) + R(kPzB1) * sq + R(kPzB2) * rs;
    ec = R(kPzGamma) / den;
    dec = -R(kPzGamma) * (R(0.5 * kPzB1) / sq + R(kPzB2)) / (den * den);
  } else {
    const R lr = log(rs);
    ec = R(kPzA) * lr + R(kPzB) + R(kPzC) * rs * lr + R(kPzD) * rs;
    dec = R(kPzA) / rs + R(kPzC) * (lr + R(1)) + R(kPzD);
  }
  eps = ex + ec;
  v = R(4.0 / 3.0) * ex + ec - rs * dec / R(3);
}

// ---------------------------------------------------------------- pointwise F_s
// ftTF at density n (already floored): f = tau0 kappa, v = T eta (the uniform
// gas chemical potential, equal to Eq. vTF), T s = tau0 zeta.
__device__ __forceinline__ void tf_point(double n, double T, double& f, double& v, double& ts) {
  const double t = 2.0 * T / cbrt(kThreePi2 * n * kThreePi2 * n);
  const TFac a = t_factors<false>(t);
  const double A = kCTF * n * cbrt(n * n);
  f = A * a.kappa;
  v = T * a.eta;
  ts = A * a.zeta;
}

// Generic finite-T GGA (Eq. FGGA) at density n (floored) and sigma = |grad n|^2.
// Outputs f, df/dn at fixed sigma, df/dsigma and T s. The t-factors are FP64;
// the enhancement-factor assembly runs in R.
template <typename R>
__device__ __forceinline__ void gga_point(double n, R sigma, double T, const EnhParams& ep,
                                          double& f_out, R& dfdn, R& dfds, double& ts_out) {
  const double n23 = cbrt(n * n);
  const double t = 2.0 * T / (cbrt(kThreePi2 * kThreePi2) * n23);
  const TFac a = t_factors<true>(t);
  const double A = kCTF * n * n23;
  const double invden = 1.0 / (kS2Den * n * n * n23);
  const double p_tau = (a.h - t * a.dh) / a.xi;
  const double p_sig = t * a.dh / a.zeta;
  const double dp_tau = (-t * a.d2h * a.xi - (a.h - t * a.dh) * a.dxi) / (a.xi * a.xi);
  const double dp_sig = ((a.dh + t * a.d2h) * a.zeta - t * a.dh * a.dzeta) / (a.zeta * a.zeta);
  const R s2 = sigma * R(invden);
  const R x_tau = s2 * R(p_tau);
  const R x_sig = s2 * R(p_sig);
  R Ft, dFt, G, dG;
  enhancement<R>(ep, x_tau, Ft, dFt);
  enhancement<R>(ep, x_sig, G, dG);
  const R Fs = R(2) - G;
  const R dFs = -dG;
  const R xi = R(a.xi), zeta = R(a.zeta);
  const R fr = R(A) * (xi * Ft - zeta * Fs);
  const R rn = R(1.0 / n);
  const R dtdn = R(-2.0 / 3.0) * R(t) * rn;
  const R ds2dn = R(-8.0 / 3.0) * s2 * rn;
  dfdn = R(5.0 / 3.0) * fr * rn +
         R(A) * ((R(a.dxi) * Ft - R(a.dzeta) * Fs) * dtdn +
                 xi * dFt * (ds2dn * R(p_tau) + s2 * R(dp_tau) * dtdn) -
                 zeta * dFs * (ds2dn * R(p_sig) + s2 * R(dp_sig) * dtdn));
  dfds = R(A) * (xi * dFt * R(p_tau) - zeta * dFs * R(p_sig)) * R(invden);
  f_out = double(fr);
  ts_out = A * a.zeta * double(Fs);
}

}  // namespace ofdft

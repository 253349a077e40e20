// Device reduced-temperature factors and pointwise free-energy densities
// (arXiv:1406.0835 Sec. III A/B, Table I; PZ XC Sec. IV).
//
// Precision split: everything that depends on t alone (the Fermi-Dirac
// inversion eta(t), kappa, xi, zeta, h~ and their t-derivatives, folded into
// the tabulated factors) is evaluated in FP64 in both the FP64 and the mixed
// path; the gradient-dependent assembly and XC run in R.
#pragma once
#include <hip/hip_runtime.h>

#include "t_tables.h"

namespace ofdft {

// Device copies of the t-factor tables, stored coefficient-major within a piece:
// c[(piece * NC + k) * NF + f] (the generated tables are function-major), so the k-th
// Chebyshev coefficients of all NF functions of a piece are one contiguous 8 NF-byte run
// that a single wide scalar load fetches.
__constant__ double c_t_gga[OFDFT_T_NP * 8 * OFDFT_T_NC];
__constant__ double c_t_tf[OFDFT_T_NP * 3 * OFDFT_T_NC];

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kCTF = 2.87123400018819181594;       // (3/10)(3 pi^2)^(2/3)
constexpr double kS2Den = 38.2831200025092242125;     // 4 (3 pi^2)^(2/3)
constexpr double kThreePi2 = 29.6088132032680758565;  // 3 pi^2
constexpr double kThreePi2_23 = 9.57078000062730605; // (3 pi^2)^(2/3)
constexpr double kLn3Pi2 = 3.38807206036691003968;     // ln(3 pi^2)
constexpr double kDensityFloor = 1.0e-12;
constexpr double kLn3Over4Pi = -1.43241195830118110158;  // ln(3/(4 pi))

// Chebyshev terms per GGA t-factor in the FP32 path, in table order (xi, zeta,
// t xi', t zeta', P_tau, P_sigma, t P_tau', t P_sigma').  Its t-factors are
// rounded to FP32, and on every piece the dropped coefficients sum to less than
// 3e-8 of the factor each entry belongs to (xi, zeta, P_tau or P_sigma for the
// t-derivatives), below FP32 unit roundoff (6e-8).
constexpr int kTermsFp32[8] = {8, 9, 9, 10, 11, 12, 12, 14};
constexpr int kTermsFp32Max = 14;

// ln x for a positive normal double.  Reduction x = 2^e (1 + f) with 1 + f in
// [sqrt(1/2), sqrt(2)) and s = f/(2 + f), so ln(1 + f) = 2 atanh(s) =
// f - (f^2/2 - s (f^2/2 + R)) with R = sum_k 2 s^(2k)/(2k + 1); the exact f
// leads and the series only corrects it (the arrangement of fdlibm's log).
// |s| <= 0.1716, so nine terms of R leave a truncation below 3e-17 relative;
// ln 2 is split so that e ln2_hi is exact.  Under 1 ulp against a long-double
// logarithm, at a third of the instructions of the general double log.
__device__ __forceinline__ double ln_pos(double x) {
  int e;
  double m = frexp(x, &e);
  if (m < 0.70710678118654752440) {
    m += m;
    --e;
  }
  const double f = m - 1.0;
  const double d = 2.0 + f;
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  r = fma(fma(-d, r, 1.0), r, r);
  const double s = f * r, z = s * s;
  double R = 2.0 / 19.0;
  R = fma(R, z, 2.0 / 17.0);
  R = fma(R, z, 2.0 / 15.0);
  R = fma(R, z, 2.0 / 13.0);
  R = fma(R, z, 2.0 / 11.0);
  R = fma(R, z, 2.0 / 9.0);
  R = fma(R, z, 2.0 / 7.0);
  R = fma(R, z, 2.0 / 5.0);
  R = fma(R, z, 2.0 / 3.0);
  R *= z;
  const double hfsq = 0.5 * f * f, ed = double(e);
  constexpr double kLn2Hi = 6.93147180369123816490e-01, kLn2Lo = 1.90821492927058770002e-10;
  return fma(ed, kLn2Hi, f - (hfsq - fma(s, hfsq + R, ed * kLn2Lo)));
}

// NF Chebyshev series of one piece (coefficients c[k * NF + f], first K terms used)
// at one x, sharing the T_k recurrence.
// With TRIM (the FP32 path of the GGA table) function f takes its first kTermsFp32[f] terms.
template <int NF, int K, bool TRIM = false>
__device__ __forceinline__ void cheb_series(const double* __restrict__ c, double x, double* s) {
  static_assert(!TRIM || NF == 8, "trimmed series are defined for the GGA table");
#pragma unroll
  for (int f = 0; f < NF; ++f) s[f] = fma(c[NF + f], x, c[f]);
  double t0 = 1.0, t1 = x;
  const double x2 = 2.0 * x;
#pragma unroll
  for (int k = 2; k < K; ++k) {
    const double t2 = fma(x2, t1, -t0);
#pragma unroll
    for (int f = 0; f < NF; ++f)
      if (!TRIM || k < kTermsFp32[f]) s[f] = fma(c[k * NF + f], t2, s[f]);
    t0 = t1;
    t1 = t2;
    // keeps the wave-uniform coefficient loads of later terms from being hoisted above this
    // one: all of them live at once overflow the scalar registers into VGPR lanes
    asm volatile("" ::: "memory");
  }
}

// Smallest cell among the lanes in `pending` (a ballot mask): start from the
// first pending lane and step to any pending lane with a smaller cell.  Only
// lanes reported by __ballot are read, so a partly populated wavefront cannot
// contribute stale values; the steps are bounded by the wavefront size.
__device__ __forceinline__ int min_pending_cell(int cell, bool pending_lane, unsigned long long pending) {
  int pm = __builtin_amdgcn_readlane(cell, __ffsll((long long)pending) - 1);
  unsigned long long lower;
  for (int step = 0; step < 64 && (lower = __ballot(pending_lane && cell < pm)) != 0ull; ++step)
    pm = __builtin_amdgcn_readlane(cell, __ffsll((long long)lower) - 1);
  return pm;
}

// The t-dependent factors at l = ln t (clamped to the tabulated range).
// Piece j spans [LLO + j H, LLO + j H + W] with W = 2 H.  Each pass takes the
// smallest cell among the lanes still pending and evaluates that piece for the
// whole wavefront with wave-uniform (scalar) coefficient loads; every pending
// lane inside the piece takes the result.  Neighbouring points have similar
// densities, so one pass usually serves the whole wavefront (always, when the
// spread of l across the wavefront is at most H).
template <int NF, int K = OFDFT_T_NC, bool TRIM = false>
__device__ __forceinline__ void t_table(const double* __restrict__ table, double l, double* s) {
  static_assert(K >= 2 && K <= OFDFT_T_NC, "series length");
  l = fmin(fmax(l, OFDFT_T_LLO), OFDFT_T_LHI);
  int cell = (int)((l - OFDFT_T_LLO) * (1.0 / OFDFT_T_H));
  cell = cell < 0 ? 0 : (cell >= OFDFT_T_NP ? OFDFT_T_NP - 1 : cell);
  // First pass: the piece of the smallest cell, written straight into s.  Every
  // lane of that cell has l - a < H, i.e. x < 0, so each pass completes at least
  // one lane; the loop below (bounded by the wavefront size) serves the rest.
  unsigned long long pending = __ballot(true);
  int pm = min_pending_cell(cell, true, pending);
  double a = OFDFT_T_LLO + pm * OFDFT_T_H;
  double x = (l - a) * (2.0 / OFDFT_T_W) - 1.0;
  cheb_series<NF, K, TRIM>(table + pm * NF * OFDFT_T_NC, x, s);
  bool done = x <= 1.0;
  pending = __ballot(!done);
  for (int pass = 1; pending != 0ull && pass < 64; ++pass) {
    pm = min_pending_cell(cell, !done, pending);
    a = OFDFT_T_LLO + pm * OFDFT_T_H;
    x = (l - a) * (2.0 / OFDFT_T_W) - 1.0;
    double r[NF];
    cheb_series<NF, K, TRIM>(table + pm * NF * OFDFT_T_NC, x, r);
    if (!done && x <= 1.0) {
#pragma unroll
      for (int f = 0; f < NF; ++f) s[f] = r[f];
      done = true;
    }
    pending = __ballot(!done);
  }
}

// l = ln t with t = 2T/(3 pi^2 n)^(2/3) (Eq. tred): ln t = lt0 - (2/3) ln n,
// lt0 = ln(2T) - (2/3) ln(3 pi^2).
__host__ __device__ inline double lt_offset(double T) { return log(2.0 * T) - (2.0 / 3.0) * kLn3Pi2; }

// ---------------------------------------------------------------- enhancement factors
// Functional ids (match the C ABI).
enum { F_TF = 0, F_SGA = 1, F_VWTF = 2, F_VT84F = 3, F_KST2 = 4, F_TW = 5, F_APBEF = 6 };

struct EnhParams {
  int kind;      // 0: 1 + mu x ; 1: 1 + c1 x/(1 + a1 x) ; 2: VT84F
  double c1, a1; // mu for kind 0
};

// Reciprocal: the hardware v_rcp_f32 (1 ulp) in FP32, a correctly rounded
// division in FP64.
template <typename R>
__device__ __forceinline__ R rcp(R x);
template <>
__device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }

// F(x) and dF/dx with x = s^2 (Eqs. VT84F, KST2F, SGA-F).
template <typename R>
__device__ __forceinline__ void enhancement(const EnhParams& p, R x, R& F, R& dF) {
  if (p.kind == 0) {
    F = R(1) + R(p.c1) * x;
    dF = R(p.c1);
  } else if (p.kind == 1) {
    const R rden = rcp<R>(R(1) + R(p.a1) * x);
    F = R(1) + R(p.c1) * x * rden;
    dF = R(p.c1) * rden * rden;
  } else {
    const R mu = R(2.778), al = R(1.2965);
    const R ex = exp(-al * x);
    const R rden = rcp<R>(R(1) + mu * x);
    const R t1 = -mu * x * ex * rden;
    // d/dx of -mu x e^{-al x}/(1 + mu x) = -mu e^{-al x} rden (rden - al x): no x^2, so
    // the FP32 path stays finite at the huge x of near-empty grid points
    const R dt1 = -mu * ex * rden * (rden - al * x);
    // q = 1 - exp(-al x^2) and the term q (1/x - 1), with its small-x series
    R q, qx, qx2;
    if (x < R(1e-4)) {
      qx = al * x - R(0.5) * al * al * x * x * x;
      qx2 = al - R(0.5) * al * al * x * x;
      q = qx * x;
    } else {
      const R rx = rcp<R>(x);
      q = -expm1(-al * x * x);
      qx = q * rx;
      qx2 = qx * rx;
    }
    F = R(1) + t1 + (qx - q) + R(5.0 / 3.0) * x;
    dF = dt1 + R(2) * al * (R(1) - q) * (R(1) - x) - qx2 + R(5.0 / 3.0);
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

// rs = (3/(4 pi n))^(1/3) and ln rs are formed from ln n, so neither a cube
// root nor a logarithm is taken here.
template <typename R>
__device__ __forceinline__ void pz81(double ln_n, R& eps, R& v) {
  const R lr = R((kLn3Over4Pi - ln_n) * (1.0 / 3.0));
  const R rs = exp(lr);
  const R rrs = rcp<R>(rs);
  const R ex = R(-0.45816529328314287) * rrs;
  R ec, dec;
  if (rs >= R(1)) {
    const R sq = sqrt(rs);
    const R rden = rcp<R>(R(1) + R(kPzB1) * sq + R(kPzB2) * rs);
    ec = R(kPzGamma) * rden;
    dec = -R(kPzGamma) * (R(0.5 * kPzB1) * sq * rrs + R(kPzB2)) * (rden * rden);
  } else {
    ec = R(kPzA) * lr + R(kPzB) + R(kPzC) * rs * lr + R(kPzD) * rs;
    dec = R(kPzA) * rrs + R(kPzC) * (lr + R(1)) + R(kPzD);
  }
  eps = ex + ec;
  v = R(4.0 / 3.0) * ex + ec - rs * dec * R(1.0 / 3.0);
}

// ---------------------------------------------------------------- KSDT finite-T LDA XC
// Eq. fit2 (spin-unpolarised, omega = 1):
//   f_xc = -(1/rs) (a + b rs^(1/2) + c rs) / (1 + d rs^(1/2) + e rs),
// with a(t)..e(t) and their parameters from the publication the paper cites for the fit
// (Karasiev, Sjostrom, Dufty, Trickey, PRL 112, 076403 (2014), unpolarised set):
//   a = 0.610887 tanh(1/t) (0.75 + 3.04363 t^2 - 0.09227 t^3 + 1.7035 t^4)/(1 + 8.31051 t^2 + 5.1105 t^4)
//   b, d = tanh(1/sqrt t) (p0 + p1 t^2 + p2 t^4)/(1 + q1 t^2 + q2 t^4);  e the same with tanh(1/t)
//   c = (c1 + c2 exp(-c3/t)) e.
// The potential is Eq. vxc1, v = f - (rs/3) df/drs - (2t/3) df/dt, and the entropy term
// T s_xc = -t df/dt.  Everything here is FP64 in both paths: t reaches ~1e10 at nearly
// empty points (t^4 overflows FP32) and the fit carries exponentially small terms.
struct KsdtRat {
  double p0, p1, p2, q1, q2;
};
constexpr KsdtRat kKsdtB{0.283997, 48.932154, 0.370919, 61.095357, 0.871837};
constexpr KsdtRat kKsdtD{0.579824, 94.537454, 97.839603, 59.939999, 24.388037};
constexpr KsdtRat kKsdtE{0.212036, 16.731249, 28.485792, 34.028876, 17.235515};
constexpr double kKsdtC1 = 0.870089, kKsdtC2 = 0.193077, kKsdtC3 = 2.414644;

// r = P(u)/Q(u) in u = t^2 and t dr/dt
__device__ __forceinline__ void ksdt_ratio(const KsdtRat& k, double u, double& r, double& tr) {
  const double P = k.p0 + u * (k.p1 + u * k.p2);
  const double Q = 1.0 + u * (k.q1 + u * k.q2);
  const double tP = u * (2.0 * k.p1 + 4.0 * k.p2 * u);
  const double tQ = u * (2.0 * k.q1 + 4.0 * k.q2 * u);
  const double iQ = 1.0 / Q;
  r = P * iQ;
  tr = (tP - r * tQ) * iQ;
}

// f_xc, v_xc and T s_xc per electron from ln n and l = ln t.
__device__ __forceinline__ void ksdt_point(double ln_n, double l, double& f, double& v, double& ts) {
  const double t = exp(l);
  const double u = t * t;
  const double rs = exp((kLn3Over4Pi - ln_n) * (1.0 / 3.0));
  const double q = sqrt(rs);
  const double it = 1.0 / t;
  const double th1 = tanh(it);                      // tanh(1/t) and t d/dt of it
  const double tth1 = -(1.0 - th1 * th1) * it;
  const double isq = 1.0 / sqrt(t);
  const double th2 = tanh(isq);                     // tanh(1/sqrt t) and t d/dt of it
  const double tth2 = -0.5 * (1.0 - th2 * th2) * isq;
  // a(t): its numerator has a t^3 term
  const double Pa = 0.75 + u * (3.04363 - 0.09227 * t + 1.7035 * u);
  const double tPa = u * (2.0 * 3.04363 - 3.0 * 0.09227 * t + 4.0 * 1.7035 * u);
  const double Qa = 1.0 + u * (8.31051 + 5.1105 * u);
  const double tQa = u * (2.0 * 8.31051 + 4.0 * 5.1105 * u);
  const double ra = Pa / Qa, tra = (tPa - ra * tQa) / Qa;
  const double a = 0.610887 * th1 * ra, ta = 0.610887 * (tth1 * ra + th1 * tra);
  double rb, trb, rd, trd, re, tre;
  ksdt_ratio(kKsdtB, u, rb, trb);
  ksdt_ratio(kKsdtD, u, rd, trd);
  ksdt_ratio(kKsdtE, u, re, tre);
  const double b = th2 * rb, tb = tth2 * rb + th2 * trb;
  const double d = th2 * rd, td = tth2 * rd + th2 * trd;
  const double e = th1 * re, te = tth1 * re + th1 * tre;
  const double ex = exp(-kKsdtC3 * it);
  const double cp = kKsdtC1 + kKsdtC2 * ex;
  const double c = cp * e, tc = kKsdtC2 * ex * kKsdtC3 * it * e + cp * te;
  const double N = a + b * q + c * rs;
  const double D = 1.0 + d * q + e * rs;
  const double iD = 1.0 / D, irs = 1.0 / rs;
  f = -N * irs * iD;
  // rs df/drs and t df/dt
  const double rs_frs = -f - ((0.5 * b * q + c * rs) * D - N * (0.5 * d * q + e * rs)) * irs * iD * iD;
  const double t_ft = -((ta + tb * q + tc * rs) * D - N * (td * q + te * rs)) * irs * iD * iD;
  v = f - (1.0 / 3.0) * rs_frs - (2.0 / 3.0) * t_ft;
  ts = -t_ft;
}

// XC at one point: PZ81 (xc == 1, in R) or KSDT (xc == 2, FP64); adds the potential to
// vl and n eps (the XC free energy density) and n T s_xc to the sums.
template <typename R, typename V>
__device__ __forceinline__ void xc_point(int xc, double n, double ln_n, double lt0, V& vl, double& exc,
                                         double& tsxc) {
  if (xc == 1) {
    R eps, vxc;
    pz81<R>(ln_n, eps, vxc);
    vl += V(vxc);
    exc += n * double(eps);
  } else if (xc == 2) {
    double fx, vx, tsx;
    ksdt_point(ln_n, lt0 - (2.0 / 3.0) * ln_n, fx, vx, tsx);
    vl += V(vx);
    exc += n * fx;
    tsxc += n * tsx;
  }
}

// ---------------------------------------------------------------- pointwise F_s
// ftTF at density n (already floored): f = tau0 kappa, v = T eta (the uniform
// gas chemical potential, equal to Eq. vTF), T s = tau0 zeta.  T eta is formed
// as (t eta) T/t with T/t = (3 pi^2 n)^(2/3)/2.
__device__ __forceinline__ void tf_point(double n, double ln_n, double lt0, double& f, double& v, double& ts) {
  double s[3];
  t_table<3>(c_t_tf, lt0 - (2.0 / 3.0) * ln_n, s);   // kappa, zeta, t eta
  const double n23 = exp((2.0 / 3.0) * ln_n);
  const double A = kCTF * n * n23;
  f = A * s[0];
  ts = A * s[1];
  v = 0.5 * kThreePi2_23 * n23 * s[2];
}

// Generic finite-T GGA (Eq. FGGA) at density n (floored) and sigma = |grad n|^2.
// Outputs f, df/dn at fixed sigma, df/dsigma and T s.  The t-factors are FP64
// table values; the enhancement-factor assembly runs in R.
template <typename R>
__device__ __forceinline__ void gga_point(double n, double ln_n, R sigma, double lt0, const EnhParams& ep,
                                          double& f_out, R& dfdn, R& dfds, double& ts_out) {
  double a[8];   // xi, zeta, t xi', t zeta', P_tau, P_sigma, t P_tau', t P_sigma'
  t_table<8, sizeof(R) == 4 ? kTermsFp32Max : OFDFT_T_NC, sizeof(R) == 4>(c_t_gga, lt0 - (2.0 / 3.0) * ln_n, a);
  const R nr = R(n);
  const R n23 = exp(R((2.0 / 3.0) * ln_n));
  const R A = R(kCTF) * nr * n23;
  const R rn = rcp<R>(nr);
  const R invden = R(1.0 / kS2Den) * rn * rn * rcp<R>(n23);
  const R s2 = sigma * invden;
  const R p_tau = R(a[4]), p_sig = R(a[5]);
  const R x_tau = s2 * p_tau;
  const R x_sig = s2 * p_sig;
  R Ft, dFt, G, dG;
  enhancement<R>(ep, x_tau, Ft, dFt);
  enhancement<R>(ep, x_sig, G, dG);
  const R Fs = R(2) - G;
  const R dFs = -dG;
  const R xi = R(a[0]), zeta = R(a[1]);
  const R fr = A * (xi * Ft - zeta * Fs);
  // df/dn at fixed sigma, with dt/dn = -(2/3) t/n and ds^2/dn = -(8/3) s^2/n, grouped
  // around A/n = c_TF n^(2/3) so that no FP32 intermediate overflows where n is tiny
  // and s^2 huge:
  //   df/dn = (A/n) [ (5/3)(xi F_t - zeta F_s) - (2/3)(t xi' F_t - t zeta' F_s)
  //                   - s^2 xi F_t' ((8/3) P_t + (2/3) t P_t') + s^2 zeta F_s' ((8/3) P_s + (2/3) t P_s') ]
  const R An = R(kCTF) * n23;
  dfdn = An * (R(5.0 / 3.0) * (xi * Ft - zeta * Fs) - R(2.0 / 3.0) * (R(a[2]) * Ft - R(a[3]) * Fs) -
               s2 * (xi * dFt * (R(8.0 / 3.0) * p_tau + R(2.0 / 3.0) * R(a[6])) -
                     zeta * dFs * (R(8.0 / 3.0) * p_sig + R(2.0 / 3.0) * R(a[7]))));
  // df/dsigma = A (ds^2/dsigma) (xi F_t' P_t - zeta F_s' P_s), A ds^2/dsigma = (c_TF / S) / n
  dfds = R(kCTF / kS2Den) * rn * (xi * dFt * p_tau - zeta * dFs * p_sig);
  f_out = double(fr);
  ts_out = double(A * zeta * Fs);
}

}  // namespace ofdft

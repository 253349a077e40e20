// C ABI of the MI355X finite-temperature OF-DFT library: argument checks,
// context state machine, the host side of the minimisers (scalar decisions;
// every vector operation and evaluation runs on the device) and the Ewald
// ion-ion term.
//
// Minimisers (the direct minimisation at constant int n of Sec. II; the CG and
// truncated-Newton optimisers named in Sec. I): phi lives on the sphere
// dv sum phi^2 = N_e; the projected gradient is g = 2 dv phi (v - mu) with
// mu = int n v / N_e (Eq. E10); steps are rotations
// phi(theta) = cos(theta) phi + sin(theta) |phi| d/|d| along a tangent d.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "ofdft_internal.h"

using namespace ofdft;

namespace {

constexpr double kPiD = 3.141592653589793238462643383279502884;
constexpr double kKelvinToHartree = 3.1668115634556e-6;   // k_B / E_h (CODATA 2018)

thread_local std::string g_last_error;

int fail(ofdft_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  g_last_error = msg;
  return code;
}

bool grid_ok(int n) {
  static const int allowed[] = {8, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 128, 160, 192, 256, 320, 400};
  for (int a : allowed)
    if (a == n) return true;
  return false;
}

// Largest power of two that divides n and is at most cap (1 if cap < 2).
int largest_pow2_divisor_upto(int n, int cap) {
  int t = 1;
  while (2 * t <= cap) t *= 2;
  while (t > 1 && n % t) t >>= 1;
  return t;
}

double alpha_of(const ofdft_options& o, double Z, double V) {
  if (o.lpp == OFDFT_LPP_HA) return 2.0 * kPiD / V * (Z * o.lpp_rc * o.lpp_rc - 2.0 / 3.0 * o.lpp_A * std::pow(o.lpp_rc, 3));
  return kPiD * Z * o.lpp_rc * o.lpp_rc / V;
}

bool is_fin(double x) { return std::isfinite(x); }

// ---------------------------------------------------------------- evaluation helpers
struct Point {
  double F;     // F_tot
  double Ne;    // measured int n
};

int eval_at(ofdft_ctx* c, const double* phi, void* v, double* sc, Point& p) {
  double h[SC_COUNT];
  int rc = dev_eval(c, phi, v, sc, h);
  if (rc) return rc;
  p.F = h[SC_FTOT];
  p.Ne = h[SC_NE];
  if (!is_fin(p.F)) return fail(c, OFDFT_E_NONFINITE, "non-finite free energy");
  return OFDFT_OK;
}

// The report of the state in h (device scalars): E_ion, which the device sums
// leave out, is added here once the host Ewald thread has finished.
int fill_report(ofdft_ctx* c, const double* h, double resid, ofdft_report* rep, int iters, int evals, int conv) {
  if (!join_ewald(c)) return fail(c, OFDFT_E_ARG, "Ewald sum failed");
  ofdft_report r{};
  r.iterations = iters;
  r.evaluations = evals;
  r.converged = conv;
  r.F_total = h[SC_FTOT] + c->E_ion;
  r.F_s = h[SC_FS];
  r.TS_s = h[SC_TS];
  r.TS_xc = h[SC_TSXC];
  r.E_internal = r.F_total + h[SC_TS] + h[SC_TSXC];
  r.E_xc = h[SC_EXC];
  r.E_H = h[SC_EH];
  r.E_ext = h[SC_EEXT];
  r.E_alphaZ = h[SC_EAZ];
  r.E_ion = c->E_ion;
  r.N_e = h[SC_NE];
  r.mu = h[SC_MU];
  r.residual = resid;
  c->last = r;
  if (rep) *rep = r;
  return OFDFT_OK;
}

// Line search along the rotation phi(theta) = ca phi + sb d (ca, sb from theta).
// On success the accepted state is in phi_t / v_t / scalars_t.  Trials alternate
// between two buffers so that the best one so far is kept while the next is
// evaluated (no re-evaluation when an earlier trial wins).  pre, when given, holds
// the scalars of a first trial at theta1 already evaluated into phi_t / v_t /
// scalars_t.
struct LS {
  double theta;
  double F;
  bool ok;
  double dth;     // dF/dtheta at the accepted angle
  double bound;   // failed search: |dF0| times the smallest angle tried, all of which raised F
};

// Strong-Wolfe slope test |dF/dtheta| <= 0.1 |dF0|.  A looser test (0.3) accepted the
// first trial more often but left F about 1e-9 (relative) above the minimum in FP64,
// outside the energy tolerance, and in the mixed path it lengthened the CG iteration
// (more evaluations per converged ionic step, not fewer).
constexpr double kSlopeTest = 0.1;

int line_search(ofdft_ctx* c, double F0, double dF0, double r, double phinorm, double dn, double theta1,
                int& nevals, LS& out, const double* pre = nullptr) {
  const double ratio = r / phinorm;   // renormalises phi to the exact sphere
  double lo = 0.0, dlo = dF0, hi = -1.0, dhi = 0.0;
  double theta = theta1;
  double best_theta = -1.0, best_F = F0, best_dth = 0.0, min_theta = theta1;
  int cur = 0, best_buf = -1;
  double* tphi[2] = {c->phi_t, c->phi_t2};
  void* tv[2] = {c->v_t, c->v_t2};
  double* tsc[2] = {c->scalars_t, c->scalars_t2};
  // leave the chosen trial in phi_t / v_t / scalars_t
  auto select = [&](int b) {
    if (b == 1) {
      std::swap(c->phi_t, c->phi_t2);
      std::swap(c->v_t, c->v_t2);
      std::swap(c->scalars_t, c->scalars_t2);
    }
  };
  // In the mixed path F and dF/dtheta carry FP32 noise, so near convergence the
  // slope test can fail at random: after three trials a point with sufficient
  // decrease is taken, and the search gives up after eight.
  const bool mixed = c->rsize == 4;
  const int max_trials = mixed ? 8 : 14;
  bool best_armijo = false;
  for (int trial = 0; trial < max_trials; ++trial) {
    double h[SC_COUNT];
    if (trial == 0 && pre) {
      std::copy(pre, pre + SC_COUNT, h);
    } else {
      const double ct = std::cos(theta), st = std::sin(theta);
      // phi_t = rotation of phi toward d, its evaluation and dF/dtheta in one pass sequence
      int rc = dev_eval_trial(c, c->phi, c->d, ct * ratio, st * r / dn, tphi[cur], tv[cur], tsc[cur],
                              -st * ratio, ct * r / dn, h);
      if (rc) return rc;
      ++nevals;
    }
    const double dth = h[SC_DOT0];
    double Ft = h[SC_FTOT];
    min_theta = std::min(min_theta, theta);
    // OFDFT_TEST_NONFINITE: the host treats this trial's energy as non-finite (tests of
    // the recovery path; the device state is untouched)
    ++c->trials_seen;
    if (c->test_nonfinite != 0 && (c->test_nonfinite < 0 || c->trials_seen == c->test_nonfinite)) Ft = NAN;
    if (!is_fin(Ft) || !is_fin(dth)) return fail(c, OFDFT_E_NONFINITE, "non-finite energy in line search");
    const bool armijo = Ft <= F0 + 1e-4 * theta * dF0;
    // once F changes at its rounding level only the slope test can decide
    const bool flat = Ft <= F0 + 1e-14 * std::fabs(F0);
    if ((armijo || flat) && std::fabs(dth) <= kSlopeTest * std::fabs(dF0)) {
      select(cur);
      out = {theta, Ft, true, dth, 0.0};
      return OFDFT_OK;
    }
    if (Ft <= F0 && (best_theta < 0 || Ft < best_F)) {
      best_theta = theta;
      best_F = Ft;
      best_dth = dth;
      best_armijo = armijo;
      best_buf = cur;
      cur ^= 1;   // keep this trial; the next one goes to the other buffer
    }
    if (mixed && trial >= 2 && best_armijo) break;
    if (dth > 0.0 || !armijo) {
      hi = theta;
      dhi = dth;
    } else {
      lo = theta;
      dlo = dth;
    }
    double next;
    if (hi < 0.0) {
      next = (dth <= dF0) ? 2.0 * theta : theta - dth * theta / (dth - dF0);
      next = std::min(std::max(next, 1.5 * theta), 4.0 * theta);
    } else {
      next = (dth > 0.0 && dhi > dlo) ? lo - dlo * (hi - lo) / (dhi - dlo) : 0.5 * (lo + hi);
      const double w = hi - lo;
      next = std::min(std::max(next, lo + 0.1 * w), hi - 0.1 * w);
    }
    theta = next;
  }
  if (best_theta < 0.0) {
    // every trial raised F: if F is convex along the line, F(theta) >= F0 + dF0 theta, and
    // it rises beyond the smallest trial angle, so no point of the line lies lower than
    // F0 - |dF0| min_theta
    out = {0.0, F0, false, dF0, std::fabs(dF0) * min_theta};
    return OFDFT_OK;
  }
  select(best_buf);
  out = {best_theta, best_F, true, best_dth, 0.0};
  return OFDFT_OK;
}

void accept_trial(ofdft_ctx* c) {
  std::swap(c->phi, c->phi_t);
  std::swap(c->v, c->v_t);
  std::swap(c->scalars, c->scalars_t);
}

// Ionic-step history (options.extrapolate): remember the converged amplitude.
int save_history(ofdft_ctx* c) {
  const size_t bytes = (size_t)c->g.N * sizeof(double);
  const int slot = c->n_hist == 0 ? 0 : (c->hist_head + 1) % 3;
  if (!c->phi_hist[slot] && ctx_malloc(c, (void**)&c->phi_hist[slot], bytes) != hipSuccess)
    return fail(c, OFDFT_E_DEVICE, "history allocation");
  if (hipMemcpyAsync(c->phi_hist[slot], c->phi, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return fail(c, OFDFT_E_DEVICE, "history copy");
  c->hist_head = slot;
  c->n_hist = std::min(c->n_hist + 1, 3);
  return OFDFT_OK;
}

// Starting amplitude after the ions moved: polynomial extrapolation in the step
// index through the last converged amplitudes, renormalised to N_e.
int extrapolate_phi(ofdft_ctx* c) {
  const int order = std::min(c->opt.extrapolate, c->n_hist - 1);
  if (order < 1) return OFDFT_OK;
  const double* h0 = c->phi_hist[c->hist_head];
  const double* h1 = c->phi_hist[(c->hist_head + 2) % 3];
  const double* h2 = c->phi_hist[(c->hist_head + 1) % 3];
  int rc = order == 1 ? dev_combine3(c, c->phi, 2.0, h0, -1.0, h1, 0.0, nullptr)
                      : dev_combine3(c, c->phi, 3.0, h0, -3.0, h1, 1.0, h2);
  if (rc) return rc;
  double s2 = 0.0;
  if ((rc = dev_read(c, c->vout, 1, &s2))) return rc;
  if (!(s2 > 0.0) || !is_fin(s2)) return fail(c, OFDFT_E_NONFINITE, "extrapolated amplitude is zero or non-finite");
  return dev_axpby(c, c->phi, std::sqrt(c->Ne / (c->g.dv * s2)), c->phi, 0.0);
}

int ensure_phi(ofdft_ctx* c) {
  if (c->have_phi) return OFDFT_OK;
  std::vector<double> h(c->g.N, std::sqrt(c->Ne / c->g.volume));
  if (hipMemcpy(c->phi, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return fail(c, OFDFT_E_DEVICE, "upload phi");
  c->have_phi = true;
  return OFDFT_OK;
}

int check_ready(ofdft_ctx* c) {
  if (!c) return fail(nullptr, OFDFT_E_ARG, "null context");
  if (!c->have_cell) return fail(c, OFDFT_E_STATE, "set_cell has not been called");
  if (!c->have_ions) return fail(c, OFDFT_E_STATE, "set_ions has not been called (after the last set_cell)");
  if (!c->have_T) return fail(c, OFDFT_E_STATE, "set_temperature has not been called");
  if (hipSetDevice(c->opt.device) != hipSuccess) return fail(c, OFDFT_E_DEVICE, "hipSetDevice");
  return ensure_phi(c);
}

bool stop_rule(const ofdft_ctx* c, int small, double resid) {
  return small >= 2 && (c->opt.tol_residual <= 0.0 || resid < c->opt.tol_residual);
}

// When no trial point lowers F, the iteration sits at the resolution of F:
// converged if the residual target (when one is set) is met, otherwise if the
// last steps were already below the energy tolerance; in the mixed path (FP32
// terms summed in FP64) also once the last decrease is below 1e-6 |F| (its
// stated accuracy).  Before any step is taken (a start at a converged density)
// the failed search's bound on the decrease along the line, |dF/dtheta(0)| times
// the smallest angle tried, stands in for the last decrease.
bool stalled_converged(ofdft_ctx* c, int small, double last_dF, double F, double resid) {
  // F is the electronic part; the stated accuracy refers to the total, E_ion included
  const bool noise_floor = c->rsize == 4 && join_ewald(c) && std::fabs(last_dF) < 1e-6 * std::fabs(F + c->E_ion);
  if (c->opt.tol_residual > 0.0) return resid < c->opt.tol_residual || noise_floor;
  return small >= 1 || std::fabs(last_dF) < c->opt.tol_energy || noise_floor;
}

// First trial angle: the minimum of the quadratic with slope dF0 and the previous
// search's curvature kappa, else the angle that repeats the previous decrease
// (Fprev - F0), clamped to [1e-6, 0.3]; 0.05 without either.  k_dir_final applies
// the same rule on the device.
double first_step(double F0, double Fprev, bool have_prev, double dF0, double kappa = 0.0) {
  if (kappa > 0.0 && dF0 < 0.0) return std::min(std::max(-dF0 / kappa, 1e-6), 0.3);
  if (have_prev && dF0 < 0.0 && Fprev > F0) return std::min(std::max(2.0 * (Fprev - F0) / (-dF0), 1e-6), 0.3);
  return 0.05;
}

// ---------------------------------------------------------------- CG
// Polak-Ribiere+ on the sphere.  With cg_precond > 0 the gradient g is filtered
// by P(G) = 1/(1 + G^2/k0^2), k0^2 = cg_precond k_F^2, and the tangent part of
// z = P g replaces g in the direction update:
//   d = -(z - cz phi) + beta (d_old transported), cz = z.phi / phi.phi,
//   beta = max(0, (z.g - zt.g_old) / (z_old.g_old)),  zt = z - cz phi
// (g is tangent at phi, so zt.g = z.g).
int minimize_cg(ofdft_ctx* c, ofdft_report* rep) {
  const double norm2 = c->Ne / c->g.dv;   // target sum phi^2
  const double r = std::sqrt(norm2);
  // the filter targets the stiff high-G modes of the gradient term; ftTF has none
  const bool pcg = c->opt.cg_precond > 0.0 && c->opt.functional != OFDFT_TF;
  if (pcg) c->g.prec_k2 = c->opt.cg_precond * std::pow(3.0 * kPiD * kPiD * c->Ne / c->g.volume, 2.0 / 3.0);
  int nevals = 0, rc;
  Point p;
  if ((rc = eval_at(c, c->phi, c->v, c->scalars, p))) return rc;
  ++nevals;
  double F = p.F, Fprev = 0.0, gg_prev = 0.0, dn_prev = 0.0, theta_prev = 0.0, last_dF = 1e300, kappa = 0.0;
  bool have_prev = false;
  int small = 0, it = 0;
  bool converged = false;
  double resid = 0.0;
  // recovery (each at most once per minimisation): a non-finite trial restarts the CG from
  // the steepest-descent direction at the last finite point; a line search that finds no
  // lower F before the stopping rule holds restarts along -g (-z when preconditioned)
  bool nonfinite_restart_used = false, ls_restart_used = false;
  int final_rc = OFDFT_OK;
  for (it = 1; it <= c->opt.max_iter; ++it) {
    // gradient dots, beta, the new direction and the first trial angle on the device;
    // that trial is evaluated before anything is read back, so one readback serves both
    const double cproj = have_prev ? std::sin(theta_prev) * dn_prev / r : 0.0;
    if ((rc = dev_cg_step(c, pcg, have_prev, gg_prev, cproj, Fprev, r, kappa))) return rc;
    double both[2 * SC_COUNT];
    if ((rc = dev_eval_trial_dev(c, c->phi, c->d, c->scalars + SC_CA, c->phi_t, c->v_t, c->scalars_t, c->scalars,
                                 both)))
      return rc;
    ++nevals;
    const double* trial0 = both;
    const double* hs = both + SC_COUNT;
    const double* dots = hs + SC_DOT0;
    p.F = hs[SC_FTOT];
    p.Ne = hs[SC_NE];
    const double phinorm2 = p.Ne / c->g.dv;
    resid = std::sqrt(dots[3] / phinorm2);
    const double gg = dots[0];   // g.g, or z.g when preconditioned
    if (gg <= 0.0 || stop_rule(c, small, resid)) { converged = true; break; }
    double dd_dg[2] = {hs[SC_DD], hs[SC_DG]};
    bool have_trial0 = true;
    if (dd_dg[1] >= 0.0) {   // not a descent direction: restart along -g (or -z); the trial is void
      if ((rc = dev_cg_restart(c, pcg))) return rc;
      if ((rc = dev_read(c, c->scalars + SC_DD, 2, dd_dg))) return rc;
      have_trial0 = false;
    }
    const double dn = std::sqrt(dd_dg[0]);
    const double dF0 = r * dd_dg[1] / dn;
    LS ls;
    const double theta1 = have_trial0 ? hs[SC_TH1] : first_step(F, Fprev, have_prev, dF0, kappa);
    rc = line_search(c, F, dF0, r, std::sqrt(phinorm2), dn, theta1, nevals, ls, have_trial0 ? trial0 : nullptr);
    if (rc == OFDFT_E_NONFINITE && !nonfinite_restart_used) {
      // phi, v and the scalars of the current point are untouched (trials live in their own buffers)
      nonfinite_restart_used = true;
      have_prev = false;
      kappa = 0.0;
      small = 0;
      continue;
    }
    if (rc == OFDFT_E_NONFINITE) {
      final_rc = rc;
      break;
    }
    if (rc) return rc;
    if (!ls.ok) {
      converged = stalled_converged(c, small, have_prev ? last_dF : ls.bound, F, resid);
      if (!converged && have_prev && !ls_restart_used) {
        ls_restart_used = true;
        have_prev = false;
        kappa = 0.0;
        continue;
      }
      break;
    }
    accept_trial(c);
    const double dF = F - ls.F;
    last_dF = dF;
    Fprev = F;
    F = ls.F;
    gg_prev = gg;
    dn_prev = dn;
    theta_prev = ls.theta;
    have_prev = true;
    // curvature along d from the slopes at 0 and at the accepted angle
    kappa = (ls.theta > 0.0 && ls.dth > dF0) ? (ls.dth - dF0) / ls.theta : 0.0;
    small = std::fabs(dF) < c->opt.tol_energy ? small + 1 : 0;
    if (small >= 2 && c->opt.tol_residual <= 0.0) { converged = true; break; }
    // with a residual target the next gradient pass measures it
  }
  double h[SC_COUNT];
  if ((rc = dev_read(c, c->scalars, SC_COUNT, h))) return rc;
  if ((rc = fill_report(c, h, resid, rep, std::min(it, c->opt.max_iter), nevals, converged ? 1 : 0))) return rc;
  c->converged = converged;
  if (final_rc == OFDFT_E_NONFINITE)
    return fail(c, OFDFT_E_NONFINITE, "non-finite energy in line search after a steepest-descent restart "
                                      "(the last finite state is kept)");
  return converged ? OFDFT_OK : fail(c, OFDFT_E_NOT_CONVERGED, "minimisation did not converge");
}

// ---------------------------------------------------------------- HIP-graph CG
// The device-resident iteration of dev_cg_graph_*: the host only replays the captured
// graph, keeping up to kGraphDepth iterations queued, and reads the status word that
// each iteration's control kernel publishes into mapped host memory.
constexpr int kGraphDepth = 2;

struct GraphRun {
  ofdft_ctx* c;
  int launched = 0;        // graph replays queued
  double seen = 0.0;       // replays whose status the host has read
  bool done = false;
  int rc = OFDFT_OK;
};

double status_word(const ofdft_ctx* c, int k) {
  double v;
  __atomic_load(&c->hmap[kMapStatus + k], &v, __ATOMIC_ACQUIRE);
  return v;
}

// Queue the starting evaluation, the state initialisation and the first replays.
int graph_begin(GraphRun& g) {
  ofdft_ctx* c = g.c;
  const double r = std::sqrt(c->Ne / c->g.dv);
  const bool pcg = c->opt.cg_precond > 0.0 && c->opt.functional != OFDFT_TF;
  if (pcg) c->g.prec_k2 = c->opt.cg_precond * std::pow(3.0 * kPiD * kPiD * c->Ne / c->g.volume, 2.0 / 3.0);
  const CgConst k{r, c->g.dv, c->opt.tol_energy, c->opt.tol_residual, c->opt.max_iter, pcg ? 1 : 0,
                  c->rsize == 4 ? 1 : 0, c->test_nonfinite};
  int rc;
  if ((rc = dev_cg_graph_prepare(c, pcg, k))) return rc;
  c->hmap[kMapStatus] = 0.0;      // the device counts replays from zero again
  if ((rc = dev_eval(c, c->phi, c->v, c->scalars))) return rc;
  if ((rc = dev_cg_graph_start(c))) return rc;
  for (; g.launched < kGraphDepth; ++g.launched)
    if ((rc = dev_cg_graph_launch(c))) return rc;
  return OFDFT_OK;
}

// Non-blocking progress: read the status word, queue replays; done once the device
// reports the minimisation stopped.  wait = true spins until there is progress.
int graph_step(GraphRun& g, bool wait) {
  ofdft_ctx* c = g.c;
  for (unsigned spin = 1;; ++spin) {
    const double n = status_word(c, 0);
    if (n > g.seen) {
      g.seen = n;
      if (status_word(c, 1) == 0.0) {
        g.done = true;
        return OFDFT_OK;
      }
      int rc;
      for (; g.launched < (int)g.seen + kGraphDepth; ++g.launched)
        if ((rc = dev_cg_graph_launch(c))) return rc;
      return OFDFT_OK;
    }
    if (!wait) return OFDFT_OK;
    if (spin > 4096) std::this_thread::yield();
    if ((spin & 255u) == 0) {
      const hipError_t e = hipStreamQuery(c->stream);
      if (e == hipSuccess) {
        if (status_word(c, 0) > g.seen) continue;
        return fail(c, OFDFT_E_DEVICE, "graph CG: the stream drained without a status update");
      }
      if (e != hipErrorNotReady) return fail(c, OFDFT_E_DEVICE, std::string("graph CG: ") + hipGetErrorString(e));
    }
    __builtin_ia32_pause();
  }
}

// The final state: report and return code from the device CG state.
int graph_finish(GraphRun& g, ofdft_report* rep) {
  ofdft_ctx* c = g.c;
  double st[CG_COUNT], h[SC_COUNT];
  int rc;
  if ((rc = dev_read(c, c->cgst, CG_COUNT, st))) return rc;
  if ((rc = dev_read(c, c->scalars, SC_COUNT, h))) return rc;
  const bool converged = st[CG_CONVERGED] != 0.0;
  if ((rc = fill_report(c, h, st[CG_RESID], rep, (int)st[CG_ITERS], (int)st[CG_EVALS], converged ? 1 : 0)))
    return rc;
  c->converged = converged;
  if (st[CG_STATUS] == CGS_NONFINITE)
    return fail(c, OFDFT_E_NONFINITE, "non-finite energy: the last finite state is kept");
  if (converged) return OFDFT_OK;
  char msg[160];
  std::snprintf(msg, sizeof(msg), "minimisation did not converge (graph CG: %s after %d iterations, residual %.3e)",
                st[CG_STATUS] == CGS_MAXITER ? "max_iter reached" : "no lower F found", (int)st[CG_ITERS],
                st[CG_RESID]);
  return fail(c, OFDFT_E_NOT_CONVERGED, msg);
}

int minimize_cg_graph(ofdft_ctx* c, ofdft_report* rep) {
  GraphRun g;
  g.c = c;
  int rc = graph_begin(g);
  while (!rc && !g.done) rc = graph_step(g, true);
  if (rc) {
    (void)dev_sync(c);
    return rc;
  }
  return graph_finish(g, rep);
}

// ---------------------------------------------------------------- truncated Newton
int minimize_tn(ofdft_ctx* c, ofdft_report* rep) {
  const double norm2 = c->Ne / c->g.dv;
  const double r = std::sqrt(norm2);
  const double two_dv = 2.0 * c->g.dv;
  double* P = c->tn[0];
  double* RES = c->tn[1];
  double* S = c->tn[2];
  double* HS = c->tn[3];
  int nevals = 0, rc;
  Point p;
  if ((rc = eval_at(c, c->phi, c->v, c->scalars, p))) return rc;
  ++nevals;
  double F = p.F, last_dF = 1e300;
  int small = 0, it = 0;
  bool converged = false;
  double resid = 0.0;
  const int max_inner = 20;
  // finite-difference step of the Hessian products: ~sqrt of the gradient's relative precision
  const double fd_rel = (c->rsize == 4) ? 3e-4 : 1e-6;
  for (it = 1; it <= c->opt.max_iter; ++it) {
    double hsc[SC_COUNT];
    if ((rc = dev_grad_dots(c, c->phi, c->v, c->scalars, nullptr, nullptr, c->scalars + SC_DOT0))) return rc;
    if ((rc = dev_read(c, c->scalars, SC_COUNT, hsc))) return rc;
    const double* dots = hsc + SC_DOT0;
    p.F = hsc[SC_FTOT];
    p.Ne = hsc[SC_NE];
    const double phinorm2 = p.Ne / c->g.dv;
    resid = std::sqrt(dots[3] / phinorm2);
    const double gnorm = std::sqrt(dots[0]);
    if (gnorm == 0.0 || stop_rule(c, small, resid)) { converged = true; break; }
    const double mu = hsc[SC_MU];
    // d = -g, gprev = g
    if ((rc = dev_cg_direction(c, 0.0, 0.0))) return rc;
    // inner CG on H p = -g: P = 0, RES = -g, S = RES
    if ((rc = dev_axpby(c, P, 0.0, c->d, 0.0))) return rc;
    if ((rc = dev_axpby(c, RES, 0.0, c->d, 1.0))) return rc;
    if ((rc = dev_axpby(c, S, 0.0, c->d, 1.0))) return rc;
    double rr = dots[0];
    const double tol_in = std::min(0.5, std::sqrt(gnorm)) * gnorm;
    bool any = false;
    for (int k = 0; k < max_inner; ++k) {
      double ss;
      if ((rc = dev_dot(c, S, S))) return rc;
      if ((rc = dev_read(c, c->vout, 1, &ss))) return rc;
      const double eps = fd_rel * r / std::sqrt(ss);
      // central difference of the unconstrained gradient along S
      if ((rc = dev_rotate(c, c->phi_t, c->phi, 1.0, S, eps))) return rc;
      if ((rc = dev_eval(c, c->phi_t, c->v_t, c->scalars_t))) return rc;
      if ((rc = dev_full_grad_acc(c, HS, c->phi_t, c->v_t, +1.0))) return rc;
      if ((rc = dev_rotate(c, c->phi_t, c->phi, 1.0, S, -eps))) return rc;
      if ((rc = dev_eval(c, c->phi_t, c->v_t, c->scalars_t))) return rc;
      if ((rc = dev_full_grad_acc(c, HS, c->phi_t, c->v_t, -1.0))) return rc;
      nevals += 2;
      // HS = P[(g+ - g-)/(2 eps)] - 2 dv mu S
      if ((rc = dev_tn_hess_finish(c, HS, c->phi, S, 0.5 / eps, 0.0))) return rc;
      double hphi;
      if ((rc = dev_read(c, c->vout, 1, &hphi))) return rc;
      if ((rc = dev_axpby(c, HS, 1.0, c->phi, -hphi / phinorm2))) return rc;
      if ((rc = dev_axpby(c, HS, 1.0, S, -two_dv * mu))) return rc;
      double curv;
      if ((rc = dev_dot(c, S, HS))) return rc;
      if ((rc = dev_read(c, c->vout, 1, &curv))) return rc;
      if (!is_fin(curv)) return fail(c, OFDFT_E_NONFINITE, "non-finite curvature");
      if (curv <= 0.0) break;
      const double alpha = rr / curv;
      if ((rc = dev_axpby(c, P, 1.0, S, alpha))) return rc;
      any = true;
      if ((rc = dev_axpby(c, RES, 1.0, HS, -alpha))) return rc;
      double rr_new;
      if ((rc = dev_dot(c, RES, RES))) return rc;
      if ((rc = dev_read(c, c->vout, 1, &rr_new))) return rc;
      if (std::sqrt(rr_new) < tol_in) break;
      if ((rc = dev_axpby(c, S, rr_new / rr, RES, 1.0))) return rc;
      rr = rr_new;
    }
    // search direction d = P projected onto the tangent space (or -g)
    if (any) {
      double pphi;
      if ((rc = dev_dot(c, P, c->phi))) return rc;
      if ((rc = dev_read(c, c->vout, 1, &pphi))) return rc;
      if ((rc = dev_axpby(c, c->d, 0.0, P, 1.0))) return rc;
      if ((rc = dev_axpby(c, c->d, 1.0, c->phi, -pphi / phinorm2))) return rc;
    }
    double dd, dg;
    if ((rc = dev_dot(c, c->d, c->d))) return rc;
    if ((rc = dev_read(c, c->vout, 1, &dd))) return rc;
    if ((rc = dev_dot(c, c->d, c->gprev))) return rc;
    if ((rc = dev_read(c, c->vout, 1, &dg))) return rc;
    if (dg >= 0.0) {
      if ((rc = dev_cg_direction(c, 0.0, 0.0))) return rc;
      double t2[2];
      if ((rc = dev_read(c, c->vout, 2, t2))) return rc;
      dd = t2[0];
      dg = t2[1];
    }
    const double dn = std::sqrt(dd);
    const double dF0 = r * dg / dn;
    const double theta1 = std::min(std::max(dn / r, 1e-8), 0.5);
    LS ls;
    if ((rc = line_search(c, F, dF0, r, std::sqrt(phinorm2), dn, theta1, nevals, ls))) return rc;
    if (!ls.ok) {
      converged = stalled_converged(c, small, last_dF < 1e300 ? last_dF : ls.bound, F, resid);
      break;
    }
    accept_trial(c);
    const double dF = F - ls.F;
    last_dF = dF;
    F = ls.F;
    small = std::fabs(dF) < c->opt.tol_energy ? small + 1 : 0;
    if (small >= 2 && c->opt.tol_residual <= 0.0) { converged = true; break; }
  }
  double h[SC_COUNT];
  if ((rc = dev_read(c, c->scalars, SC_COUNT, h))) return rc;
  if ((rc = fill_report(c, h, resid, rep, std::min(it, c->opt.max_iter), nevals, converged ? 1 : 0))) return rc;
  c->converged = converged;
  return converged ? OFDFT_OK : fail(c, OFDFT_E_NOT_CONVERGED, "minimisation did not converge");
}

}  // namespace

namespace ofdft {

hipError_t ctx_malloc(ofdft_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 1;
  if (c->opt.alloc) {
    *p = c->opt.alloc(bytes, c->opt.alloc_ctx);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

void ctx_free(ofdft_ctx* c, void* p) {
  if (!p) return;
  if (c->opt.alloc) c->opt.free_(p, c->opt.alloc_ctx);
  else (void)hipFree(p);
}

}  // namespace ofdft

// ==================================================================== C ABI
extern "C" {

void ofdft_default_options(ofdft_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->functional = OFDFT_TF;
  o->mu_sga = 5.0 / 27.0;
  o->xc = OFDFT_XC_PZ81;
  o->lpp = OFDFT_LPP_GAUSS;
  o->lpp_rc = 0.5;
  o->lpp_A = 0.0;
  o->lpp_qc = 1e30;
  o->precision = OFDFT_FP64;
  o->minimizer = OFDFT_CG;
  o->tol_energy = 1e-8;
  o->tol_residual = 0.0;
  o->max_iter = 1000;
  o->device = 0;
  o->stream = nullptr;
  o->cg_precond = 8.0;
  o->extrapolate = 0;
}

int ofdft_create(const ofdft_options* opt, ofdft_ctx** out) {
  if (!out) return fail(nullptr, OFDFT_E_ARG, "out is NULL");
  *out = nullptr;
  ofdft_options o;
  if (opt) o = *opt;
  else ofdft_default_options(&o);
  if (o.functional < OFDFT_TF || o.functional > OFDFT_APBEF) return fail(nullptr, OFDFT_E_ARG, "unknown functional");
  if (o.xc != OFDFT_XC_NONE && o.xc != OFDFT_XC_PZ81 && o.xc != OFDFT_XC_KSDT)
    return fail(nullptr, OFDFT_E_ARG, "unknown xc");
  if (o.lpp != OFDFT_LPP_GAUSS && o.lpp != OFDFT_LPP_HA) return fail(nullptr, OFDFT_E_ARG, "unknown pseudopotential");
  if (!(o.lpp_rc > 0.0)) return fail(nullptr, OFDFT_E_ARG, "lpp_rc must be > 0");
  if (o.lpp == OFDFT_LPP_HA && !(o.lpp_qc > 0.0)) return fail(nullptr, OFDFT_E_ARG, "lpp_qc must be > 0");
  if (o.precision != OFDFT_FP64 && o.precision != OFDFT_MIXED) return fail(nullptr, OFDFT_E_ARG, "unknown precision");
  if (o.minimizer != OFDFT_CG && o.minimizer != OFDFT_TN) return fail(nullptr, OFDFT_E_ARG, "unknown minimizer");
  if (!(o.tol_energy > 0.0) || o.tol_residual < 0.0 || o.max_iter < 1)
    return fail(nullptr, OFDFT_E_ARG, "tolerances must be positive and max_iter >= 1");
  if (o.functional == OFDFT_SGA && !(o.mu_sga >= 0.0)) return fail(nullptr, OFDFT_E_ARG, "mu_sga must be >= 0");
  if (!(o.cg_precond >= 0.0) || !std::isfinite(o.cg_precond))
    return fail(nullptr, OFDFT_E_ARG, "cg_precond must be finite and >= 0");
  if (o.extrapolate < 0 || o.extrapolate > 2) return fail(nullptr, OFDFT_E_ARG, "extrapolate must be 0, 1 or 2");
  if ((o.alloc == nullptr) != (o.free_ == nullptr))
    return fail(nullptr, OFDFT_E_ARG, "alloc and free_ must be set together");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(nullptr, OFDFT_E_DEVICE, "no HIP device");
  if (o.device < 0 || o.device >= ndev) return fail(nullptr, OFDFT_E_ARG, "device ordinal out of range");
  if (hipSetDevice(o.device) != hipSuccess) return fail(nullptr, OFDFT_E_DEVICE, "hipSetDevice failed");
  if (dev_upload_tables(o.device) != OFDFT_OK) return fail(nullptr, OFDFT_E_DEVICE, "uploading the t-factor tables failed");
  ofdft_ctx* c = new ofdft_ctx();
  c->opt = o;
  c->rsize = (o.precision == OFDFT_MIXED) ? 4 : 8;
  if (const char* pp = std::getenv("OFDFT_PLANE_PASSES")) c->plane_passes = std::atoi(pp) != 0;
  if (const char* pg = std::getenv("OFDFT_FUSED_GGA")) c->fused_gga = std::atoi(pg) != 0;
  if (const char* pf = std::getenv("OFDFT_ION_FORCES")) c->ion_forces = std::atoi(pf) != 0 ? 1 : 0;
  if (const char* pn = std::getenv("OFDFT_TEST_NONFINITE")) c->test_nonfinite = std::atoi(pn);
  if (o.stream) {
    c->stream = (hipStream_t)o.stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(nullptr, OFDFT_E_DEVICE, "stream creation failed");
    }
    c->own_stream = true;
  }
  *out = c;
  return OFDFT_OK;
}

int ofdft_destroy(ofdft_ctx* c) {
  if (!c) return fail(nullptr, OFDFT_E_ARG, "null context");
  join_ewald(c);
  (void)hipSetDevice(c->opt.device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  dev_free_grid(c);
  ctx_free(c, c->phase);
  ctx_free(c, c->dZ);
  ctx_free(c, c->fpart);
  ctx_free(c, c->dforces);
  if (c->hmap) (void)hipHostFree(c->hmap);
  for (hipEvent_t e : c->timing.events) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return OFDFT_OK;
}

int ofdft_set_cell(ofdft_ctx* c, const double lattice[9], double cell_scale, const int grid[3]) {
  if (!c) return fail(nullptr, OFDFT_E_ARG, "null context");
  if (!lattice || !grid) return fail(c, OFDFT_E_ARG, "lattice and grid must not be NULL");
  if (!(cell_scale > 0.0) || !is_fin(cell_scale)) return fail(c, OFDFT_E_ARG, "cell_scale must be > 0");
  for (int k = 0; k < 9; ++k)
    if (!is_fin(lattice[k])) return fail(c, OFDFT_E_ARG, "non-finite lattice");
  for (int k = 0; k < 3; ++k)
    if (!grid_ok(grid[k])) return fail(c, OFDFT_E_GRID,
                                         "grid sizes must be one of 8,12,16,20,24,32,40,48,64,80,96,128,160,192,"
                                         "256,320,400");
  double lat[9];
  for (int k = 0; k < 9; ++k) lat[k] = lattice[k] * cell_scale;
  const double* a1 = lat;
  const double* a2 = lat + 3;
  const double* a3 = lat + 6;
  const double det = a1[0] * (a2[1] * a3[2] - a2[2] * a3[1]) - a1[1] * (a2[0] * a3[2] - a2[2] * a3[0]) +
                     a1[2] * (a2[0] * a3[1] - a2[1] * a3[0]);
  const double scale = std::pow(std::fabs(a1[0]) + std::fabs(a2[1]) + std::fabs(a3[2]) + 1e-300, 3.0);
  if (!(std::fabs(det) > 1e-10 * scale)) return fail(c, OFDFT_E_ARG, "singular lattice");
  if (hipSetDevice(c->opt.device) != hipSuccess) return fail(c, OFDFT_E_DEVICE, "hipSetDevice");
  GridDesc g{};
  g.n1 = grid[0];
  g.n2 = grid[1];
  g.n3 = grid[2];
  g.n3h = g.n3 / 2 + 1;
  g.n3k = g.n3 / 2;   // grids are even: the k3 = n3/2 plane holds Nyquist modes only
  g.N = (long long)g.n1 * g.n2 * g.n3;
  g.NS = (long long)g.n3h * g.n1 * g.n2;
  // b_i = 2 pi (a_j x a_k)/det
  auto cross = [](const double* u, const double* v, double* w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
  };
  cross(a2, a3, g.b);
  cross(a3, a1, g.b + 3);
  cross(a1, a2, g.b + 6);
  for (int k = 0; k < 9; ++k) g.b[k] *= 2.0 * kPiD / det;
  g.volume = std::fabs(det);
  g.dv = g.volume / (double)g.N;
  g.inv_n = 1.0 / (double)g.N;
  // default tiles: at most 16 rows or columns, within the register-staged tile size
  g.tr = std::max(2, largest_pow2_divisor_upto(g.n2, std::min(g.n3 >= 256 ? 8 : 16, kStageElems / g.n3)));
  const int tc_cap = std::min((g.n1 >= 256) ? 8 : 16, kStageElems / g.n1);
  g.tc = largest_pow2_divisor_upto(g.n2, tc_cap);
  g.rb = 1;
  while (2 * g.rb * g.n2 <= 1024) g.rb *= 2;   // largest power of two with rb * n2 <= 1024
  join_ewald(c);
  std::memcpy(c->lat, lat, sizeof(lat));
  c->cell_scale = cell_scale;
  c->g = g;
  c->have_cell = false;
  c->have_ions = false;
  c->have_phi = false;
  c->converged = false;
  int rc = dev_alloc_grid(c);
  if (rc) return fail(c, rc, c->err.empty() ? "device allocation failed" : c->err);
  c->have_cell = true;
  return OFDFT_OK;
}

int ofdft_set_ions(ofdft_ctx* c, int nat, const double* tau, const double* Z) {
  if (!c) return fail(nullptr, OFDFT_E_ARG, "null context");
  if (!c->have_cell) return fail(c, OFDFT_E_STATE, "set_cell must come first");
  if (nat <= 0 || !tau || !Z) return fail(c, OFDFT_E_ARG, "nat must be >= 1 and tau, Z non-NULL");
  for (int i = 0; i < nat; ++i) {
    if (!(Z[i] > 0.0) || !is_fin(Z[i])) return fail(c, OFDFT_E_ARG, "charges must be finite and > 0");
    for (int a = 0; a < 3; ++a)
      if (!is_fin(tau[3 * i + a])) return fail(c, OFDFT_E_ARG, "non-finite ion position");
  }
  if (hipSetDevice(c->opt.device) != hipSuccess) return fail(c, OFDFT_E_DEVICE, "hipSetDevice");
  join_ewald(c);
  // the ion state is rebuilt below; until the structure factor and E_rec exist for
  // the new ions the context has no valid ions (a failure leaves it that way)
  c->have_ions = false;
  c->converged = false;
  // positions are given in the frame of the unscaled lattice (cellScale, Sec. V B)
  const double Ne_old = c->Ne;
  c->nat = nat;
  c->tau.assign(tau, tau + 3 * (size_t)nat);
  for (double& x : c->tau) x *= c->cell_scale;
  c->Z.assign(Z, Z + nat);
  double Ne = 0.0, asum = 0.0;
  for (int i = 0; i < nat; ++i) {
    Ne += Z[i];
    asum += alpha_of(c->opt, Z[i], c->g.volume);
  }
  c->Ne = Ne;
  c->alpha_sum = asum;
  start_ewald(c);
  int rc = dev_structure_factor(c);
  if (rc) return fail(c, rc, c->err.empty() ? "structure factor failed" : c->err);
  if (c->have_phi && Ne_old > 0.0 && Ne_old != Ne) {
    // keep the shape of the warm start, rescale to the new electron count
    if ((rc = dev_axpby(c, c->phi, std::sqrt(Ne / Ne_old), c->phi, 0.0))) return fail(c, rc, c->err);
    c->n_hist = 0;
  } else if (c->have_phi && c->opt.extrapolate > 0) {
    if ((rc = extrapolate_phi(c))) return fail(c, rc, c->err);
  }
  c->have_ions = true;
  c->converged = false;
  return OFDFT_OK;
}

int ofdft_set_temperature(ofdft_ctx* c, double T_kelvin) {
  if (!c) return fail(nullptr, OFDFT_E_ARG, "null context");
  if (!(T_kelvin > 0.0) || !is_fin(T_kelvin)) return fail(c, OFDFT_E_ARG, "temperature must be finite and > 0");
  c->T_ha = T_kelvin * kKelvinToHartree;
  c->have_T = true;
  c->converged = false;
  return OFDFT_OK;
}

int ofdft_minimize_density(ofdft_ctx* c, ofdft_report* rep) {
  int rc = check_ready(c);
  if (rc) return rc;
  c->converged = false;
  rc = c->opt.minimizer == OFDFT_TN ? minimize_tn(c, rep)
       : c->opt.graph_cg          ? minimize_cg_graph(c, rep)
                                  : minimize_cg(c, rep);
  if (rc == OFDFT_OK && c->opt.extrapolate > 0 && (rc = save_history(c))) return rc;
  return rc;
}

int ofdft_stress(ofdft_ctx* c, double sigma[9]) {
  if (!c) return fail(nullptr, OFDFT_E_ARG, "null context");
  if (!sigma) return fail(c, OFDFT_E_ARG, "sigma is NULL");
  if (!c->converged) return fail(c, OFDFT_E_STATE, "no converged density: call ofdft_minimize_density first");
  if (hipSetDevice(c->opt.device) != hipSuccess) return fail(c, OFDFT_E_DEVICE, "hipSetDevice");
  double s[20];
  int rc = dev_stress(c, s);
  if (rc) return fail(c, rc, c->err);
  if (!join_ewald(c)) return fail(c, OFDFT_E_ARG, "Ewald sum failed");
  const double* ew = c->ewald_strain;   // from the set_ions thread
  const double V = c->g.volume;
  const ofdft_report& r = c->last;
  // V Sigma per term: local delta (sum(f - n df/dn) + sum n (eps - v_xc) - tr B) - B,
  // Hartree V H - delta E_H, pseudopotential -X - delta E_ext, alpha -delta E_alphaZ, Ewald
  const double trB = s[2] + s[3] + s[4];
  double t[6];
  for (int k = 0; k < 6; ++k) t[k] = -s[2 + k] + V * s[8 + k] - s[14 + k] + ew[k];
  // the device reciprocal sums carry the Ewald G-space strain terms; -delta E_rec here
  for (int k = 0; k < 3; ++k) t[k] += s[0] + s[1] - trB - r.E_H - r.E_ext - r.E_alphaZ - c->E_rec;
  const int ia[6] = {0, 1, 2, 0, 1, 0}, ib[6] = {0, 1, 2, 1, 2, 2};
  for (int k = 0; k < 6; ++k) {
    sigma[3 * ia[k] + ib[k]] = t[k] / V;
    sigma[3 * ib[k] + ia[k]] = t[k] / V;
  }
  for (int k = 0; k < 9; ++k)
    if (!is_fin(sigma[k])) return fail(c, OFDFT_E_NONFINITE, "non-finite stress");
  return OFDFT_OK;
}

int ofdft_free_energy_and_forces(ofdft_ctx* c, double* F_total, double* E_internal, double* forces,
                                 double* pressure) {
  if (!c) return fail(nullptr, OFDFT_E_ARG, "null context");
  if (!c->converged) return fail(c, OFDFT_E_STATE, "no converged density: call ofdft_minimize_density first");
  if (pressure) {
    double sig[9];
    int rc = ofdft_stress(c, sig);
    if (rc) return rc;
    *pressure = -(sig[0] + sig[4] + sig[8]) / 3.0;
  }
  if (hipSetDevice(c->opt.device) != hipSuccess) return fail(c, OFDFT_E_DEVICE, "hipSetDevice");
  if (F_total) *F_total = c->last.F_total;
  if (E_internal) *E_internal = c->last.E_internal;
  if (forces) {
    int rc = dev_forces(c, forces);
    if (rc) return fail(c, rc, c->err);
    if (!join_ewald(c)) return fail(c, OFDFT_E_ARG, "Ewald sum failed");
    for (int k = 0; k < 3 * c->nat; ++k) {
      forces[k] += c->F_ion[k];
      if (!is_fin(forces[k])) return fail(c, OFDFT_E_NONFINITE, "non-finite force");
    }
  }
  return OFDFT_OK;
}

int ofdft_get_density(ofdft_ctx* c, double* phi_out) {
  if (!c) return fail(nullptr, OFDFT_E_ARG, "null context");
  if (!phi_out) return fail(c, OFDFT_E_ARG, "phi_out is NULL");
  if (!c->have_cell) return fail(c, OFDFT_E_STATE, "set_cell has not been called");
  if (!c->have_phi) return fail(c, OFDFT_E_STATE, "no density yet");
  (void)hipSetDevice(c->opt.device);
  if (hipMemcpyAsync(phi_out, c->phi, c->g.N * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return fail(c, OFDFT_E_DEVICE, "copy phi");
  return OFDFT_OK;
}

int ofdft_set_density(ofdft_ctx* c, const double* phi) {
  if (!c) return fail(nullptr, OFDFT_E_ARG, "null context");
  if (!phi) return fail(c, OFDFT_E_ARG, "phi is NULL");
  if (!c->have_cell) return fail(c, OFDFT_E_STATE, "set_cell has not been called");
  if (!c->have_ions) return fail(c, OFDFT_E_STATE, "set_ions has not been called");
  double s = 0.0;
  for (long long i = 0; i < c->g.N; ++i) {
    if (!is_fin(phi[i])) return fail(c, OFDFT_E_ARG, "non-finite phi");
    s += phi[i] * phi[i];
  }
  if (!(s > 0.0)) return fail(c, OFDFT_E_ARG, "phi is zero");
  const double k = std::sqrt(c->Ne / (c->g.dv * s));
  std::vector<double> h(phi, phi + c->g.N);
  for (double& x : h) x *= k;
  (void)hipSetDevice(c->opt.device);
  if (hipMemcpy(c->phi, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return fail(c, OFDFT_E_DEVICE, "upload phi");
  c->n_hist = 0;
  c->have_phi = true;
  c->converged = false;
  return OFDFT_OK;
}

int ofdft_eval(ofdft_ctx* c, ofdft_report* rep, double* potential_out) {
  int rc = check_ready(c);
  if (rc) return rc;
  Point p;
  if ((rc = eval_at(c, c->phi, c->v, c->scalars, p))) return rc;
  double h[SC_COUNT];
  if ((rc = dev_grad_dots(c, c->phi, c->v, c->scalars, nullptr, nullptr, c->scalars + SC_DOT0))) return rc;
  if ((rc = dev_read(c, c->scalars, SC_COUNT, h))) return rc;
  if ((rc = fill_report(c, h, std::sqrt(h[SC_DOT0 + 3] / (p.Ne / c->g.dv)), rep, 0, 1, 0))) return rc;
  if (potential_out) {
    if (c->rsize == 8) {
      if (hipMemcpy(potential_out, c->v, c->g.N * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, OFDFT_E_DEVICE, "copy potential");
    } else {
      std::vector<float> tmp(c->g.N);
      if (hipMemcpy(tmp.data(), c->v, c->g.N * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, OFDFT_E_DEVICE, "copy potential");
      for (long long i = 0; i < c->g.N; ++i) potential_out[i] = tmp[i];
    }
  }
  return OFDFT_OK;
}

int ofdft_eval_noalloc(ofdft_ctx* c, const double* phi_dev, double* v_dev, ofdft_report* rep) {
  if (!c) return fail(nullptr, OFDFT_E_ARG, "null context");
  if (!phi_dev || !v_dev) return fail(c, OFDFT_E_ARG, "phi_dev and v_dev must not be NULL");
  if (!c->have_cell || !c->have_ions || !c->have_T)
    return fail(c, OFDFT_E_STATE, "set_cell, set_ions and set_temperature must come first");
  if (hipSetDevice(c->opt.device) != hipSuccess) return fail(c, OFDFT_E_DEVICE, "hipSetDevice");
  ScratchSave sv;
  int rc = dev_scratch_bind(c, &sv);
  if (rc) return fail(c, rc, c->err);
  // every step below uses the scratch-bound buffers; the context's own come back afterwards
  double h[SC_COUNT];
  Point p;
  rc = eval_at(c, phi_dev, c->v, c->scalars, p);
  if (!rc) rc = dev_grad_dots(c, phi_dev, c->v, c->scalars, nullptr, nullptr, c->scalars + SC_DOT0);
  if (!rc) rc = dev_read(c, c->scalars, SC_COUNT, h);
  if (!rc) rc = dev_to_double(c, c->v, v_dev);
  if (!rc) rc = dev_sync(c);
  dev_scratch_restore(c, &sv);
  if (rc) return fail(c, rc, c->err);
  // the report goes to the caller only: the context's last report and state (phi, converged)
  // stay those of its own calls
  ofdft_report r{};
  const bool conv = c->converged;
  const ofdft_report last = c->last;
  if ((rc = fill_report(c, h, std::sqrt(h[SC_DOT0 + 3] / (p.Ne / c->g.dv)), &r, 0, 1, 0))) return rc;
  c->last = last;
  c->converged = conv;
  if (rep) *rep = r;
  return OFDFT_OK;
}

int ofdft_time_evals(ofdft_ctx* c, int n_evals, double* total_ms, int max_kernels, const char** kernel_names,
                     double* kernel_ms, int* n_kernels) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (n_evals < 1 || !total_ms || max_kernels < 0 || (max_kernels > 0 && (!kernel_names || !kernel_ms)) || !n_kernels)
    return fail(c, OFDFT_E_ARG, "invalid timing arguments");
  Timing& t = c->timing;
  const size_t need = max_kernels > 0 ? (size_t)n_evals * 16 + 2 : 2;
  while (t.events.size() < need) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return fail(c, OFDFT_E_DEVICE, "hipEventCreate");
    t.events.push_back(e);
  }
  if (max_kernels == 0) {
    // whole-sequence timing only: one event before the first and one after the last evaluation
    if (hipEventRecord(t.events[0], c->stream) != hipSuccess) return fail(c, OFDFT_E_DEVICE, "hipEventRecord");
    for (int k = 0; k < n_evals; ++k)
      if ((rc = dev_eval(c, c->phi, c->v, c->scalars))) return fail(c, rc, c->err);
    if (hipEventRecord(t.events[1], c->stream) != hipSuccess) return fail(c, OFDFT_E_DEVICE, "hipEventRecord");
    if ((rc = dev_sync(c))) return fail(c, rc, c->err);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, t.events[0], t.events[1]);
    *total_ms = ms;
    *n_kernels = 0;
    return OFDFT_OK;
  }
  t.names.clear();
  t.used = 0;
  t.on = true;
  for (int k = 0; k < n_evals; ++k) {
    rc = dev_eval(c, c->phi, c->v, c->scalars);
    if (rc) {
      t.on = false;
      return fail(c, rc, c->err);
    }
  }
  t.on = false;
  if ((rc = dev_sync(c))) return fail(c, rc, c->err);
  const int per = t.used / n_evals;   // marks per evaluation (kernels + end)
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, t.events[0], t.events[t.used - 1]);
  *total_ms = ms;
  const int nk = std::min(per - 1, max_kernels);
  for (int k = 0; k < nk; ++k) {
    double acc = 0.0;
    for (int e = 0; e < n_evals; ++e) {
      float d = 0.0f;
      (void)hipEventElapsedTime(&d, t.events[e * per + k], t.events[e * per + k + 1]);
      acc += d;
    }
    kernel_ms[k] = acc / n_evals;
    kernel_names[k] = t.names[k];
  }
  *n_kernels = nk;
  return OFDFT_OK;
}

static bool tiles_valid(const ofdft_ctx* c, int tr, int tc, int rb) {
  const GridDesc& g = c->g;
  auto pow2 = [](int v) { return v >= 1 && (v & (v - 1)) == 0; };
  if (!pow2(tr) || tr < 2 || g.n2 % tr || !pow2(tc) || g.n2 % tc || !pow2(rb)) return false;
  // tiles staged through registers
  if (tr * g.n3 > kStageElems || (g.n3 / 2 + 1) * tr > kStageElems || g.n1 * tc > kStageElems ||
      rb * g.n2 > kX2Elems)
    return false;
  // the per-block partial sums were sized for tiles of at least 2
  if ((long long)(g.n2 / tr) * g.n1 > c->max_blocks || (long long)(g.n2 / tc) * g.n3h > c->max_blocks) return false;
  return true;
}

int ofdft_set_tiles(ofdft_ctx* c, const int tiles[3]) {
  if (!c) return fail(nullptr, OFDFT_E_ARG, "null context");
  if (!tiles) return fail(c, OFDFT_E_ARG, "tiles is NULL");
  if (!c->have_cell) return fail(c, OFDFT_E_STATE, "set_cell has not been called");
  if (!tiles_valid(c, tiles[0], tiles[1], tiles[2])) return fail(c, OFDFT_E_ARG, "invalid tiles for this grid");
  const GridDesc old = c->g;
  c->g.tr = tiles[0];
  c->g.tc = tiles[1];
  c->g.rb = tiles[2];
  if (dev_max_lds(c) > 159 * 1024) {   // 1 KB stays for the kernels' static LDS
    c->g = old;
    return fail(c, OFDFT_E_ARG, "tiles exceed the 160 KB LDS of a workgroup");
  }
  return OFDFT_OK;
}

int ofdft_autotune(ofdft_ctx* c, int n_evals, int tiles[3]) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (n_evals < 1) return fail(c, OFDFT_E_ARG, "n_evals must be >= 1");
  auto time_cfg = [&](int tr, int tc, int rb, double& ms) -> int {
    const int t[3] = {tr, tc, rb};
    if (!tiles_valid(c, tr, tc, rb)) return OFDFT_E_ARG;
    if (ofdft_set_tiles(c, t) != OFDFT_OK) return OFDFT_E_ARG;
    double tot;
    int nk = 0;
    int r2 = ofdft_time_evals(c, 1, &tot, 0, nullptr, nullptr, &nk);   // warm-up
    if (r2) return r2;
    r2 = ofdft_time_evals(c, n_evals, &tot, 0, nullptr, nullptr, &nk);
    ms = tot / n_evals;
    return r2;
  };
  int best[3] = {c->g.tr, c->g.tc, c->g.rb};
  double best_ms;
  if ((rc = time_cfg(best[0], best[1], best[2], best_ms))) return rc;
  const int cand[] = {1, 2, 4, 8, 16, 32, 64};
  for (int param = 2; param >= 0; --param) {   // x2 rows, then columns, then rows
    for (int v : cand) {
      int t[3] = {best[0], best[1], best[2]};
      t[param] = v;
      if (t[0] == best[0] && t[1] == best[1] && t[2] == best[2]) continue;
      double ms;
      const int r2 = time_cfg(t[0], t[1], t[2], ms);
      if (r2 == OFDFT_E_ARG) continue;
      if (r2) return fail(c, r2, c->err);
      if (ms < best_ms) {
        best_ms = ms;
        best[0] = t[0];
        best[1] = t[1];
        best[2] = t[2];
      }
    }
  }
  if ((rc = ofdft_set_tiles(c, best))) return rc;
  if (tiles) {
    tiles[0] = best[0];
    tiles[1] = best[1];
    tiles[2] = best[2];
  }
  return OFDFT_OK;
}

int ofdft_batch_minimize(ofdft_ctx* const* ctxs, int n, ofdft_report* reps) {
  if (!ctxs || n < 0) return fail(nullptr, OFDFT_E_ARG, "invalid batch");
  for (int i = 0; i < n; ++i)
    if (!ctxs[i]) return fail(nullptr, OFDFT_E_ARG, "null context in batch");
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j)
      if (ctxs[i] == ctxs[j]) return fail(nullptr, OFDFT_E_ARG, "a context appears twice in the batch");
  std::vector<int> rcs(n, OFDFT_OK);
  // graph-mode CG contexts: one host thread replays every cell's captured iteration
  std::vector<GraphRun> runs;
  std::vector<int> run_of(n, -1);
  for (int i = 0; i < n; ++i) {
    ofdft_ctx* c = ctxs[i];
    if (c->opt.graph_cg && c->opt.minimizer == OFDFT_CG) {
      int rc = check_ready(c);
      if (rc) { rcs[i] = rc; continue; }
      c->converged = false;
      GraphRun g;
      g.c = c;
      run_of[i] = (int)runs.size();
      runs.push_back(g);
    }
  }
  for (GraphRun& g : runs) {
    if (hipSetDevice(g.c->opt.device) != hipSuccess) g.rc = fail(g.c, OFDFT_E_DEVICE, "hipSetDevice");
    if (!g.rc) g.rc = graph_begin(g);
  }
  // other contexts: one host thread each (the host-driven minimisers block on readbacks)
  std::vector<std::thread> th;
  for (int i = 0; i < n; ++i)
    if (run_of[i] < 0 && rcs[i] == OFDFT_OK)
      th.emplace_back([&, i]() { rcs[i] = ofdft_minimize_density(ctxs[i], reps ? reps + i : nullptr); });
  for (bool busy = true; busy;) {
    busy = false;
    bool progress = false;
    for (GraphRun& g : runs) {
      if (g.rc || g.done) continue;
      const double before = g.seen;
      g.rc = graph_step(g, false);
      progress |= g.seen != before || g.done;
      busy |= !g.rc && !g.done;
    }
    if (busy && !progress) {
      std::this_thread::yield();
      // a failed launch or a drained stream shows up here rather than as a silent spin
      for (GraphRun& g : runs) {
        if (g.rc || g.done) continue;
        const hipError_t e = hipStreamQuery(g.c->stream);
        if (e != hipSuccess && e != hipErrorNotReady)
          g.rc = fail(g.c, OFDFT_E_DEVICE, std::string("graph CG: ") + hipGetErrorString(e));
        else if (e == hipSuccess && status_word(g.c, 0) <= g.seen)
          g.rc = fail(g.c, OFDFT_E_DEVICE, "graph CG: the stream drained without a status update");
      }
    }
  }
  for (int i = 0; i < n; ++i) {
    if (run_of[i] < 0) continue;
    GraphRun& g = runs[run_of[i]];
    if (g.rc) {
      (void)dev_sync(g.c);
      rcs[i] = g.rc;
    } else {
      rcs[i] = graph_finish(g, reps ? reps + i : nullptr);
    }
    if (rcs[i] == OFDFT_OK && g.c->opt.extrapolate > 0) rcs[i] = save_history(g.c);
  }
  for (auto& t : th) t.join();
  for (int i = 0; i < n; ++i)
    if (rcs[i]) {
      g_last_error = "batch member " + std::to_string(i) + ": " + ctxs[i]->err;
      return rcs[i];
    }
  return OFDFT_OK;
}

int ofdft_ewald(const double lattice[9], int nat, const double* tau, const double* Z, double* E, double* forces,
                double* stress) {
  if (!lattice || !tau || !Z || !E) return fail(nullptr, OFDFT_E_ARG, "NULL argument");
  if (nat < 1) return fail(nullptr, OFDFT_E_ARG, "nat must be >= 1");
  for (int k = 0; k < 9; ++k)
    if (!is_fin(lattice[k])) return fail(nullptr, OFDFT_E_ARG, "non-finite lattice");
  const double* a1 = lattice;
  const double* a2 = lattice + 3;
  const double* a3 = lattice + 6;
  const double det = a1[0] * (a2[1] * a3[2] - a2[2] * a3[1]) - a1[1] * (a2[0] * a3[2] - a2[2] * a3[0]) +
                     a1[2] * (a2[0] * a3[1] - a2[1] * a3[0]);
  if (!(std::fabs(det) > 1e-12)) return fail(nullptr, OFDFT_E_ARG, "singular lattice");
  for (int i = 0; i < nat; ++i) {
    if (!is_fin(tau[3 * i]) || !is_fin(tau[3 * i + 1]) || !is_fin(tau[3 * i + 2]))
      return fail(nullptr, OFDFT_E_ARG, "non-finite position");
    if (!(Z[i] > 0.0) || !is_fin(Z[i])) return fail(nullptr, OFDFT_E_ARG, "charges must be finite and > 0");
  }
  std::vector<double> F;
  double e = 0.0, s6[6];
  ewald_sum(lattice, nat, tau, Z, e, F, stress ? s6 : nullptr);
  *E = e;
  if (forces) std::copy(F.begin(), F.end(), forces);
  if (stress) {
    const double V = std::fabs(det);
    const int ia[6] = {0, 1, 2, 0, 1, 0}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int k = 0; k < 6; ++k) stress[3 * ia[k] + ib[k]] = stress[3 * ib[k] + ia[k]] = s6[k] / V;
  }
  return OFDFT_OK;
}

const char* ofdft_last_error(const ofdft_ctx* c) {
  if (c) return c->err.c_str();
  return g_last_error.c_str();
}

}  // extern "C"

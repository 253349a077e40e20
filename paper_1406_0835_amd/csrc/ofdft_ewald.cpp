// Ewald energy and forces of the ions (point charges Z_I in a neutralising
// background): the ion-ion term E_ion of the total free energy (arXiv:1406.0835
// Sec. II, the E_ion of the energy expression) and its forces.
//
// Host FP64, multithreaded.  Real space: for each pair the minimum-image
// separation plus the lattice translations that can bring it within r_cut.
// Reciprocal space: half of the G sphere (S(-G) = S(G)*), with e^{iG.R} built
// from per-ion phase tables along the three reciprocal axes.  Each thread sums
// a fixed slice and the slices are added in order, so a run is reproducible
// for a given thread count.  The standalone entry point sums both parts with a
// balanced splitting parameter; a context sums only the real-space, self and
// background terms, with the splitting parameter of grid_ewald_split, and takes
// the reciprocal part on the device from its structure factor.
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "ofdft_internal.h"

namespace ofdft {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

struct Partial {
  double E = 0.0;
  std::vector<double> F;
  double S[6] = {0, 0, 0, 0, 0, 0};   // strain-derivative sums (xx, yy, zz, xy, yz, xz)
};

// Threads for `items` independent work items, at least `per_thread` items each;
// one hardware thread is left to the caller that keeps the device busy meanwhile.
int thread_count(size_t items, size_t per_thread) {
  const unsigned hw = std::max(2u, std::thread::hardware_concurrency());
  const size_t by_work = std::max<size_t>(1, items / per_thread);
  return (int)std::min<size_t>({(size_t)std::min(hw - 1, 16u), by_work});
}

template <class Fn>
void run_threads(int nt, Fn&& fn) {
  if (nt <= 1) {
    fn(0);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(nt - 1);
  for (int t = 1; t < nt; ++t) th.emplace_back(fn, t);
  fn(0);
  for (auto& x : th) x.join();
}

}  // namespace

void ewald_sum(const double lat[9], int nat, const double* pos, const double* Z, double& E,
               std::vector<double>& F, double* strain6, double split_in, bool reciprocal) {
  const double* a[3] = {lat, lat + 3, lat + 6};
  auto cross = [](const double* u, const double* v, double* w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
  };
  double b[9];   // reciprocal rows, a_i . b_j = 2 pi delta_ij
  cross(a[1], a[2], b);
  cross(a[2], a[0], b + 3);
  cross(a[0], a[1], b + 6);
  const double det = a[0][0] * b[0] + a[0][1] * b[1] + a[0][2] * b[2];
  const double V = std::fabs(det);
  for (int k = 0; k < 9; ++k) b[k] *= 2.0 * kPi / det;
  // fractional coordinates f = R . b / (2 pi)
  std::vector<double> frac(3 * (size_t)nat);
  for (int i = 0; i < nat; ++i)
    for (int k = 0; k < 3; ++k)
      frac[3 * i + k] =
          (pos[3 * i] * b[3 * k] + pos[3 * i + 1] * b[3 * k + 1] + pos[3 * i + 2] * b[3 * k + 2]) / (2.0 * kPi);

  // splitting parameter: 1.4 x the textbook balance sqrt(pi) (N/V^2)^(1/6), which moves
  // work from the (erfc-bound) real-space sum to the cheaper reciprocal sum
  const double split = split_in > 0.0 ? split_in : 1.4 * std::sqrt(kPi) * std::pow(nat / (V * V), 1.0 / 6.0);
  const double cfac = std::sqrt(-std::log(1e-16));   // erfc(cfac) ~ 1e-17
  const double rcut = cfac / split, gcut = 2.0 * split * cfac;
  double Q = 0.0, Q2 = 0.0;
  for (int i = 0; i < nat; ++i) {
    Q += Z[i];
    Q2 += Z[i] * Z[i];
  }

  // ---- real space: translations T with |T| < rcut + (longest minimum-image separation),
  // the separation being sum_k d_k a_k with |d_k| <= 1/2, largest at a corner
  double half_diag = 0.0;
  for (int sg = 0; sg < 8; ++sg) {
    double c[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 3; ++k) {
      const double w = ((sg >> k) & 1) ? 0.5 : -0.5;
      for (int x = 0; x < 3; ++x) c[x] += w * a[k][x];
    }
    half_diag = std::max(half_diag, std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]));
  }
  const double reach = rcut + half_diag;
  int nmax[3];
  for (int k = 0; k < 3; ++k) {
    const double bn = std::sqrt(b[3 * k] * b[3 * k] + b[3 * k + 1] * b[3 * k + 1] + b[3 * k + 2] * b[3 * k + 2]);
    nmax[k] = (int)std::ceil(reach * bn / (2.0 * kPi));
  }
  // translations sorted by length: a pair at separation |d0| needs only |T| < rcut + |d0|
  std::vector<std::array<double, 4>> Ts;   // x, y, z, |T|
  for (int i = -nmax[0]; i <= nmax[0]; ++i)
    for (int j = -nmax[1]; j <= nmax[1]; ++j)
      for (int k = -nmax[2]; k <= nmax[2]; ++k) {
        const double t[3] = {i * a[0][0] + j * a[1][0] + k * a[2][0], i * a[0][1] + j * a[1][1] + k * a[2][1],
                             i * a[0][2] + j * a[1][2] + k * a[2][2]};
        const double tl = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
        if (tl < reach) Ts.push_back({t[0], t[1], t[2], tl});
      }
  std::sort(Ts.begin(), Ts.end(), [](const std::array<double, 4>& x, const std::array<double, 4>& y) {
    return x[3] < y[3] || (x[3] == y[3] && (x[0] < y[0] || (x[0] == y[0] && (x[1] < y[1] || (x[1] == y[1] && x[2] < y[2])))));
  });
  const size_t nT = Ts.size();
  const double c2 = 2.0 * split / std::sqrt(kPi);
  const double rc2 = rcut * rcut;
  // pairs i <= j, row i handled by one thread (rows interleaved for balance)
  const int ntr = thread_count((size_t)nat * (nat + 1) / 2, 512);
  std::vector<Partial> pr(ntr);
  run_threads(ntr, [&](int t) {
    Partial& P = pr[t];
    P.F.assign(3 * (size_t)nat, 0.0);
    for (int i = t; i < nat; i += ntr) {
      for (int j = i; j < nat; ++j) {
        // minimum-image separation of i and j (wrap the fractional difference)
        double df[3];
        for (int k = 0; k < 3; ++k) {
          const double x = frac[3 * i + k] - frac[3 * j + k];
          df[k] = x - std::nearbyint(x);
        }
        const double d0[3] = {df[0] * a[0][0] + df[1] * a[1][0] + df[2] * a[2][0],
                              df[0] * a[0][1] + df[1] * a[1][1] + df[2] * a[2][1],
                              df[0] * a[0][2] + df[1] * a[1][2] + df[2] * a[2][2]};
        const double tmax = rcut + std::sqrt(d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2]);
        double e = 0.0, fx = 0.0, fy = 0.0, fz = 0.0, sd[6] = {0, 0, 0, 0, 0, 0};
        for (size_t m = 0; m < nT && Ts[m][3] < tmax; ++m) {
          const double dx = d0[0] + Ts[m][0], dy = d0[1] + Ts[m][1], dz = d0[2] + Ts[m][2];
          const double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 >= rc2 || r2 < 1e-20) continue;
          const double r = std::sqrt(r2);
          const double ec = std::erfc(split * r) / r;
          e += ec;
          const double fm = (ec + c2 * std::exp(-split * split * r2)) / r2;
          fx += fm * dx;
          fy += fm * dy;
          fz += fm * dz;
          if (strain6) {
            sd[0] += fm * dx * dx; sd[1] += fm * dy * dy; sd[2] += fm * dz * dz;
            sd[3] += fm * dx * dy; sd[4] += fm * dy * dz; sd[5] += fm * dx * dz;
          }
        }
        const double zz = Z[i] * Z[j];
        P.E += (i == j ? 0.5 : 1.0) * zz * e;
        // d/d eps_ab of erfc(a r)/r summed: phi'(r) r_a r_b / r = -fm r_a r_b
        for (int k = 0; k < 6; ++k) P.S[k] -= (i == j ? 0.5 : 1.0) * zz * sd[k];
        if (i != j) {
          P.F[3 * i] += zz * fx; P.F[3 * i + 1] += zz * fy; P.F[3 * i + 2] += zz * fz;
          P.F[3 * j] -= zz * fx; P.F[3 * j + 1] -= zz * fy; P.F[3 * j + 2] -= zz * fz;
        }
      }
    }
  });

  // ---- reciprocal space: G = h b1 + k b2 + l b3, half space (h, k, l) > 0 lexicographically
  std::vector<Partial> pg;
  if (reciprocal) {
  int gmax[3];
  for (int k = 0; k < 3; ++k) {
    const double an = std::sqrt(a[k][0] * a[k][0] + a[k][1] * a[k][1] + a[k][2] * a[k][2]);
    gmax[k] = (int)std::ceil(gcut * an / (2.0 * kPi));
  }
  // phase tables e^{i m 2 pi f_k} for m in [-gmax_k, gmax_k]
  std::vector<std::complex<double>> tab[3];
  for (int k = 0; k < 3; ++k) {
    const int M = 2 * gmax[k] + 1;
    tab[k].resize((size_t)nat * M);
    for (int i = 0; i < nat; ++i)
      for (int m = -gmax[k]; m <= gmax[k]; ++m) {
        const double ph = 2.0 * kPi * m * frac[3 * i + k];
        tab[k][(size_t)i * M + m + gmax[k]] = {std::cos(ph), std::sin(ph)};
      }
  }
  struct GVec {
    int h, k, l;
  };
  std::vector<GVec> gl;
  for (int h = 0; h <= gmax[0]; ++h)
    for (int k = (h == 0 ? 0 : -gmax[1]); k <= gmax[1]; ++k)
      for (int l = (h == 0 && k == 0 ? 1 : -gmax[2]); l <= gmax[2]; ++l) {
        const double G[3] = {h * b[0] + k * b[3] + l * b[6], h * b[1] + k * b[4] + l * b[7],
                             h * b[2] + k * b[5] + l * b[8]};
        if (G[0] * G[0] + G[1] * G[1] + G[2] * G[2] <= gcut * gcut) gl.push_back({h, k, l});
      }
  const int ntg = thread_count(gl.size() * (size_t)nat, 16384);
  pg.resize(ntg);
  const int M0 = 2 * gmax[0] + 1, M1 = 2 * gmax[1] + 1, M2 = 2 * gmax[2] + 1;
  run_threads(ntg, [&](int t) {
    Partial& P = pg[t];
    P.F.assign(3 * (size_t)nat, 0.0);
    std::vector<std::complex<double>> e(nat);
    for (size_t q = t; q < gl.size(); q += ntg) {
      const GVec& gv = gl[q];
      const double G[3] = {gv.h * b[0] + gv.k * b[3] + gv.l * b[6], gv.h * b[1] + gv.k * b[4] + gv.l * b[7],
                           gv.h * b[2] + gv.k * b[5] + gv.l * b[8]};
      const double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
      const double w = std::exp(-G2 / (4.0 * split * split)) / G2;
      std::complex<double> S = 0.0;
      for (int i = 0; i < nat; ++i) {
        e[i] = tab[0][(size_t)i * M0 + gv.h + gmax[0]] * tab[1][(size_t)i * M1 + gv.k + gmax[1]] *
               tab[2][(size_t)i * M2 + gv.l + gmax[2]];
        S += Z[i] * e[i];
      }
      // +G and -G together: 2 w |S|^2 and forces 2 (4 pi/V) Z_I w G Im[e^{iG.R_I} S*]
      P.E += 2.0 * w * std::norm(S);
      if (strain6) {
        // strain derivative of w(G): w 2 G_a G_b (1/G^2 + 1/(4 a^2)) (G scales as (1 + eps)^-T)
        const double k2 = 2.0 * w * std::norm(S) * 2.0 * (1.0 / G2 + 1.0 / (4.0 * split * split));
        P.S[0] += k2 * G[0] * G[0]; P.S[1] += k2 * G[1] * G[1]; P.S[2] += k2 * G[2] * G[2];
        P.S[3] += k2 * G[0] * G[1]; P.S[4] += k2 * G[1] * G[2]; P.S[5] += k2 * G[0] * G[2];
      }
      for (int i = 0; i < nat; ++i) {
        const double im = e[i].imag() * S.real() - e[i].real() * S.imag();
        const double f = 2.0 * 4.0 * kPi / V * Z[i] * w * im;
        P.F[3 * i] += f * G[0];
        P.F[3 * i + 1] += f * G[1];
        P.F[3 * i + 2] += f * G[2];
      }
    }
  });
  }

  F.assign(3 * (size_t)nat, 0.0);
  double Er = 0.0, Eg = 0.0;
  for (const Partial& P : pr) {
    Er += P.E;
    for (size_t k = 0; k < F.size(); ++k) F[k] += P.F[k];
  }
  for (const Partial& P : pg) {
    Eg += P.E;
    for (size_t k = 0; k < F.size(); ++k) F[k] += P.F[k];
  }
  Eg *= 2.0 * kPi / V;
  const double Es = -split / std::sqrt(kPi) * Q2;
  const double Eb = -kPi * Q * Q / (2.0 * V * split * split);
  E = Er + Eg + Es + Eb;
  if (strain6) {
    // V Sigma: real-space pair terms, reciprocal terms minus delta E_rec, minus delta E_bg
    // (the self term does not depend on the cell)
    double sr[6] = {0, 0, 0, 0, 0, 0}, sg[6] = {0, 0, 0, 0, 0, 0};
    for (const Partial& P : pr)
      for (int k = 0; k < 6; ++k) sr[k] += P.S[k];
    for (const Partial& P : pg)
      for (int k = 0; k < 6; ++k) sg[k] += P.S[k];
    for (int k = 0; k < 6; ++k) strain6[k] = sr[k] + 2.0 * kPi / V * sg[k] - (k < 3 ? Eg + Eb : 0.0);
  }
}

double grid_ewald_split(const ofdft_ctx* c) {
  // |m_k| = |G . a_k| / 2 pi <= |G| |a_k| / 2 pi, so the sphere |G| < G_in with
  // G_in = min_k 2 pi (n_k/2 - 1) / |a_k| lies inside the kept modes
  const int n[3] = {c->g.n1, c->g.n2, c->g.n3};
  double g_in = 1e300;
  for (int k = 0; k < 3; ++k) {
    const double* a = c->lat + 3 * k;
    const double an = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    g_in = std::min(g_in, 2.0 * kPi * (n[k] / 2 - 1) / an);
  }
  return g_in / (2.0 * std::sqrt(-std::log(1e-16)));
}

void start_ewald(ofdft_ctx* c) {
  join_ewald(c);
  c->ewald_failed = false;
  c->ewald_pending = true;
  c->ewald_split = grid_ewald_split(c);
  c->ewald_thread = std::thread([c] {
    try {
      ewald_sum(c->lat, c->nat, c->tau.data(), c->Z.data(), c->E_ion_host, c->F_ion, c->ewald_strain,
                c->ewald_split, false);
    } catch (...) {
      c->ewald_failed = true;
    }
  });
}

bool join_ewald(ofdft_ctx* c) {
  if (c->ewald_pending) {
    c->ewald_thread.join();
    c->ewald_pending = false;
    c->E_ion = c->E_ion_host + c->E_rec;
  }
  return !c->ewald_failed;
}

}  // namespace ofdft

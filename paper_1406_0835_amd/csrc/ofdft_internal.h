// Internal context shared by the kernel file and the host API.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <thread>
#include <vector>

#include "../../include/ofdft.h"

namespace ofdft {

// Slots of the per-block partial sums written by the evaluation kernels.
// SL_DT1, SL_DT2: sums phi_t v_t q and phi_t q of a line-search trial (q = ms phi + mc d),
// from which the reduction forms dF/dtheta once mu is known.
// SL_TSXC: n T s_xc of a temperature-dependent XC (KSDT), zero otherwise.
enum Slot { SL_PHI2 = 0, SL_FS, SL_TS, SL_EXC, SL_EH, SL_EEXT, SL_NV, SL_DT1, SL_DT2, SL_TSXC, SL_COUNT };
// Reduced scalars of one evaluation (double[SC_COUNT] on the device).  On the device
// SC_FTOT is the electronic part of F (E_ion, a constant of the minimisation, is
// added on the host) and SC_EION is 0.
constexpr int kMapDoubles = 64;
enum Scal {
  SC_NE = 0, SC_FS, SC_TS, SC_EXC, SC_EH, SC_EEXT, SC_NV, SC_MU, SC_EAZ, SC_EION, SC_FTOT,
  SC_DOT0 = 11,   // slots 11..15: minimiser dot products written after an evaluation
  SC_BETA = 16,   // CG coefficients formed on the device from those dots: beta, c_z
  SC_CZ = 17,
  SC_DD = 18,     // d.d and d.g of the new CG direction
  SC_DG = 19,
  SC_TH1 = 20,    // first line-search angle along it and the rotation/slope
  SC_CA = 21,     // coefficients of that trial: ca, sb, ms, mc (contiguous)
  SC_SB = 22,
  SC_MS = 23,
  SC_MC = 24,
  SC_TSXC = 25,   // T S_xc = -T dF_xc/dT (KSDT; 0 for PZ81)
  SC_COUNT = 26
};

// State of the device-resident CG iteration (HIP-graph mode), doubles in device memory.
// The control kernels of an iteration read and write it; every other kernel of the
// iteration reads one of the gate words on entry.
enum CgSlot {
  CG_ACTIVE = 0,   // 1 while the minimisation runs (gate of the CG-step kernels)
  CG_GATE1,        // the direction descends: evaluate the first trial
  CG_GATE2,        // the first trial failed the line-search test: evaluate a second one
  CG_GATEACC,      // a trial was accepted: copy it into the current state
  CG_SRC,          // the trial taken (1 or 2; 0 none)
  CG_HAVE_PREV, CG_GG_PREV, CG_CPROJ, CG_F, CG_F_PREV, CG_KAPPA, CG_SMALL, CG_LAST_DF,
  CG_ITERS, CG_EVALS, CG_CONVERGED, CG_STATUS, CG_NF_USED, CG_LSR_USED, CG_TRIALS,
  CG_DF0, CG_DN, CG_RESID, CG_GG, CG_LAUNCHES, CG_F1, CG_D1, CG_TH2,
  CG_THCAP,        // cap on the next first trial angle after a failed line search (0: none)
  CG_COEF2,        // ca, sb, ms, mc of the second trial (4 doubles)
  CG_COUNT = CG_COEF2 + 4
};
enum CgStatus { CGS_RUNNING = 0, CGS_CONVERGED = 1, CGS_STALLED = 2, CGS_MAXITER = 3, CGS_NONFINITE = 4 };
// Where the control kernel publishes an iteration's status in the context's mapped host
// memory (hmap[kMapStatus + k]): launches, active, status, iterations, evaluations, F.
constexpr int kMapStatus = 54;

// Constants of one graph-mode minimisation, captured with the graph.
struct CgConst {
  double r;           // sphere radius sqrt(N_e / dv)
  double dv, tol_energy, tol_residual;
  int max_iter, pcg, mixed, inject_at;
};

// Largest tiles the kernels stage through registers: a contiguous-axis tile
// (tr rows of N3 reals, or (N3/2+1) tr spectrum elements) and an x1 tile
// (N1 tc elements) hold at most kStageElems elements; an x2 tile (rb rows of
// N2) at most kX2Elems.  All tile sizes are powers of two.
constexpr int kStageElems = 2048;
constexpr int kX2Elems = 4096;

struct GridDesc {
  int n1, n2, n3, n3h;
  int n3k;        // k3 planes that carry kept modes: k3 < n3/2 (the k3 = n3/2 plane is all Nyquist)
  long long N;    // n1 n2 n3 real points
  long long NS;   // n3h n1 n2 half-spectrum points (layout [k3][k1][k2])
  double b[9];    // reciprocal lattice rows b1, b2, b3 (a_i . b_j = 2 pi delta_ij)
  double volume, dv, inv_n;
  double prec_k2; // reciprocal-space filter 1/(1 + G^2/prec_k2) of the preconditioned minimiser
  int tr;         // rows per block in the contiguous-axis pass (power of two >= 2, divides n2)
  int tc;         // columns per block in the strided pass (power of two, divides n2)
  int rb;         // rows per block in the x2 pass (power of two)
  int pwb;        // blocks of the pointwise kernels: one resident round on the device (0: default)
  // Device flag the evaluation and CG kernels read on entry: 0.0 makes the whole launch
  // return at once (the HIP-graph CG iteration skips work this way); nullptr: always run.
  const double* gate;
};

struct LppParams {
  int kind;       // 0 Gaussian, 1 Heine-Abarenkov
  double rc, A, qc;
};

struct EvalParams {
  int functional;
  int xc;
  double T;           // hartree
  double lt0;         // ln t = lt0 - (2/3) ln n
  double alpha_sum;   // sum_I alpha_I (G = 0 remainder of the pseudopotential)
  double enh_kind, enh_c1, enh_a1;   // enhancement-factor parameters (kind as double)
  const double* gate;                // as GridDesc::gate
};

// What a captured CG-iteration graph depends on: the launches bake in the grid and tiles,
// the evaluation parameters, the minimisation constants and the buffers the line search
// alternates between (their pointers are swapped by the host-driven minimisers).
struct GraphKey {
  GridDesc g;
  EvalParams ep;
  CgConst k;
  const void* bufs[9];
  int pcg, plane;
};

struct Timing {
  bool on = false;
  std::vector<hipEvent_t> events;   // one before each kernel, one at the end
  std::vector<const char*> names;
  int used = 0;
};

}  // namespace ofdft

struct ofdft_ctx {
  ofdft_options opt{};
  std::string err;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool have_cell = false, have_ions = false, have_T = false, have_phi = false, converged = false;

  // cell and grid
  double lat[9] = {0};
  double cell_scale = 1.0;
  ofdft::GridDesc g{};
  double T_ha = 0.0;

  // ions
  int nat = 0;
  std::vector<double> tau, Z;
  double Ne = 0.0, alpha_sum = 0.0, E_ion = 0.0;
  std::vector<double> F_ion;
  double ewald_strain[6] = {0, 0, 0, 0, 0, 0};   // V Sigma of the Ewald energy (xx yy zz xy yz xz)
  // The host thread sums the real-space, self and background Ewald terms with the
  // splitting parameter ewald_split into E_ion_host, F_ion and ewald_strain; the
  // reciprocal-space energy E_rec comes from the device structure factor (set_ions),
  // its forces and strain terms from the force and stress kernels.  join_ewald sets
  // E_ion = E_ion_host + E_rec.
  double E_ion_host = 0.0, E_rec = 0.0, ewald_split = 0.0;
  // E_ion and F_ion come from a host thread started by set_ions; every reader
  // (and every writer of lat, nat, tau, Z) joins it first (ofdft::join_ewald)
  std::thread ewald_thread;
  bool ewald_pending = false, ewald_failed = false;

  // device buffers (R = float or double by precision)
  size_t rsize = 8;
  double* phi = nullptr;     // current amplitude
  double* phi_t = nullptr;   // trial amplitude
  void* v = nullptr;         // potential at phi (R)
  void* v_t = nullptr;       // potential at phi_t (R)
  void* vloc = nullptr;      // local part df/dn + v_xc (R)
  void* A = nullptr;         // spectra, cplx<R>[NS]
  void* B[3] = {nullptr, nullptr, nullptr};
  void* S0 = nullptr;
  void* D = nullptr;
  void* gr[3] = {nullptr, nullptr, nullptr};   // real grad n / W components (R)
  void* Vext = nullptr;
  void* tw[3] = {nullptr, nullptr, nullptr};   // twiddles per axis, cplx<R>[n_a]
  double* partials = nullptr;  // [SL_COUNT][max_blocks]
  int max_blocks = 0;
  double* scalars = nullptr;   // current point, double[SC_COUNT]
  double* scalars_t = nullptr; // trial point
  // a second trial buffer: the line search keeps its best trial while it evaluates the next
  double* phi_t2 = nullptr;
  void* v_t2 = nullptr;
  double* scalars_t2 = nullptr;
  // minimiser vectors
  double* d = nullptr;
  double* gprev = nullptr;
  // converged amplitudes of the last ionic steps (extrapolate > 0): slot
  // (hist_head - j) mod 3 holds phi_{k-j}, j < n_hist
  double* phi_hist[3] = {nullptr, nullptr, nullptr};
  int n_hist = 0, hist_head = 0;
  double* tn[4] = {nullptr, nullptr, nullptr, nullptr};
  double* vpart = nullptr;     // vector-reduction partials
  double* vout = nullptr;      // vector-reduction results
  // Fine-grained pinned host memory the device writes small results into:
  // doubles [0, kMapDoubles) of data, then a 64-bit sequence word the host waits on.
  // x3 and x2 transforms as one plane pass where the grid allows (on unless
  // OFDFT_PLANE_PASSES=0 in the environment at ofdft_create)
  bool plane_passes = true;
  // mixed precision on square planes of 32, 64 or 128: the inverse gradient transforms and
  // the pointwise functional as one fused plane pass, and the density and final passes split
  // without repeated transform work (on unless OFDFT_FUSED_GGA=0 in the environment at
  // ofdft_create)
  bool fused_gga = true;
  // force kernel: -1 picks by ion count, 0 the G-parallel one, 1 one thread per ion
  // (OFDFT_ION_FORCES in the environment at ofdft_create)
  int ion_forces = -1;
  // recovery tests (OFDFT_TEST_NONFINITE at ofdft_create): the host treats line-search trial
  // number test_nonfinite (counted from 1 over the context's life; < 0: every trial) as
  // non-finite.  0 = off.
  int test_nonfinite = 0;
  long long trials_seen = 0;
  double* hmap = nullptr;
  double* dmap = nullptr;      // the same memory as seen by kernels
  unsigned long long read_seq = 0;
  // ions on the device
  double* phase = nullptr;     // [nat][n1 + n2 + n3h] complex doubles
  // structure factors sum_I Z_I e^{-iG.R_I} and sum_I e^{-iG.R_I} on the half spectrum
  // ([2][NS] complex doubles), written with V_ext and read by the stress
  double* sfac = nullptr;
  double* dZ = nullptr;
  double* fpart = nullptr;
  double* dforces = nullptr;
  long long phase_cap = 0;   // entries of the phase tables (nat * (n1 + n2 + n3h))
  int ion_cap = 0;           // ions that dZ and dforces are sized for
  long long fpart_cap = 0;   // doubles in fpart (force, stress and energy partial sums)

  // HIP-graph CG (options.graph_cg): device state (CgSlot doubles) and the captured iteration
  double* cgst = nullptr;
  hipGraph_t cg_graph = nullptr;
  hipGraphExec_t cg_exec = nullptr;
  ofdft::GraphKey cg_key{};

  ofdft::Timing timing;
  ofdft_report last{};
};

namespace ofdft {

// Ewald energy and forces of the ions (ofdft_ewald.cpp, host FP64): lat rows a1..a3 (bohr),
// Cartesian pos[3 nat], charges Z[nat]; F receives 3 nat forces (hartree/bohr).
// strain6, if given, receives V Sigma of the Ewald energy (xx, yy, zz, xy, yz, xz).
// split > 0 fixes the splitting parameter; reciprocal = false leaves out the
// reciprocal-space sum (energy, forces and strain), which the library's contexts
// take on the device from the stored structure factor.
void ewald_sum(const double lat[9], int nat, const double* pos, const double* Z, double& E, std::vector<double>& F,
               double* strain6 = nullptr, double split = 0.0, bool reciprocal = true);
// Splitting parameter for which the reciprocal Ewald sum is complete on the FFT
// grid of the context (exp(-G^2/4a^2) <= 1e-16 beyond the largest sphere inside
// the grid's G set).
double grid_ewald_split(const ofdft_ctx* c);
// Start ewald_sum for the context's current ions on a host thread / wait for it
// (false if it failed).
void start_ewald(ofdft_ctx* c);
bool join_ewald(ofdft_ctx* c);

// Size of the static device scratch array of ofdft_eval_noalloc (OFDFT_NOALLOC_SCRATCH_BYTES).
constexpr size_t kNoAllocScratchBytes = OFDFT_NOALLOC_SCRATCH_BYTES;

// The context's evaluation buffers while ofdft_eval_noalloc points them into the static
// scratch array (dev_scratch_bind saves them, dev_scratch_restore puts them back).
struct ScratchSave {
  void* A; void* S0; void* D; void* B[3]; void* gr[3]; void* vloc; void* v;
  double* partials; double* scalars; double* vpart; double* vout;
};

// Device memory of a context: the caller's allocator (options.alloc / free_) when
// one is set, else hipMalloc / hipFree.  ctx_malloc returns hipErrorOutOfMemory
// when the callback returns NULL; ctx_free ignores NULL.
hipError_t ctx_malloc(ofdft_ctx* c, void** p, size_t bytes);
void ctx_free(ofdft_ctx* c, void* p);

// kernels (ofdft_kernels.hip)
// Uploads the t-factor tables and resolves the static scratch address, once per device.
int dev_upload_tables(int device);
// Scratch bytes one evaluation of the context needs; binding fails with OFDFT_E_ARG above
// kNoAllocScratchBytes.
size_t dev_noalloc_bytes(const ofdft_ctx* c);
int dev_scratch_bind(ofdft_ctx* c, ScratchSave* sv);
void dev_scratch_restore(ofdft_ctx* c, const ScratchSave* sv);
// out[0..N) = the grid array v (context precision) as doubles, on the context's stream.
int dev_to_double(ofdft_ctx* c, const void* v, double* out);
int dev_alloc_grid(ofdft_ctx* c);
void dev_free_grid(ofdft_ctx* c);
int dev_alloc_ions(ofdft_ctx* c);
int dev_structure_factor(ofdft_ctx* c);
// With host != NULL the reduced scalars are also delivered to host[SC_COUNT] (through
// c->hmap, written by the reduction kernel) before the call returns.
int dev_eval(ofdft_ctx* c, const double* phi, void* v_out, double* scalars_out, double* host = nullptr);
// One line-search trial as a single evaluation: phi_out = ca phi + sb dir is formed inside
// the density pass, and dF/dtheta = g_t . (ms phi + mc dir) lands in scalars_out[SC_DOT0].
int dev_eval_trial(ofdft_ctx* c, const double* phi, const double* dir, double ca, double sb, double* phi_out,
                   void* v_out, double* scalars_out, double ms, double mc, double* host = nullptr);
// The same trial with ca, sb, ms, mc read on the device from coef[0..3]; host receives
// the trial's scalars followed by extra[0..SC_COUNT) (2 SC_COUNT doubles).
int dev_eval_trial_dev(ofdft_ctx* c, const double* phi, const double* dir, const double* coef, double* phi_out,
                       void* v_out, double* scalars_out, const double* extra, double* host);
int dev_forces(ofdft_ctx* c, double* forces_host);
// Stress sums at the current density: sums[0] = dv sum (f - n df/dn), sums[1] = dv sum
// n (eps_xc - v_xc), sums[2..7] = dv sum W_a d_b n, sums[8..13] Hartree and
// sums[14..19] pseudopotential reciprocal sums (xx, yy, zz, xy, yz, xz).
int dev_stress(ofdft_ctx* c, double* sums);
// vector operations for the minimisers; results land in c->vout (device)
// g = 2 dv phi (v - mu): writes g.g, g.gprev, g.d, sum n (v-mu)^2 into out[0..3]
int dev_grad_dots(ofdft_ctx* c, const double* phi, const void* v, const double* sc, const double* gprev,
                  const double* d, double* out);
int dev_cg_direction(ofdft_ctx* c, double beta, double cproj);
// One CG step's device part, leaving everything the host needs in c->scalars.
// Dots into SC_DOT0..: plain, g.g, g.gprev, g.d, sum n (v-mu)^2; preconditioned
// (pcg), z.g, z.gprev, z.phi, sum n (v-mu)^2, phi.gprev with z = P g, P the
// reciprocal-space filter with g.prec_k2, formed as g + w, w = (P - 1) g in
// c->gr[0].  Then c_z = z.phi / phi.phi and beta = max(0, (z.g - (z.gprev -
// c_z phi.gprev)) / gg_prev) (0 without have_prev; plain: c_z = 0) into
// SC_CZ/SC_BETA, and the new direction d = -(z - c_z phi) + beta (d - cproj phi)
// (gprev = g) with d.d, d.g into SC_DD/SC_DG.
// Also the first line-search angle along d (the rule of first_step with the
// previous free energy F_prev, the previous curvature kappa (0: none) and the
// sphere radius r) and that trial's rotation and slope coefficients into SC_TH1,
// SC_CA..SC_MC.
int dev_cg_step(ofdft_ctx* c, bool pcg, bool have_prev, double gg_prev, double cproj, double F_prev, double r,
                double kappa);
// The same direction with beta = 0 (after a step that was not a descent direction).
int dev_cg_restart(ofdft_ctx* c, bool pcg);
// HIP-graph CG: capture one device-resident CG iteration (when the key changed), start a
// minimisation from the evaluation in c->scalars (k_cg_init), replay the iteration.
int dev_cg_graph_prepare(ofdft_ctx* c, bool pcg, const CgConst& k);
int dev_cg_graph_start(ofdft_ctx* c);
int dev_cg_graph_launch(ofdft_ctx* c);
void dev_cg_graph_release(ofdft_ctx* c);
int dev_rotate(ofdft_ctx* c, double* dst, const double* phi, double ca, const double* dir, double sb);
// dF/dtheta at the trial point, written to out[0]
int dev_dtheta(ofdft_ctx* c, const double* phi_t, const void* v_t, const double* sc_t, const double* phi,
               const double* d, double ms, double mc, double* out);
int dev_full_grad_acc(ofdft_ctx* c, double* out, const double* phi_t, const void* v_t, double sign);
int dev_dot(ofdft_ctx* c, const double* a, const double* b);
int dev_axpby(ofdft_ctx* c, double* y, double a, const double* x, double b);
// dst = c0 x0 + c1 x1 + c2 x2 (x2 may be NULL when c2 = 0); dst.dst into c->vout[0]
int dev_combine3(ofdft_ctx* c, double* dst, double c0, const double* x0, double c1, const double* x1, double c2,
                 const double* x2);
int dev_tn_hess_finish(ofdft_ctx* c, double* hs, const double* phi, const double* s, double inv2e,
                       double mu_term);
// n <= kMapDoubles doubles from device memory to the host (a one-wavefront kernel
// writes them into c->hmap and raises its sequence word; no stream synchronisation).
int dev_read(ofdft_ctx* c, const double* dptr, int n, double* host);
int dev_sync(ofdft_ctx* c);
// largest dynamic LDS (bytes) any evaluation kernel needs with the tiles in c->g
size_t dev_max_lds(const ofdft_ctx* c);

}  // namespace ofdft

/*
 * ofdft.h - C ABI of the MI355X finite-temperature orbital-free DFT library.
 *
 * The library evaluates and minimises the electronic free energy of a periodic
 * cell at electron temperature T with the density written as n = phi^2 on a
 * real-space grid, and returns the free energy and the ionic forces at the
 * minimum.  This is the per-ionic-step work of orbital-free DFT molecular
 * dynamics (Karasiev, Sjostrom, Trickey, arXiv:1406.0835):
 *   - objective: F_tot[n] = F_s[n] + F_H[n] + F_xc[n] + int n v_ext + E_ion
 *     (Sec. II, Eqs. E1, E3, E4), minimised directly at fixed int n = N_e;
 *   - F_s: finite-T Thomas-Fermi (Eqs. TF, fTF, tred, vTF) or a finite-T
 *     GGA of the form of Eq. FGGA (SGA, VWTF, VT84F, KST2, TW, APBEF;
 *     Eqs. xizeta, s_s, s_0defn, VT84F, KST2F, SGA-F, vftGGA);
 *   - F_xc: ground-state LDA in the Perdew-Zunger parametrisation (the "PZ"
 *     XC of Sec. VI), the finite-T LDA of Sec. IV A (KSDT, Eq. fit2) or none;
 *   - F_H in reciprocal space (Eq. E2); v_ext from a local pseudopotential
 *     structure-factor sum (Gaussian-regularised Coulomb, or the
 *     Heine-Abarenkov form of Eq. E4A);
 *   - forces at the converged density (Eq. M12) plus the Ewald ion-ion term.
 * The call pattern mirrors the interface of Sec. V D (ions and temperature in,
 * free energy, internal energy and forces out), with the geometry keywords of
 * Sec. V B (TEMP in kelvin, cellScale).
 *
 * Conventions
 *   - Hartree atomic units (bohr, hartree, hartree/bohr); temperature in kelvin.
 *   - Every function returns an int status: OFDFT_OK (0) or a negative
 *     OFDFT_E_* code; ofdft_last_error() gives a message.  No C++ exception
 *     crosses the boundary.  Arguments are validated before any device work.
 *   - All array arguments are host pointers owned by the caller.  They are
 *     copied in by set_* and written by the output functions; the library
 *     keeps no reference to them.  The library owns its device buffers.
 *   - Grid arrays (phi, potentials, gradients) are row-major [N1][N2][N3]
 *     with the third index contiguous; point (j1,j2,j3) sits at
 *     r = j1/N1 a1 + j2/N2 a2 + j3/N3 a3.
 *   - A context is not thread-safe; different contexts may be used from
 *     different threads.
 */
#ifndef OFDFT_H
#define OFDFT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define OFDFT_OK 0
#define OFDFT_E_ARG (-1)           /* invalid argument (NULL, nat <= 0, T <= 0, singular cell, ...) */
#define OFDFT_E_GRID (-2)          /* grid size not one of the supported lengths (ofdft_set_cell) */
#define OFDFT_E_NOT_CONVERGED (-3) /* minimisation hit max_iter; the best state is kept */
#define OFDFT_E_NONFINITE (-4)     /* a non-finite energy or gradient appeared */
#define OFDFT_E_DEVICE (-5)        /* HIP runtime or allocation failure */
#define OFDFT_E_STATE (-6)         /* call out of order (e.g. forces before a converged minimisation) */

/* non-interacting free-energy functional (Table I keywords KINE ...) */
#define OFDFT_TF 0      /* finite-T Thomas-Fermi */
#define OFDFT_SGA 1     /* second-order gradient approximation, mu = mu_sga (default 5/27) */
#define OFDFT_VWTF 2    /* SGA form with mu = 5/3 */
#define OFDFT_VT84F 3   /* VT84F */
#define OFDFT_KST2 4    /* KST2: C1 = 2.03087, a1 = 0.29424 */
#define OFDFT_TW 5      /* finite-T Tran-Wesolowski: C1 = 0.2319, a1 = 0.2748 */
#define OFDFT_APBEF 6   /* finite-T APBEK: C1 = 0.23889, a1 = C1/0.804 */

#define OFDFT_XC_NONE 0
#define OFDFT_XC_PZ81 1 /* ground-state LDA, Perdew-Zunger parametrisation (temperature-independent) */
#define OFDFT_XC_KSDT 2 /* finite-T LDA XC free energy of Sec. IV A (Eq. fit2, spin-unpolarised,
                           parameters of the fit's publication), potential by Eq. vxc1, stress by
                           Eq. stressLSDAxc; evaluated in FP64 in both precisions */

#define OFDFT_LPP_GAUSS 0 /* v(r) = -Z erf(r/rc)/r */
#define OFDFT_LPP_HA 1    /* Heine-Abarenkov, Eq. E4A (rc, A, qc) */

#define OFDFT_FP64 0  /* everything in FP64 */
#define OFDFT_MIXED 1 /* FFTs and gradient terms in FP32; Fermi-Dirac inversion, t-factors,
                         reductions, minimiser vectors and line search in FP64 */

#define OFDFT_CG 0 /* Polak-Ribiere nonlinear CG on the electron-count sphere */
#define OFDFT_TN 1 /* truncated Newton (Newton-CG in the tangent space) */

typedef struct ofdft_ctx ofdft_ctx;

typedef struct {
  int functional;      /* OFDFT_TF ... OFDFT_APBEF */
  double mu_sga;       /* SGA coefficient (PARA MU); used by OFDFT_SGA */
  int xc;              /* OFDFT_XC_NONE, OFDFT_XC_PZ81 or OFDFT_XC_KSDT */
  int lpp;             /* OFDFT_LPP_GAUSS or OFDFT_LPP_HA */
  double lpp_rc;       /* bohr */
  double lpp_A;        /* hartree (HA only) */
  double lpp_qc;       /* bohr^-1 (HA only) */
  int precision;       /* OFDFT_FP64 or OFDFT_MIXED */
  int minimizer;       /* OFDFT_CG or OFDFT_TN */
  double tol_energy;   /* stop when |F_k - F_{k-1}| < tol_energy (hartree) twice in a row */
  double tol_residual; /* and, if > 0, sqrt(sum n (v-mu)^2 / sum n) < tol_residual (hartree) */
  int max_iter;        /* outer iterations */
  int device;          /* HIP device ordinal */
  void* stream;        /* hipStream_t to launch on; NULL = a stream owned by the context */
  double cg_precond;   /* CG with a gradient functional: > 0 filters the gradient with
                          1/(1 + G^2/(cg_precond k_F^2)) in reciprocal space (k_F^2 = (3 pi^2 N_e/V)^(2/3))
                          before the direction update (preconditioned Polak-Ribiere); 0 = plain CG.
                          ftTF always uses plain CG.  Changes the iteration path, not the minimum. */
  int extrapolate;     /* starting amplitude of the next ofdft_minimize_density after ofdft_set_ions
                          moves the ions (an ionic step): 0 = the last density as it is; 1 = linear
                          extrapolation 2 phi_k - phi_{k-1} of the last two converged amplitudes;
                          2 = quadratic, 3 phi_k - 3 phi_{k-1} + phi_{k-2}.  The result is renormalised
                          to N_e.  Converged amplitudes are remembered per context; ofdft_set_cell,
                          ofdft_set_density and a change of N_e clear the history, and the order drops
                          to what the history holds.  Changes the starting point, not the minimum. */
  /* Device memory of the context.  alloc == NULL: the library calls hipMalloc/hipFree.
     Otherwise every device buffer of the context (grids, spectra, minimiser vectors,
     ion tables, partial sums) comes from alloc(bytes, alloc_ctx), which returns a
     device pointer on opt.device aligned to at least 256 bytes, or NULL (then the
     calling entry point fails with OFDFT_E_DEVICE), and goes back through
     free_(ptr, alloc_ctx) when the context releases it (set_cell, destroy).  Both
     must be set together (OFDFT_E_ARG otherwise).  Buffers are used only on the
     context's stream; a caching allocator bound to that stream (e.g. PyTorch's,
     with stream = its current stream) may hand them out.  The callbacks may be
     called from the thread that calls any entry point of the context, including
     the worker threads of ofdft_batch_minimize.  The small pinned host buffer the
     device writes its results into stays with hipHostMalloc. */
  void* (*alloc)(size_t bytes, void* alloc_ctx);
  void (*free_)(void* ptr, void* alloc_ctx);
  void* alloc_ctx;
  int graph_cg;        /* CG minimiser only.  1: each CG iteration is one replay of a HIP graph whose
                          launches take every decision on the device (stop rule, line search with at
                          most two trials: the first at the curvature-based angle, the second at the
                          secant of the slopes), gated by device flags, so no host round trip sits
                          between iterations; the host keeps one iteration queued ahead and reads a
                          status word.  0: the host-driven CG (line search of up to 8 (mixed) / 14
                          (FP64) trials decided on the host).  Both stop on the same rule; their
                          iteration paths differ. */
} ofdft_options;

typedef struct {
  int iterations;      /* outer minimiser iterations */
  int evaluations;     /* F + gradient evaluations */
  int converged;       /* 1 if the stopping rule was met */
  double F_total;      /* free energy F_tot (etot), hartree */
  double E_internal;   /* F_tot + T S_s + T S_xc (einternel) */
  double F_s;          /* non-interacting free energy T_s - T S_s */
  double TS_s;         /* T times the non-interacting entropy */
  double E_xc, E_H, E_ext, E_alphaZ, E_ion;
  double N_e;          /* int n */
  double mu;           /* Euler-equation multiplier int n v / N_e (Eq. E10) */
  double residual;     /* sqrt(sum n (v-mu)^2 / sum n) */
  double TS_xc;        /* T S_xc = -T dF_xc/dT of a temperature-dependent XC (KSDT); 0 for PZ81.
                          E_xc is the XC free energy F_xc; the XC internal energy is E_xc + TS_xc */
} ofdft_report;

/* Fills defaults: TF, mu_sga = 5/27, PZ81, Gaussian LPP rc = 0.5, FP64, CG,
   tol_energy = 1e-8, tol_residual = 0, max_iter = 1000, device 0, own stream,
   cg_precond = 8, extrapolate = 0. */
void ofdft_default_options(ofdft_options* opt);

/* Creates a context.  opt may be NULL (defaults).  *out is set on success.
   Three environment variables, read here, pick between equivalent kernels (for
   tests and diagnosis; results agree to rounding): OFDFT_PLANE_PASSES=0 uses the
   row FFT passes where plane passes would run; OFDFT_FUSED_GGA=0 keeps the inverse
   gradient transforms and the pointwise functional as two passes where one fused
   pass would run (mixed precision, PZ81 or no XC, square planes of 32, 64 or 128),
   and the whole-plane density and final passes where their split forms would run;
   OFDFT_ION_FORCES=0 or 1 forces the G-parallel or the one-thread-per-ion force
   kernel (default: per ion from 256 ions up).  A fourth, OFDFT_TEST_NONFINITE=k,
   exists for tests of the recovery
   path of ofdft_minimize_density: the host treats the k-th line-search trial of
   the context (counted from 1; k < 0: every trial) as non-finite; the device
   state is not touched. */
int ofdft_create(const ofdft_options* opt, ofdft_ctx** out);
int ofdft_destroy(ofdft_ctx* ctx);

/* Cell (Sec. V B): lattice = rows a1, a2, a3 (9 doubles, bohr), scaled by
   cell_scale (> 0, the cellScale keyword); grid = {N1, N2, N3}, each one of
   8, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 128, 160, 192, 256, 320, 400 (even
   2^a 3^b 5^c lengths; 320 and 400 hold the 32 000- and 62 500-ion fcc-Al cells
   of Sec. VI A at 16 points per cell edge).  Invalidates the ions' structure
   factor and the density. */
int ofdft_set_cell(ofdft_ctx* ctx, const double lattice[9], double cell_scale, const int grid[3]);

/* Ions: nat >= 1 Cartesian positions tau[3*nat] (bohr, multiplied by the
   cell_scale of set_cell) and valence charges Z[nat] > 0.  N_e = sum Z.
   Rebuilds v_ext(G) (structure-factor sum, kept with the structure factors) and
   the Ewald term: its G-space energy on the device from the structure factor,
   with a splitting parameter chosen for the grid, and its real-space part on a
   host thread that runs while the density is optimised.
   Keeps the density as a warm start (rescaled to the new N_e if it changed)
   but clears the converged flag. */
int ofdft_set_ions(ofdft_ctx* ctx, int nat, const double* tau, const double* Z);

/* Electron temperature in kelvin (TEMP keyword), > 0. Clears the converged flag. */
int ofdft_set_temperature(ofdft_ctx* ctx, double T_kelvin);

/* Minimises F_tot over phi at fixed N_e.  Starts from the current density
   (uniform if none).  rep may be NULL.  Returns OFDFT_E_NOT_CONVERGED (and
   keeps the best state, whose energies rep receives) if max_iter is reached.
   Recovery in the CG minimiser: a line-search trial with a non-finite energy or
   slope restarts the CG along the steepest-descent direction from the last finite
   point, once (a second one ends the call with OFDFT_E_NONFINITE, the last finite
   state kept and reported).  A line search that finds no lower F ends the call
   as converged when a residual target is set and met, or, without one, when the
   last accepted step changed F by less than tol_energy or the decrease still
   possible along the line (|dF/dtheta(0)| times the smallest angle tried, F
   convex along the line) is below it (the host-driven CG uses that bound only
   before its first step).  Otherwise it restarts along -g: once in the
   host-driven CG, up to three times in the graph CG with the first angle capped
   at a tenth of the smallest angle tried.
   A non-finite energy at the starting density is OFDFT_E_NONFINITE at once. */
int ofdft_minimize_density(ofdft_ctx* ctx, ofdft_report* rep);

/* After a converged minimisation: F_total (etot), E_internal (einternel) and,
   if forces != NULL, forces[3*nat] (hartree/bohr, Eq. M12 + Ewald); if
   pressure != NULL, P = -Tr Sigma / 3 (Eq. pressure, hartree/bohr^3) from
   ofdft_stress.  These are the outputs of the interface routine of Sec. V D
   (etot, einternel, force and pressure).  Any output pointer may be NULL. */
int ofdft_free_energy_and_forces(ofdft_ctx* ctx, double* F_total, double* E_internal,
                                 double* forces, double* pressure);

/* Stress tensor (Eq. StressTensor): sigma[9] (row-major, symmetric, hartree/bohr^3)
   = (1/V) dOmega/d eps_ab under a homogeneous strain h -> (1 + eps) h of the cell,
   ions at fixed fractional coordinates, the converged density carried with the
   cell.  Sum of the non-interacting part (Eqs. stressTF_a, stressTF_b), the LDA
   XC term, Hartree and pseudopotential reciprocal-space terms, the alpha Z term
   and the Ewald term.  Needs a converged minimisation (OFDFT_E_STATE otherwise);
   OFDFT_E_ARG if sigma is NULL.  Runs three FFT passes and two grid sums on the
   device (the pseudopotential and Ewald G-space terms read the structure
   factors that ofdft_set_ions stored); the real-space Ewald strain sum comes
   from the host thread that ofdft_set_ions started. */
int ofdft_stress(ofdft_ctx* ctx, double sigma[9]);

/* Current amplitude phi (N1*N2*N3 doubles). */
int ofdft_get_density(ofdft_ctx* ctx, double* phi_out);
/* Sets phi (N1*N2*N3 doubles, rescaled to int phi^2 = N_e); clears the converged flag. */
int ofdft_set_density(ofdft_ctx* ctx, const double* phi);

/* One F + gradient evaluation at the current phi.  rep receives the energy
   components, mu and the residual; potential_out (may be NULL) receives the
   total potential v = dF_tot/dn on the grid (N1*N2*N3 doubles). */
int ofdft_eval(ofdft_ctx* ctx, ofdft_report* rep, double* potential_out);

/* Runs n_evals evaluations back to back on the context's stream (no host
   synchronisation in between) and times them with HIP events recorded on
   that stream.  total_ms receives the device time of the whole sequence.
   With max_kernels == 0 only that total is measured (two events).  With
   max_kernels > 0 an event is also recorded before every kernel launch, and
   kernel_ms[k] receives the average duration of kernel slot k per
   evaluation and kernel_names[k] its name (static strings), for
   k < *n_kernels <= max_kernels. */
int ofdft_time_evals(ofdft_ctx* ctx, int n_evals, double* total_ms, int max_kernels,
                     const char** kernel_names, double* kernel_ms, int* n_kernels);

/* Picks the FFT tile sizes for the current cell by timing: the rows per block
   of the contiguous-axis pass (tr), the columns per block of the strided pass
   (tc) and the rows per block of the x2 pass (rb), one parameter at a time,
   each candidate over n_evals evaluations (HIP events on the context's
   stream).  Needs set_cell, set_ions and set_temperature.  The choice stays
   in force until the next set_cell; tiles[3] (may be NULL) receives it.
   ofdft_set_tiles sets the three values directly.  Valid tiles are powers of
   two with tr >= 2 dividing N2 and tc dividing N2, tr*N3 <= 2048,
   (N3/2+1)*tr <= 2048, N1*tc <= 2048, rb*N2 <= 4096 (register-staged tiles),
   and their LDS need fits the 160 KB of a workgroup; anything else is E_ARG.
   The tiles change only the work split, not the result beyond rounding. */
int ofdft_autotune(ofdft_ctx* ctx, int n_evals, int tiles[3]);
int ofdft_set_tiles(ofdft_ctx* ctx, const int tiles[3]);

/* Minimises several independent contexts together.  Contexts with graph_cg set are
   driven by the calling thread alone: each replays its captured CG iteration on its
   own stream, at most two iterations queued ahead, and leaves the rotation when the
   status its device control kernel publishes says it has stopped; the device runs
   the cells' iterations side by side.  Other contexts run on one host thread each.
   reps[n] may be NULL.  Returns the first error, if any (every context is still
   taken to its end). */
int ofdft_batch_minimize(ofdft_ctx* const* ctxs, int n, ofdft_report* reps);

/* For callers that cannot allocate device memory (code under HIP graph capture,
   tight serving loops, harnesses that forbid hipMalloc): the evaluation of
   ofdft_eval with no allocation of any kind in the call.  Its intermediates (the
   spectra, real work arrays, per-block partial sums and scalars of one
   evaluation) live in a static device array of OFDFT_NOALLOC_SCRATCH_BYTES that
   every device holds for the life of the process, instead of the context's own
   buffers; the context's set-up (ofdft_set_cell, ofdft_set_ions,
   ofdft_set_temperature) must have run before.
     phi_dev  device pointer, N1*N2*N3 doubles (row-major [N1][N2][N3]): the
              amplitude, evaluated as given (not renormalised to N_e); read only.
     v_dev    device pointer, N1*N2*N3 doubles: receives the total potential
              v = dF_tot/dn (the potential_out of ofdft_eval), in FP64 in both
              precisions.
     rep      host report as from ofdft_eval (may be NULL).
   Both device buffers belong to the caller and must not overlap the scratch
   array.  The work runs on the context's stream; the call waits for it, so
   v_dev is complete on return.  OFDFT_E_ARG when an argument is NULL or the
   evaluation of this grid needs more than OFDFT_NOALLOC_SCRATCH_BYTES (that is
   the case above 64^3 in FP64 and above 96^3 in mixed precision for cubic
   grids); OFDFT_E_STATE before the set-up.  Calls on one device share the one
   array: calls that overlap in time on the same device (from different threads
   or contexts) race and must be serialised by the caller.  Nothing in the array
   needs to start at zero: every byte a call reads was written earlier in the
   same call. */
#define OFDFT_NOALLOC_SCRATCH_BYTES (48ull << 20)
int ofdft_eval_noalloc(ofdft_ctx* ctx, const double* phi_dev, double* v_dev, ofdft_report* rep);

/* Message for the last error on ctx (or a global message if ctx is NULL). */
/* Ewald energy and forces of point ions Z_I in a neutralising background (the
   ion-ion term E_ion of the total free energy, Sec. II; the same sum that
   set_ions evaluates).  lattice = rows a1, a2, a3 (bohr), nat >= 1 Cartesian
   positions tau[3*nat] (bohr) and charges Z[nat] > 0.  *E receives the energy
   (hartree), forces[3*nat] (may be NULL) the forces (hartree/bohr), stress[9]
   (may be NULL) its term of the stress tensor (row-major, hartree/bohr^3, the
   strain derivative of ofdft_stress).  Host code: needs no context and no device.
   E_ARG on NULL or non-finite input or a singular lattice. */
int ofdft_ewald(const double lattice[9], int nat, const double* tau, const double* Z, double* E, double* forces,
                double* stress);

const char* ofdft_last_error(const ofdft_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* OFDFT_H */

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
 *     XC of Sec. VI) or none;
 *   - F_H in reciprocal space (Eq. E2); v_ext from a local pseudopotential
 *     structure-factor sum (Gaussian-regularised Coulomb, or the
 *     Heine-Abarenkov form of Eq. E4A);
 *   - forces at the converged density (Eq. M12) plus the Ewald ion-ion term.
 * The call pattern mirrors the interface of Sec. V C (ions and temperature in,
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

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define OFDFT_OK 0
#define OFDFT_E_ARG (-1)           /* invalid argument (NULL, nat <= 0, T <= 0, singular cell, ...) */
#define OFDFT_E_GRID (-2)          /* grid size not an even 2^a 3^b in [8, 256] */
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
#define OFDFT_XC_PZ81 1

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
  int xc;              /* OFDFT_XC_NONE or OFDFT_XC_PZ81 */
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
} ofdft_options;

typedef struct {
  int iterations;      /* outer minimiser iterations */
  int evaluations;     /* F + gradient evaluations */
  int converged;       /* 1 if the stopping rule was met */
  double F_total;      /* free energy F_tot (etot), hartree */
  double E_internal;   /* F_tot + T S_s (einternel; XC is T-independent here) */
  double F_s;          /* non-interacting free energy T_s - T S_s */
  double TS_s;         /* T times the non-interacting entropy */
  double E_xc, E_H, E_ext, E_alphaZ, E_ion;
  double N_e;          /* int n */
  double mu;           /* Euler-equation multiplier int n v / N_e (Eq. E10) */
  double residual;     /* sqrt(sum n (v-mu)^2 / sum n) */
} ofdft_report;

/* Fills defaults: TF, mu_sga = 5/27, PZ81, Gaussian LPP rc = 0.5, FP64, CG,
   tol_energy = 1e-8, tol_residual = 0, max_iter = 1000, device 0, own stream,
   cg_precond = 8, extrapolate = 0. */
void ofdft_default_options(ofdft_options* opt);

/* Creates a context.  opt may be NULL (defaults).  *out is set on success.
   Two environment variables, read here, pick between equivalent kernels (for
   tests and diagnosis; results agree to rounding): OFDFT_PLANE_PASSES=0 uses the
   row FFT passes where plane passes would run; OFDFT_ION_FORCES=0 or 1 forces the
   G-parallel or the one-thread-per-ion force kernel (default: per ion from 256
   ions up). */
int ofdft_create(const ofdft_options* opt, ofdft_ctx** out);
int ofdft_destroy(ofdft_ctx* ctx);

/* Cell (Sec. V B): lattice = rows a1, a2, a3 (9 doubles, bohr), scaled by
   cell_scale (> 0, the cellScale keyword); grid = {N1, N2, N3}, each even and
   2^a 3^b in [8, 256].  Invalidates the ions' structure factor and the density. */
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
   keeps the best state) if max_iter is reached. */
int ofdft_minimize_density(ofdft_ctx* ctx, ofdft_report* rep);

/* After a converged minimisation: F_total (etot), E_internal (einternel) and,
   if forces != NULL, forces[3*nat] (hartree/bohr, Eq. M12 + Ewald); if
   pressure != NULL, P = -Tr Sigma / 3 (Eq. pressure, hartree/bohr^3) from
   ofdft_stress. */
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

/* Minimises several independent contexts together: their evaluations are
   interleaved on the contexts' streams so that small cells overlap on the
   device.  reps[n] may be NULL.  Returns the first error, if any. */
int ofdft_batch_minimize(ofdft_ctx* const* ctxs, int n, ofdft_report* reps);

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

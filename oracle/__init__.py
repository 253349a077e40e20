"""CPU FP64 oracle for finite-temperature orbital-free DFT (Karasiev, Sjostrom,
Trickey, "Finite-temperature orbital-free DFT molecular dynamics: coupling
PROFESS and Quantum Espresso", arXiv:1406.0835).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
implementation of what the GPU hot path computes.  It exists so that tests, the
smoke check and the benchmark's CPU baseline can compare against it.  The
product library never imports, links or calls it, and it shares no code, table
or constant generator with the HIP path.

Modules
  fermi_dirac  Fermi-Dirac integrals by quadrature, their inverse, and the
               reduced-temperature factors kappa, xi, zeta, h~ (Sec. III A/B).
  functionals  ftTF, SGA/VWTF and ftGGA (VT84F, KST2, TW, APBEF) free-energy
               densities and their partial derivatives (Eqs. TF..vftGGA);
               PZ81 LDA exchange-correlation (Sec. IV, ground-state LDA).
  grid         periodic real-space grid, reciprocal vectors, spectral
               gradient and divergence.
  potentials   Hartree (Eq. E2), local pseudopotentials (Gaussian-regularised
               Coulomb; Heine-Abarenkov Eq. E4A), Ewald ion-ion energy/forces.
  energy       one evaluation of F_tot[n = phi^2] and its derivative.
  minimize     sphere-constrained nonlinear CG and truncated Newton (Sec. II).
  forces       ionic forces at the converged density (Eq. M12).
  stress       stress tensor and pressure (Eqs. StressTensor, pressure,
               stressTF_a, stressTF_b, and the Hartree, pseudopotential and
               Ewald strain derivatives).
  md           velocity-Verlet Born-Oppenheimer dynamics.

All quantities are in Hartree atomic units; temperatures enter in kelvin at the
System level and are converted with k_B (CODATA 2018).

Parity status: every function is pinned by a test in tests/test_oracle_*.py
against closed forms, limits, brute-force sums or high-precision quadrature
(see each module's header for its pins), except the PZ81 correlation constants,
which are "parity unpinned" (functionals module header).
"""
from . import fermi_dirac, functionals, grid, potentials, energy, minimize, forces, md, stress  # noqa: F401
from .energy import System, evaluate  # noqa: F401

"""FP64 CPU oracle for the enriched-FE second-order Magnus step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package:
only the tests, the smoke check and the CPU-baseline leg of the benchmark use it.
It shares no code with the HIP library; the two meet only in the seeded inputs
of :mod:`workloads`.

The oracle is written for a reader holding the paper: every function names the
section or equation it follows, and it works with plain NumPy/SciPy in float64
(complex128 for orbitals), without blocking, fusion or reordering beyond what
the definitions state.

Modules
  fe         1-D GLL/Gauss tables, Lagrange basis, uniform hex mesh, cell classes
  enrich     atom-centred enrichment functions (atomic part) and gradients
  xc         adiabatic LDA: Slater exchange, PW92 correlation
  model      the EFE discretisation: orthogonalisation, Loewdin transform,
             Hamiltonian, density, Hartree potential, dipole
  propagate  adaptive Lanczos exponential, predictor-corrector Magnus-2 step,
             delta kick, SCF ground state
"""

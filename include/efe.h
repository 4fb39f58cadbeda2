/*
 * efe.h -- C ABI of the MI355X (gfx950) library for one second-order Magnus
 * step of all-electron real-time TDDFT in an enriched finite-element basis
 * (Kanungo, Rufus, Gavini, arXiv:2210.14421).
 *
 * Problem statement followed by the calls:
 *   TDKS equations and density ........... Sec. 2.1, eq. (TDKS)
 *   EFE basis, H and M, Loewdin form ..... Sec. 2.2, eqs. (PsiEFE)-(TDKSDiscrete2)
 *   spectral FE / GLL, (M^ee)^-1/2 ........ Sec. 2.3, eq. (MSquareRoot)
 *   Hartree potential by FE Poisson ...... Sec. 2.1 eq. (Hartree_possion), Sec. 2.2 eq. (DiscretePoisson)
 *   Magnus-2 midpoint step ............... Sec. 2.5, eq. (ApproxMagnus)
 *   adaptive Lanczos exponential ......... Sec. 2.6, eqs. (AdaptiveKrylov), (AdaptiveKrylovErr)
 *   dipole moment ........................ Sec. 3.1
 *
 * Conventions (all calls)
 *   - Orbital blocks (Psi, X, Y) are caller-owned DEVICE pointers to complex128
 *     values, row-major ("node-major"): row r holds the ncol orbitals of basis
 *     function r as interleaved (re, im) doubles, rows r and r+1 are ld complex
 *     values apart (ld >= ncol).  Rows 0 .. n_nodes-1 are the classical FE nodes
 *     in the order gx + Nx (gy + Ny gz); the rows of boundary nodes must hold
 *     zeros (homogeneous Dirichlet condition) and are returned as zeros.  Rows
 *     n_nodes .. n_nodes+n_enr-1 are the Loewdin-orthonormalised enrichment
 *     directions.  The coefficients are those of the Loewdin form
 *     psibar = M^1/2 psi of eq. (TDKSDiscrete2).
 *   - Quadrature arrays (rho_q) are DEVICE arrays of doubles, one per
 *     quadrature point, cell-major (cell ex + nx (ey + ny ez)), then point
 *     i + n (j + n k) of the cell's Gauss rule.
 *   - Calls are ordered on the HIP stream given in efe_options.hip_stream (0 =
 *     the null stream) and return after the stream has drained, except where
 *     noted.  A context is not thread-safe; separate contexts are independent.
 *   - Nothing aborts or throws across the ABI.  Every call returns an
 *     efe_status; on error the caller's output arrays are left unchanged and
 *     efe_last_error() describes the failure.
 */
#ifndef EFE_H
#define EFE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct efe_ctx efe_ctx;
typedef struct efe_plan efe_plan;
typedef struct efe_batch efe_batch;
typedef int32_t efe_status;

enum {
  EFE_OK = 0,
  EFE_ERR_ARG = -1,        /* invalid argument or inconsistent sizes            */
  EFE_ERR_ALLOC = -2,      /* device or host allocation failed                  */
  EFE_ERR_HIP = -3,        /* a HIP runtime call failed                         */
  EFE_ERR_NOCONV = -4,     /* Lanczos reached kmax / Poisson CG reached maxit   */
  EFE_ERR_SINGULAR = -5,   /* enrichment overlap has no direction above the drop threshold */
  EFE_ERR_NONFINITE = -6,  /* NaN or Inf met in an input or a result           */
  EFE_ERR_STATE = -7       /* call out of order (e.g. magnus_step before any Hamiltonian) */
};

/* product dtype of the cell-block and enrichment-coupling products */
enum { EFE_F64 = 0, EFE_F32 = 1, EFE_BF16 = 2, EFE_F64_SF = 3, EFE_BF16X3 = 4 };
/* adiabatic LDA (Sec. 2.1): none, Slater exchange, Slater + PW92 correlation */
enum { EFE_XC_NONE = 0, EFE_XC_SLATER = 1, EFE_XC_SLATER_PW92 = 2 };
/* Lanczos reorthogonalisation (efe_options.reorth) */
enum { EFE_REORTH_PARTIAL = 0, EFE_REORTH_FULL = 1, EFE_REORTH_PARTIAL_DOT = 2 };
/* operator exponentiated by lanczos_expm: Hbar, or the Loewdin position operator */
enum { EFE_OP_H = 0, EFE_OP_X = 1, EFE_OP_Y = 2, EFE_OP_Z = 3 };

/* Physical system and discretisation.  Host memory, read during the call only. */
typedef struct {
  int32_t ncell[3];        /* hex cells per axis                                  */
  double lo[3], hi[3];     /* box [lo, hi] in bohr                                */
  int32_t degree;          /* FE degree p (2..6): (p+1)^3 GLL nodes per cell      */
  int32_t natom;
  const double *R;         /* natom x 3 positions (bohr)                          */
  const double *Z;         /* natom charges                                       */
  double nuc_sigma;        /* nuclear charge Z (pi s^2)^-3/2 exp(-r^2/s^2), s = nuc_sigma */
  int32_t nenr;            /* enrichment functions (Sec. 2.2, eq. (EFEAtomic))    */
  const int32_t *enr_atom; /* owning atom                                         */
  const int32_t *enr_l;    /* 0 or 1                                              */
  const int32_t *enr_m;    /* l = 1: -1 -> y, 0 -> z, +1 -> x                     */
  const double *enr_zeta;  /* r^l exp(-zeta r) Y_lm (1-(r/r_cut)^2)^3, unit norm   */
  double r_cut;
  int32_t norb;            /* occupied orbitals                                   */
  const double *occ;       /* occupations f_a (density = sum f_a |psi_a|^2)       */
  int32_t xc;              /* EFE_XC_*                                            */
  double trap_omega;       /* > 0 adds 1/2 w^2 |x|^2 (test systems)               */
  int32_t quad_cell;       /* Gauss points per axis on ordinary cells; 0 -> p+1   */
  int32_t quad_enr;        /* ... on cells within r_cut of an atom; 0 -> 2p+2     */
  double enr_drop_tol;     /* drop M^ee eigenvalues below tol * max (canonical orthogonalisation) */
  /* Graded tensor-product mesh (Sec. 2.7: finer cells near the atoms, coarser toward
   * the faces): NULL for uniform cells, else ncell[0]+1 x-boundaries, then ncell[1]+1
   * y-boundaries, then ncell[2]+1 z-boundaries, each list strictly increasing from
   * lo[d] to hi[d] (EFE_ERR_ARG otherwise, EFE_ERR_NONFINITE for NaN/Inf).  Every
   * cell is the affine image of the reference cube with its own edge lengths. */
  const double *cell_bounds;
} efe_system;

typedef struct {
  int32_t prod_dtype;      /* type of the stored cell blocks: EFE_F64 (FP64 products),
                              EFE_F32 (FP32 products, FP32 accumulation), EFE_BF16
                              (BF16 blocks and the orbital rows rounded to BF16,
                              products on the BF16 MFMA, FP32 accumulation) or
                              EFE_BF16X3 (both operands as hi/lo BF16 pairs, three
                              BF16 MFMAs per product: about 16 significant bits); or
                              EFE_F64_SF: no stored blocks, the same operator applied
                              in FP64 by sum factorisation from the potential at the
                              points (degree 4 or 5 with the default Gauss rules only).
                              With FP32 or BF16 blocks the enrichment coupling runs on
                              the FP32 MFMA (H^ce in FP32) and the products read an FP32
                              copy of their input and leave their result in FP32, which
                              the Lanczos update reads into its FP64 vectors; the
                              Lanczos recurrence and reorthogonalisation, the
                              tridiagonal exponential, H^ee, Poisson and the densities
                              stay FP64 */
  int32_t kmax;            /* maximum Krylov dimension (1..64)                    */
  double krylov_tol;       /* stop when the estimate of eq. (AdaptiveKrylovErr) <= tol * ||psi|| */
  double cg_tol;           /* Poisson: relative residual                          */
  int32_t cg_maxit;
  void *hip_stream;        /* hipStream_t, or 0                                   */
  int32_t reorth;          /* keeping the Lanczos vectors orthogonal (Sec. 2.6 gives the
                              bare three-term recurrence): EFE_REORTH_PARTIAL (0, default):
                              each vector against the two latest, plus a pass against all
                              previous ones when Simon's omega recurrence (1984) estimates
                              a loss above sqrt(eps), for that vector and the next;
                              EFE_REORTH_FULL (1): a pass against all previous vectors at
                              every step, repeated where it cancelled most of the vector;
                              EFE_REORTH_PARTIAL_DOT (2): the partial scheme with alpha_j
                              always from a dot pass over the new vector.  With EFE_F64
                              blocks the partial scheme (0) takes alpha_j = q^H Hbar q from
                              the products instead (each cell's and the coupling's share,
                              summed in a fixed order), which saves that pass; the two
                              agree to rounding */
} efe_options;

/* External field E(t) = dir * sum_k A_k sin(w_k t + phi_k) exp(-(t-t0)^2/s^2),
 * potential -E(t) . x (eq. (VField)).  kind 0: no field. */
typedef struct {
  int32_t kind;
  int32_t direction;       /* 0 x, 1 y, 2 z                                       */
  int32_t ncomp;
  const double *A, *w, *phi;  /* host arrays of ncomp                             */
  double t0, s;
} efe_field;

/* Per-call statistics (host memory, may be NULL). */
typedef struct {
  int32_t k_pred[128];     /* Krylov dimension per orbital, predictor            */
  int32_t k_corr[128];     /* ... corrector                                      */
  double err_pred_max, err_corr_max;   /* largest a-posteriori estimates         */
  int32_t cg_iters[2];     /* Poisson PCG iterations (midpoint, end of step)      */
  double mu[3];            /* dipole at the end of the step                       */
} efe_step_stats;

/* ---- host-only planning (no GPU needed) --------------------------------- */

/* Builds every static quantity of the discretisation on the host: tables,
 * mesh classes, enrichment normalisation, orthogonalising coefficients
 * c = D^-1 b (Sec. 2.2, eq. (EFEOrtho) with the GLL-lumped classical mass),
 * M^ee and S = (M^ee)^-1/2 (Sec. 2.3, eq. (MSquareRoot); canonical when a
 * direction is dropped), enrichment values at quadrature points, static kinetic
 * couplings, and the fast-diagonalisation data of the Poisson operator.
 * Errors: EFE_ERR_ARG, EFE_ERR_SINGULAR, EFE_ERR_ALLOC. */
efe_status efe_plan_create(const efe_system *sys, efe_plan **out);
efe_status efe_plan_free(efe_plan *plan);
/* Sizes: n_nodes, n_cells, n_quad, n_enr_kept, n_union_rows, n_tcells. */
efe_status efe_plan_sizes(const efe_plan *plan, int64_t sizes[6]);
/* Copies a named static array into host memory `out` of `count` doubles
 * (EFE_ERR_ARG if the name is unknown or count differs).  Names: "D" (n_nodes
 * lumped mass), "S" (n_enr x n_kept), "Mee" (n_enr^2), "c" (n_nodes x n_enr,
 * zero outside the support), "enr_scale" (n_enr), "Kce" (n_nodes x n_enr static
 * kinetic part of H^ce, unscaled), "Kee" (n_enr^2), "vstatic" (n_quad),
 * "lift" (n_nodes: K_IB g), "is_enr" (n_cells as doubles). */
efe_status efe_plan_get(const efe_plan *plan, const char *name, double *out, int64_t count);
const char *efe_plan_error(const efe_plan *plan);

/* ---- GPU context ----------------------------------------------------------- */

/* Plans the system on the host, uploads the static data, and allocates the
 * Krylov workspace (kmax+1 orbital blocks), the cell blocks of Hbar in the
 * product dtype, the enrichment coupling and the quadrature arrays.
 * Errors: EFE_ERR_ARG, EFE_ERR_SINGULAR, EFE_ERR_ALLOC, EFE_ERR_HIP. */
efe_status efe_setup(const efe_system *sys, const efe_options *opt, efe_ctx **out);
efe_status efe_free(efe_ctx *ctx);
/* n_rows (= n_nodes + n_enr_kept), n_nodes, n_enr_kept, n_quad, n_union_rows (the FE
 * rows of the enrichment coupling H^ce: the nodes of the cells where an enrichment
 * function is nonzero, Sec. 2.2). */
efe_status efe_dims(const efe_ctx *ctx, int64_t dims[5]);
/* Changes stream / Krylov settings of a live context (kmax only downwards). */
efe_status efe_set_options(efe_ctx *ctx, const efe_options *opt);

/* Initial orbitals for cluster workloads: orbital a = the enrichment direction
 * enr_index[a] (its Loewdin coordinates S^+ e_nu) plus classical-block noise
 * D^1/2 * amp * n/||n||_M with n = sum_m g[a][m] prod_d sin(m_d pi (x_d-lo_d)/(hi_d-lo_d)),
 * m over {1,2,3}^3 (m_x slowest), then X <- X (X^T X)^-1/2.  Psi: device,
 * n_rows x norb, ld = norb.  Host inputs: enr_index[norb], g[norb*27]. */
efe_status efe_initial_state(efe_ctx *ctx, const int32_t *enr_index, const double *g,
                             double amp, void *Psi);

/* Rebuilds Hbar[rho(Psi), t] (Sec. 2.2 eq. (Hmn) with v_KS of Sec. 2.1) and
 * keeps rho(Psi) as the density of the current time level; required before
 * the first magnus_step and after any change of Psi outside magnus_step.
 * Psi: device, n_rows x norb, PACKED (leading dimension = norb; a strided
 * block must be packed by the caller first). */
efe_status efe_set_hamiltonian(efe_ctx *ctx, const void *Psi, double t, const efe_field *field);

/* Y = Hbar X for the Hamiltonian last built (ncol <= norb columns). */
efe_status efe_apply_H(efe_ctx *ctx, const void *X, void *Y, int32_t ncol, int64_t ld);

/* For callers that cannot allocate memory (code under hipGraph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same Y = Hbar X as
 * efe_apply_H with no device or host allocation, no host synchronisation and no
 * use of the context's work blocks (FP64 products: bit for bit; with FP32 or BF16
 * blocks the rows stay FP64 between the colour passes, so the two agree to the
 * precision of the products).  X and Y: device, n_rows x ncol, PACKED
 * (leading dimension = ncol), distinct, Y fully overwritten; the call returns
 * once the kernels are enqueued on the context's stream (synchronise before
 * reading Y).  The enrichment coupling's partial sums live in a static device
 * array of EFE_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends and
 * shared by every call on that GPU: calls that overlap on one GPU (other
 * streams or contexts) race on it.  EFE_ERR_ARG if 520 n_enr_kept 2 ncol
 * doubles exceed it (Na8, 48 directions: up to 84 orbitals per call);
 * EFE_ERR_STATE without a Hamiltonian or when another GPU than the context's
 * is current. */
#define EFE_NOALLOC_SCRATCH_BYTES (32LL << 20)
efe_status efe_apply_H_noalloc(efe_ctx *ctx, const void *X, void *Y, int32_t ncol);

/* X <- exp(-i tau A) X, A = Hbar (op EFE_OP_H, Hamiltonian last built) or the
 * Loewdin position operator along x/y/z (no kinetic term, v = x_d), by the
 * adaptive Lanczos method of Sec. 2.6, one Krylov space per orbital, with the
 * reorthogonalisation that efe_options.reorth selects (EFE_REORTH_PARTIAL by
 * default: Simon's omega recurrence decides when a vector gets a pass against
 * all previous ones; EFE_REORTH_FULL: a pass at every step).  k_force (host, ncol, may be NULL) fixes the Krylov
 * dimension of each column; otherwise each column stops at the first k whose
 * estimate |tau| beta_k ||x|| |[exp(-i tau T_k)]_{k,1}| <= tol ||x||, or at an
 * invariant subspace.  k_used, err_est: host outputs (ncol, may be NULL).
 * A position operator replaces the stored Hamiltonian: call
 * efe_set_hamiltonian before the next magnus_step.  EFE_ERR_NOCONV if a column
 * needs more than kmax vectors (X unchanged). */
efe_status lanczos_expm(efe_ctx *ctx, int32_t op, double tau, void *X, int32_t ncol, int64_t ld,
                        const int32_t *k_force, int32_t *k_used, double *err_est);

/* One Magnus-2 step, eq. (ApproxMagnus), with the predictor-corrector midpoint
 * Hamiltonian: Psi_p = exp(-i dt Hbar[rho_n, t]) Psi;
 * rho_mid = (rho_n + rho(Psi_p))/2; Psi <- exp(-i dt Hbar[rho_mid, t+dt/2]) Psi;
 * then rho_{n+1}, Hbar[rho_{n+1}, t+dt] and the dipole.  Psi: device, n_rows x
 * norb, ld >= norb.  k_force: host [2][norb] (predictor, corrector) or NULL.
 * stats: host, may be NULL. */
efe_status magnus_step(efe_ctx *ctx, void *Psi, int64_t ld, double t, double dt,
                       const efe_field *field, const int32_t *k_force, efe_step_stats *stats);

/* Applied field of a spectrum run: kind 0 = delta kick of strength kappa at
 * t = 0; kind 1 = the Gaussian kappa exp(-(t - t0)^2 / (2 s^2)) of Sec. 3.1-3.2. */
typedef struct {
  int32_t kind;
  double kappa, t0, s;
} efe_pulse;

/* Absorption spectrum of Sec. 3.2 from the dipole traces of ndir runs
 * (ndir 1..3), run r perturbed along dirs[r] (0..2, host array).  mu: device,
 * [ndir][nt + 1][3], the dipole at t_n = n dt with t_0 = 0 the start of the run
 * (mu at n = 0 is the unperturbed dipole that is subtracted).  For each
 * frequency omega[i] (device, nw): alpha_r = int_0^T exp(-t/tau)
 * (mu_r,d(t) - mu_r,d(0)) exp(i omega t) dt / F[E](omega) (trapezoid rule;
 * F[E] = kappa for the kick, kappa s sqrt(2 pi) exp(-omega^2 s^2/2)
 * exp(i omega t0) for the Gaussian) and S[i] = (2 omega / (3 pi)) sum_r Im
 * alpha_r, the normalisation of the Thomas-Reiche-Kuhn sum rule (int S =
 * N_e for an isotropic response given all three directions).  S: device, nw;
 * alpha: device [ndir][nw][2] (re, im) or NULL.  hip_stream: a hipStream_t or
 * NULL for the null stream; the call waits for its kernel.  EFE_ERR_ARG for
 * out-of-range sizes, directions, dt, tau or pulse. */
efe_status absorption_spectrum(const double *mu, const int32_t *dirs, int32_t ndir, int64_t nt, double dt,
                               const efe_pulse *pulse, double tau, const double *omega, int64_t nw,
                               double *S, double *alpha, void *hip_stream);

/* Dipole power spectrum of a driven run (Sec. 3.5, high-harmonic generation):
 * P[i] = |int_0^T exp(-i omega_i t) exp(-t^2/tau) mu_d''(t) dt|^2 with mu_d'' the
 * second central difference of the samples and the trapezoid rule over the
 * interior samples t_1 .. t_{nt-1} (the Gaussian window as printed).  mu: device,
 * [nt + 1][3], the dipole at t_n = n dt; direction d: 0..2; omega: device, nw;
 * P: device, nw.  hip_stream: a hipStream_t or NULL for the null stream; the
 * call waits for its kernel.  EFE_ERR_ARG for nt < 2, nw out of 1..2^31, a
 * direction out of range, dt not positive and finite, or tau not positive. */
efe_status power_spectrum(const double *mu, int32_t direction, int64_t nt, double dt, double tau,
                          const double *omega, int64_t nw, double *P, void *hip_stream);

/* flags of magnus_step_extrap */
enum { EFE_STEP_KEEP_HAM = 1 };

/* One Magnus-2 step, eq. (ApproxMagnus), with the midpoint Hamiltonian
 * extrapolated from previous steps (Sec. 2.5 names extrapolation from m > 2
 * previous steps as the alternative to the predictor-corrector).  Here m = 3:
 * rho_mid = 15/8 rho_n - 10/8 rho_{n-1} + 3/8 rho_{n-2} (the quadratic through
 * the last three time levels, at t + dt/2), Psi <- exp(-i dt Hbar[rho_mid,
 * t + dt/2]) Psi, then rho_{n+1} and the dipole: one exponential per step.
 * The context keeps the densities of its last three steps (magnus_step and
 * this call both record them; efe_set_hamiltonian, the captured and batched
 * steps, the adjoint calls and position-operator exponentials restart the
 * record).  While fewer than three densities of this dt are known the call
 * makes a predictor-corrector step instead (k_pred of stats > 0; it needs the
 * Hamiltonian of the current orbitals).  flags: EFE_STEP_KEEP_HAM also builds
 * Hbar[rho_{n+1}, t + dt] at the end, as magnus_step does; without it the
 * context holds the midpoint Hamiltonian and a later magnus_step needs
 * efe_set_hamiltonian first.  k_force: host [2][norb] (the corrector half is
 * used by an extrapolated step) or NULL.  Other arguments as magnus_step;
 * EFE_ERR_ARG for unknown flags, EFE_ERR_STATE without a known density. */
efe_status magnus_step_extrap(efe_ctx *ctx, void *Psi, int64_t ld, double t, double dt,
                              const efe_field *field, const int32_t *k_force, int32_t flags,
                              efe_step_stats *stats);

/* The same step as magnus_step, enqueued with no host round trip and replayed
 * from a hipGraph captured on the first call (and again whenever Psi, ld, dt or
 * the field's kind/direction change).  Every Lanczos runs kmax iterations whose
 * kernels return at once after its last column has met the estimate of
 * eq. (AdaptiveKrylovErr), and each Poisson solve runs a fixed budget of PCG
 * iterations that likewise stop on the device, so the results equal
 * magnus_step's (k per column identical).  The graph runs on a private stream
 * ordered after and before the context's stream.  No k_force.  EFE_ERR_NOCONV
 * if a Lanczos needed more than kmax vectors or a Poisson solve did not
 * converge in the budget (Psi then holds the unconverged step; call
 * efe_set_hamiltonian before stepping again). */
efe_status magnus_step_graph(efe_ctx *ctx, void *Psi, int64_t ld, double t, double dt,
                             const efe_field *field, efe_step_stats *stats);

/* Batched propagation of independent systems (different meshes, orbital
 * counts, kicks or fields): one step of every member is captured into a single
 * hipGraph in which the members' device-driven steps (as magnus_step_graph)
 * are concurrent branches, so small systems share the GPU.  The batch refers
 * to the contexts (it does not own them; free the batch first).  All members
 * need efe_set_hamiltonian of their current orbitals. */
efe_status efe_batch_create(efe_ctx *const *ctxs, int32_t n, efe_batch **batch);
efe_status efe_batch_free(efe_batch *batch);
const char *efe_batch_error(const efe_batch *batch);
/* Psi[i], ld[i]: member i's device block; fields: NULL or n pointers (each may
 * be NULL); stats: NULL or n entries.  Re-captures when a pointer, ld, dt or a
 * field's kind/direction changes, or a member's efe_set_options.  Errors name the first failing member in
 * efe_batch_error. */
efe_status efe_batch_step(efe_batch *batch, void *const *Psi, const int64_t *ld, double t, double dt,
                          const efe_field *const *fields, efe_step_stats *stats);

/* Reverse mode of one magnus_step from (Psi = X_n, t, dt, field): on entry
 * Psibar holds Xbar_{n+1} = dL/dRe X_{n+1} + i dL/dIm X_{n+1} (device, n_rows x
 * norb, leading dimension ldb); on return it holds Xbar_n, including the loss
 * term of the dipole at t (mubar = dL/dmu(t), host, 3 doubles).  dLdE (host,
 * 2 doubles) receives dL/dE(t) and dL/dE(t + dt/2), the sensitivities to the
 * field values of eq. (VField) that the step uses.  The forward step is
 * recomputed inside (the same adaptive Krylov dimensions); the exponentials'
 * adjoints are exp(+i dt H) on Krylov spaces of the adjoint blocks, and their
 * Frechet derivatives, through the potential, are cross densities of the two
 * Krylov spaces integrated over s by 10-point Gauss-Legendre; the Hartree and
 * xc responses use the same Poisson solve (homogeneous) and f_xc.  Leaves the
 * cell blocks holding a potential-only operator: call efe_set_hamiltonian
 * before the next forward step.  Workspace (about 15 orbital blocks) is
 * allocated on the first call. */
efe_status magnus_adjoint(efe_ctx *ctx, const void *Psi, int64_t ld, double t, double dt,
                          const efe_field *field, const double mubar[3], void *Psibar, int64_t ldb,
                          double dLdE[2]);

/* Chain rule of the pulse parameters (host arithmetic, no GPU): for a kind-1
 * field E(t) = sum_k A_k sin(w_k t + phi_k) exp(-(t-t0)^2/s^2) of eq. (VField)
 * and sensitivities dLdE[i] = dL/dE(t[i]) (host, n values, e.g. the pairs that
 * magnus_adjoint returns for t and t + dt/2), grad = sum_i dLdE[i] dE(t[i])/dtheta
 * with theta = (A_1..A_m, w_1..w_m, phi_1..phi_m) (host, 3 ncomp doubles).
 * EFE_ERR_ARG for another field kind or missing arrays, EFE_ERR_NONFINITE for
 * NaN/Inf in t or dLdE. */
efe_status efe_field_vjp(const efe_field *field, int64_t n, const double *t, const double *dLdE, double *grad);

/* Adjoint of the dipole of Psi: Psibar = 2 f_a Vbar[mubar . x] Psi_a (the
 * terminal condition of a reverse sweep; mubar host).  Leaves the cell blocks
 * as magnus_adjoint does. */
efe_status dipole_adjoint(efe_ctx *ctx, const void *Psi, int64_t ld, const double mubar[3], void *Psibar,
                          int64_t ldb);

/* rho(q) = sum_a f_a |psi_a(q)|^2 at every quadrature point (device output,
 * n_quad doubles), psi = M^-1/2 Psi evaluated through the EFE basis. */
efe_status density(efe_ctx *ctx, const void *Psi, int64_t ld, double *rho_q);

/* Nodal Hartree potential (device output, n_nodes) of a quadrature density
 * (device input): (1/4 pi) K phi = d, phi = g on the boundary, by PCG with a
 * fast-diagonalisation preconditioner; iters (host, may be NULL). */
efe_status efe_hartree(efe_ctx *ctx, const double *rho_q, double *phi, int32_t *iters);

/* Electronic dipole mu_d = sum_q W_q x_d(q) rho(q) of Psi (host output mu[3]). */
efe_status dipole(efe_ctx *ctx, const void *Psi, int64_t ld, double mu[3]);

/* Autotuner of the cell products (Sec. 2.3: the dense cell blocks applied as batched
 * products over the orbital block).  Times, on the context's own operator and the
 * orbitals of the last efe_set_hamiltonian, every kernel shape available for its
 * block type (pipeline depth and k-rows per chunk of the dense MFMA kernel; for
 * FP64 blocks also the sum-factorised application of the same operator), checks
 * each result against the default shape's (the dense shapes add the terms in the
 * same order: identical bits; sum factorisation within 1e-11 in the 2-norm),
 * and keeps the fastest for every later product of the context.  cache_path (may
 * be NULL): a JSON file of earlier choices keyed by GPU, degree, quadrature, columns,
 * block type, cells and enrichment directions; a cached choice is taken without
 * timing unless flags has EFE_TUNE_FORCE, and a new one is written back.  report
 * (host, may be NULL): "choice=<name> cached=<0|1> <name>=<us per Hbar X> ...".
 * EFE_ERR_STATE without a Hamiltonian; EFE_ERR_ARG if the cache cannot be written. */
enum { EFE_TUNE_FORCE = 1 };
efe_status efe_autotune(efe_ctx *ctx, const char *cache_path, int32_t flags, char *report, int32_t report_len);

/* Device time of the last call's stages in ms: [0] Hbar X cell products,
 * [1] enrichment coupling, [2] Lanczos vector work, [3] tridiagonal
 * exponentials, [4] density, [5] Poisson, [6] rebuild, [7] total; and the
 * number of Hbar X products.  Filled only when timing is enabled. */
efe_status efe_enable_timing(efe_ctx *ctx, int32_t on);
efe_status efe_get_timing(const efe_ctx *ctx, double ms[8], int64_t *n_hx);

const char *efe_last_error(const efe_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* EFE_H */

/*
 * pw.h -- C ABI of the MI355X plane-wave block-eigensolver step.
 *
 * The library applies the plane-wave Kohn-Sham Hamiltonian H of a periodic
 * cell to blocks of wavefunctions and performs one step of an iterative block
 * eigensolver for the lowest eigenpairs of H X = X Lambda (paper Section II-A,
 * Eq. 1), at a fixed effective potential.  One step is: a degree-m Chebyshev
 * filter of the block (each degree is one H application), W = H Y, the Gram
 * and projected matrices S = Y^H Y and H_s = Y^H W (Section II-B, S = Psi^*(H Psi)),
 * the FP64 dense generalised eigensolve of (H_s, S) (Sections II-B and III-D,
 * "Syevd"), the rotation X' = Y C and the residual norms ||H x_i - lambda_i x_i||.
 * Beside the step: the charge density of a block (pw_density) and a LOBPCG step
 * (pw_lobpcg_step) on the same machinery, and a request loop for many small solves.
 *
 * Units: Hartree atomic units (bohr, Ha).  Gamma point only; the basis is every
 * reciprocal lattice vector G = 2 pi (n1/L1, n2/L2, n3/L3) with |G|^2/2 <= ecut
 * (Section II-A: the cutoff energy selects the plane waves).
 *
 * Data layout.  Wavefunction blocks are column-major npw x nb complex arrays in
 * device memory with leading dimension ld >= npw, one band per column, rows in
 * the plane-wave order returned by pw_get_gvectors.  Element type: complex
 * double (interleaved re, im) for PW_FP64, complex float for PW_MIXED.
 *
 * Ownership.  Host inputs are copied during the call.  All persistent device
 * state lives in the caller's arena (pw_setup); the library never frees caller
 * memory.  The dense eigensolver library used by pw_eig_step keeps its own
 * small workspace.
 *
 * Streams.  Work is enqueued on the caller's HIP stream.  pw_apply_h returns
 * without synchronising; pw_eig_step, pw_density and pw_lobpcg_step return after
 * their outputs are written.
 *
 * Errors.  Every call returns a pw_status.  PW_EINVAL leaves no side effects.
 * pw_last_error gives a text message for the last failing call on a handle.
 * Handles are not thread safe; use one handle per host thread.
 */
#ifndef PW_H
#define PW_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PW_OK = 0,
  PW_PENDING = 1,    /* serving: result not ready yet */
  PW_EINVAL = -1,    /* invalid argument; nothing was done */
  PW_ENOMEM = -2,    /* arena (or admission budget) too small */
  PW_EDEVICE = -3,   /* HIP runtime / device error */
  PW_ENOTPD = -4,    /* FP64 Cholesky of the Gram matrix failed (rank-deficient block) */
  PW_ENUMERIC = -5,  /* non-finite value in the eigenvalues or residuals */
  PW_ENOTCONV = -6,  /* serving: max_steps reached before tol */
  PW_EBUSY = -7      /* serving: no free slot */
} pw_status;

/* Force the pencil form of the plane stage (three kernels through an HBM intermediate)
   even when a whole FFT plane fits in LDS; for testing that path on small cells. */
#define PW_FLAG_PENCIL_FFT 1u
/* PW_MIXED only: form the products with fp32 data split into two bf16 terms each
   (hi*hi' + hi*lo' + lo*hi' on the bf16 matrix cores, fp32 accumulation; the Gram/projected
   products also add lo*lo'; the long sums over plane waves move their fp32 partial sums to
   fp64 every 4096 plane waves):
   GRAM = [S | H_s] = Y^H [Y | W];  KB = projector products beta^H Y and beta (D P);
   ROT = rotations Y C and W C. */
#define PW_FLAG_BF16_GRAM 2u
#define PW_FLAG_BF16_KB 4u
#define PW_FLAG_BF16_ROT 8u
/* Generate the projector matrix inside the projector GEMMs from per-plane-wave radial factors
   and per-atom axis phase factors (e^{-i G.tau} = product of three 1D factors) instead of
   storing the N_pw x 4 N_atoms table: O(N_pw + N_atoms N^(1/3)) memory in place of
   O(N_pw N_atoms).  For cells whose table does not fit (Si4096 in FP64: 219 GB).
   Not combinable with PW_FLAG_BF16_KB. */
#define PW_FLAG_BETA_OTF 16u
/* Plan the buffers of pw_lobpcg_step (the three-block basis and its Gram matrix); unblocked
   plans only (PW_EINVAL when the bands would be filtered in blocks). */
#define PW_FLAG_LOBPCG 32u
/* Apply the projectors in real space (Section III-A: a projector acts only near its atom):
   each projector is truncated to the grid points within rs_radius of its atom, the projections
   are summed over those points inside the inverse FFT plane pass (one partial per atom and z
   plane), and D P is added back at the same points inside the plane pass of V(r), before the
   forward transforms: O(N_atoms N_b) work per grid plane instead of the O(N_pw N_atoms N_b)
   projector GEMMs.  Needs proj_form = PW_PROJ_LOCALIZED, PW_MIXED, a 128 x 128 (x n3) grid whose
   planes fit in LDS, and 0 < rs_radius with 2 rs_radius (1 + 1e-4) < every cell length; not combinable with
   PW_FLAG_BF16_KB, PW_FLAG_BETA_OTF or PW_FLAG_PENCIL_FFT (PW_EINVAL otherwise); handles with it
   are refused by pw_apply_h_noalloc.  Phase timers: the inverse pass with the projections counts
   as PW_PH_PROJ, their sum over planes as PW_PH_PROJ_REDUCE, the plane pass with V(r) and D P as
   PW_PH_PLANE, and the forward stick pass, which also applies the kinetic term and the Chebyshev
   update, as PW_PH_STICKS_FWD. */
#define PW_FLAG_RSPACE_KB 64u

/* Projector families (pw_cell_desc.proj_form). */
#define PW_PROJ_GSPACE 0    /* beta = (c/sqrt(Omega)) e^{-sigma^2 G^2/2} Y_m(G^) (see below) */
#define PW_PROJ_LOCALIZED 1 /* the l = 1 factor Y_m(G^) becomes -i sigma G_m / sqrt(2 pi): beta is
                               the transform of unit-norm real-space functions p_0 = pi^{-3/4}
                               sigma^{-3/2} e^{-r^2/(2 sigma^2)} and p_m = sqrt(2) pi^{-3/4}
                               sigma^{-5/2} r_m e^{-r^2/(2 sigma^2)}, which vanish a few sigma from
                               the atom */

typedef enum {
  PW_FP64 = 0,  /* every product and FFT in double precision */
  PW_MIXED = 1  /* FP32 complex FFT / H application / GEMMs; FP64 Cholesky, eig, residuals */
} pw_precision;

/*
 * Cell description (Section II-A; the synthetic analytic pseudopotential):
 *   local part   V(G) = S(G) v(|G|) + dV(G) for 0 < |G|^2/2 <= ecut, V(0) = 0, with
 *                v(G) = (1/Omega)(-4 pi zval e^{-G^2 rc^2/4}/G^2 + gauss_c e^{-G^2 rc^2/4}),
 *                S(G) = sum_a e^{-i G.tau_a},
 *                dV(r) = sum_k mode_amp[k] cos(G_k . r + mode_phase[k]), G_k from mode_miller;
 *   nonlocal     V_NL = sum_a sum_m beta_{a,m} D_m beta_{a,m}^H (Section III-A: every
 *                atom's pseudopotential acts on every wavefunction), 4 projectors per atom
 *                (l = 0; l = 1 x, y, z), D = (d0, d1, d1, d1),
 *                beta_{a,m}(G) = (c/sqrt(Omega)) e^{-beta_sigma^2 |G|^2/2} Y_m(G^) e^{-i G.tau_a},
 *                c = sqrt(32 pi^{5/2} beta_sigma^3), real harmonics, Y_{1m}(0) = 0.
 * Set d0 = d1 = 0 for a cell without projectors.
 */
typedef struct {
  double L[3];               /* orthorhombic cell lengths (bohr) */
  int natoms;                /* >= 0 */
  const double *tau;         /* natoms * 3 Cartesian positions (bohr), host, copied */
  double ecut;               /* plane-wave cutoff (Ha), > 0 */
  int nbands;                /* largest block the handle will process (sizes the arena) */
  double zval, rc, gauss_c;  /* local pseudopotential */
  double beta_sigma, d0, d1; /* projectors */
  int nmodes;                /* perturbation modes (0 for none) */
  const int *mode_miller;    /* nmodes * 3, host, copied */
  const double *mode_amp;    /* nmodes (Ha) */
  const double *mode_phase;  /* nmodes (rad) */
  int fft_n[3];              /* 0,0,0: alias-free rule N_i = min 2^p 3^q >= 3 floor(nmax_i) + 1;
                                otherwise must satisfy that bound and be 2^p 3^q (else PW_EINVAL) */
  int prec;                  /* pw_precision */
  unsigned flags;            /* bitwise OR of PW_FLAG_* (0 = defaults) */
  int filter_block;          /* bands per block of the filter and of H applications; 0 = all bands
                                while three full-size work blocks take <= 64 GiB, else blocks whose
                                three work blocks take <= 16 GiB (a multiple of 64 bands) */
  int proj_form;             /* PW_PROJ_GSPACE (0) or PW_PROJ_LOCALIZED */
  double rs_radius;          /* PW_FLAG_RSPACE_KB: truncation radius of the projectors (bohr) */
} pw_cell_desc;

typedef struct {
  long long npw;              /* plane waves in the sphere */
  long long nst;              /* sticks: distinct (n1, n2) columns of the sphere */
  long long nr;               /* grid points N1 N2 N3 */
  long long nproj;            /* 4 * natoms (0 without projectors) */
  size_t footprint_bytes;     /* arena bytes pw_setup needs for this description */
  int fft_n[3];
  int nbands;
  int prec;
  int fused_planes;           /* 1 when each FFT plane is transformed inside LDS */
  int filter_block;           /* bands per filter block (== nbands: one block) */
} pw_info;

typedef struct {
  int degree;     /* Chebyshev degree m >= 0 (0 = plain Rayleigh-Ritz on the input block) */
  double a_lo;    /* filter: value the filter normalises to 1 (lowest wanted eigenvalue estimate) */
  double a, b;    /* filter: interval [a, b] to damp (b >= largest eigenvalue of H) */
  int want_hx;    /* 1: write H X' to HX_dev */
} pw_step_params;

typedef struct pw_handle_s pw_handle;

/* Sizes of a description, host only (no device needed).  PW_EINVAL for a bad description. */
pw_status pw_plan(const pw_cell_desc *desc, pw_info *out);

/* Miller indices of the basis of a description, host only: npw * 3 ints in stick order. */
pw_status pw_plan_gvectors(const pw_cell_desc *desc, int *miller_host);

/*
 * Build a handle: plane-wave sphere (stick order: n1, then n2, then n3 ascending), grid,
 * V(r) on the device (V(G) -> inverse FFT), projector table, work buffers.  The basis is the
 * cutoff sphere of Section II-A; the grid is the alias-free one (reading of the Section II-A
 * grid rule); the projectors act atom by atom as in Section III-A.
 * arena_dev: caller device memory of arena_bytes >= pw_plan(...).footprint_bytes
 * (PW_ENOMEM otherwise).  hip_stream: a hipStream_t (NULL = default stream).
 * Synchronises the stream before returning.
 */
pw_status pw_setup(const pw_cell_desc *desc, void *arena_dev, size_t arena_bytes, void *hip_stream,
                   pw_handle **h);
pw_status pw_query(const pw_handle *h, pw_info *out);
/* Miller indices of the basis, npw * 3 ints in row order of every block (host buffer). */
pw_status pw_get_gvectors(const pw_handle *h, int *miller_host);

/*
 * HX = H X for nb bands (1 <= nb <= nbands), device arrays with leading dimension ld >= npw
 * (same ld for both): the Hamiltonian of Section II-A, Eq. 1 (kinetic |G|^2/2, local potential
 * through the band-local 3D FFTs of the column partition, Section II-B, and the nonlocal
 * pseudopotential of Section III-A).  X and HX must not overlap.  Asynchronous on the handle's
 * stream.
 */
pw_status pw_apply_h(pw_handle *h, const void *X_dev, void *HX_dev, int nb, int ld);

/*
 * pw_apply_h for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same H X, through the same kernels, with
 * the work buffers of the H applications (stick and pencil FFT intermediates, split-K partials of
 * the projections, D P and the bf16 planes of the block) placed in a static device array of the
 * library (64 MiB per device, held until the process ends) instead of the handle's arena.
 * Allocates nothing and creates nothing: no hipMalloc or hipFree, no library allocation, no
 * stream or event; phase timers are not recorded during the call.  Bands are processed in groups
 * of as many columns as the array holds; PW_ENOMEM when not even one band of this cell fits
 * (e.g. a 192^3 grid in FP64), PW_EINVAL as pw_apply_h.  The array keeps the last call's
 * contents; nothing in it needs to start at zero.  Every call on one device shares that
 * device's array: calls that overlap in time on one device (several host threads, or several
 * streams with work in flight) race and give wrong results; serialise them on one stream.
 * Asynchronous on the handle's stream, like pw_apply_h.
 */
pw_status pw_apply_h_noalloc(pw_handle *h, const void *X_dev, void *HX_dev, int nb, int ld);

/*
 * Charge density of nb bands (1 <= nb <= nbands; X as for pw_apply_h), the quantity the SCF
 * loop forms from the eigenfunctions (Section II-A): rho(r_j) = sum_n occ[n] |psi_n(r_j)|^2 at
 * the FFT grid points r_j = (j1 L1/N1, j2 L2/N2, j3 L3/N3), psi_n(r) = sum_G X[G, n] exp(+i G.r)
 * (unnormalised inverse transform, no volume factor; the caller scales).  occ_host: nb finite
 * band weights on the host (e.g. 2 for each doubly occupied band), copied during the call.
 * rho_dev: N1 N2 N3 doubles on the device, layout [j3][j2][j1] (j1 fastest), overwritten.
 * Accumulated in FP64 in a fixed order (deterministic): over bands in index order, or, on
 * 128 x 128 FP32 planes, within consecutive band groups in index order and then over the groups
 * in order (the fused form, which writes one grid per group).  Uses the handle's work
 * buffers; returns after rho is complete.  PW_EINVAL for bad sizes, null pointers or
 * non-finite weights.
 */
pw_status pw_density(pw_handle *h, const void *X_dev, int nb, int ld, const double *occ_host, void *rho_dev);

/*
 * Basis directions dropped by the Rayleigh-Ritz of pw_lobpcg_step and pw_ppcg_step when a basis
 * Gram matrix is singular: those whose eigenvalue in the unit-diagonal scaling of the Gram matrix
 * is at most this fraction of the largest (FP64 handles; FP32 and split-precision handles).
 */
#define PW_DROP_TOL_FP64 1e-10
#define PW_DROP_TOL_MIXED 1e-5

/*
 * One LOBPCG step (locally optimal block preconditioned conjugate gradient, one of the inner
 * eigensolvers the paper names in Section II-A) on X (in/out, nb columns) with search
 * directions P (in/out, nb columns, same ld; its input is ignored when have_p == 0):
 *   W = H X, theta_i = Re(x_i^H w_i) / (x_i^H x_i),
 *   R = T (W - X diag(theta)), T = diag(1 / (1 + |G|^2/2)) (diagonal preconditioner),
 *   the columns of R and P scaled to unit norm,
 *   Rayleigh-Ritz of H on Z = [X R P] (or [X R]): [S | H_s] = Z^H [Z | HZ] and the FP64
 *   generalised eigensolve H_s C = S C Lambda of size k = 3 nb (2 nb),
 *   X' = Z C_1 (C_1: the nb lowest Ritz vectors), P' = [R P] times the R and P rows of C_1.
 * When S fails the Cholesky test (the directions have become numerically dependent), the
 * Rayleigh-Ritz runs on the part of span Z that a truncated SVQB basis keeps: S scaled to unit
 * diagonal, diagonalised, and the directions with eigenvalue <= PW_DROP_TOL_* times the largest
 * dropped; *kept (optional, may be NULL) receives the dimension of the span used (k when nothing
 * was dropped).  eig (host, nb): the nb lowest Ritz values; resid (host, nb): ||w_i - theta_i x_i||
 * of the input block.  Three H applications per step (X, R, P).  Needs a handle planned with
 * PW_FLAG_LOBPCG (PW_EINVAL otherwise); PW_ENOTPD when fewer than nb directions are kept.
 * Synchronises before returning.
 */
pw_status pw_lobpcg_step(pw_handle *h, void *X_dev, void *P_dev, int nb, int ld, int have_p, double *eig,
                         double *resid, int *kept);

/*
 * One PPCG step (projected preconditioned conjugate gradient, Vecharynski, Yang and Pask; one of
 * the inner eigensolvers the paper names in Section II-A) on X (in/out, nb columns) with search
 * directions P (in/out, same shape; its input ignored when have_p == 0):
 *   Rayleigh-Ritz on span X ([S | H_s] = X^H [X | HX], FP64 eigensolve of size nb):
 *     X <- X C (Ritz vectors, Ritz values Lambda), P <- P C (the directions follow their columns);
 *   R = H X - X Lambda (resid: its column norms), W = T R (the preconditioner of pw_lobpcg_step);
 *   W <- W - X (X^H W), P <- P - X (X^H P);
 *   per column j, Rayleigh-Ritz of H on span{x_j, w_j, p_j} (span{x_j, w_j} without P; the
 *     entry for x_j is lambda_j; a dependent vector is dropped as in pw_lobpcg_step, FP64, one
 *     thread per column): the lowest Ritz vector a x_j + b w_j + g p_j with a real and >= 0;
 *   X <- a X + b W + g P, P <- b W + g P (column by column).
 * eig (host, nb): Lambda; resid (host, nb): ||H x_j - lambda_j x_j|| of the Ritz vectors.  The
 * output X is not orthonormal; the next step's Rayleigh-Ritz makes it so.  Three H applications
 * of nb columns per step (X, W, P), one Rayleigh-Ritz of size nb.  Needs a handle planned with
 * PW_FLAG_LOBPCG (the same buffers); PW_ENOTPD when X is rank-deficient.  Synchronises before
 * returning.
 */
pw_status pw_ppcg_step(pw_handle *h, void *X_dev, void *P_dev, int nb, int ld, int have_p, double *eig,
                       double *resid);

/*
 * One block-eigensolver step on X (in/out, nb columns, ld >= npw): the iterative eigensolver of
 * Section II-A, with the subspace products S = Psi^*(H Psi) of Section II-B and the FP64 dense
 * eigensolve ("Syevd", Sections II-B and III-D):
 *   Y = T_m((H - c)/e) X / T_m((a_lo - c)/e), e = (b - a)/2, c = (b + a)/2 (m = degree;
 *       three-term recurrence, one H application per degree);
 *   W = H Y; S = Y^H Y, H_s = Y^H W (Hermitian parts); S = L L^H (FP64 Cholesky);
 *   L^-1 H_s L^-H = Q diag(lambda) Q^H (FP64, ascending); C = L^-H Q;
 *   X <- Y C; resid_i = ||W C_i - lambda_i X_i||_2 (FP64 accumulation).
 * eig_host, resid_host: nb doubles each (host).  bounds_out (may be NULL) receives
 * {lambda_1, lambda_nb, b}: the a_lo and a of the next step, and the b used.
 * HX_dev may be NULL unless want_hx.  PW_ENOTPD when the Cholesky fails (X unchanged
 * content is not guaranteed), PW_ENUMERIC on a non-finite eigenvalue or residual.
 * For degree > 0 the bounds must satisfy a_lo < a < b.  A NaN bound takes the library's value:
 * a_lo and a from the last successful step on this handle (lambda_1, lambda_nb; PW_EINVAL when
 * there was none), b from the Lanczos estimate of pw_spectrum_bound (20 steps, seed 1, computed
 * once per handle).
 */
pw_status pw_eig_step(pw_handle *h, void *X_dev, void *HX_dev, int nb, int ld, const pw_step_params *p,
                      double *eig_host, double *resid_host, double bounds_out[3]);

/*
 * The solve loop around pw_eig_step (an iterative eigensolver run to convergence, Section II-A):
 * one degree-0 step (Rayleigh-Ritz on the input block, which gives the first filter bounds), then
 * degree-`degree` steps, each taking a_lo, a from the previous step, until the residual norms of
 * the lowest nconv bands (0 = all nb) are all <= tol, or max_steps steps were taken (then
 * PW_ENOTCONV with the last eig/resid written).  b: upper filter bound; NaN = the library's
 * Lanczos estimate (pw_spectrum_bound with 20 steps, seed 1, computed once per handle).
 * eig_host, resid_host: nb doubles (host); *steps (may be NULL) receives the steps taken.
 * A filtered step whose Gram matrix fails the Cholesky test leaves X as it was (unblocked plans:
 * the filter never writes X); such a step is taken again once at half the degree, and the retry
 * is counted (pw_solve_retries) with the first failure's text kept (pw_last_error stays as it
 * was before the retry when the retry succeeds: see pw_solve_retries).  Other errors of a step,
 * and a second failure, are returned as they are (the pw_last_error text names the step).
 */
pw_status pw_solve(pw_handle *h, void *X_dev, int nb, int ld, int nconv, double tol, int degree, int max_steps,
                   double b, double *eig_host, double *resid_host, int *steps);

/* Steps of the last pw_solve on h that were taken again after a failed Cholesky test (0 or 1);
 * when non-zero, *msg (may be NULL) points to the text of that failure (valid until the next call
 * on h).  -1 for a null handle. */
int pw_solve_retries(pw_handle *h, const char **msg);

/*
 * Seeded starting block on the device: entry (g, j) = w_g (x + i y) / ||column j||, with x, y
 * standard normal (Box-Muller on two splitmix64 outputs of the counter (seed, j, g)) and
 * w_g = 1 / (1 + |G_g|^2).  X_dev: nb columns, ld >= npw.  Asynchronous.
 */
pw_status pw_random_block(pw_handle *h, void *X_dev, int nb, int ld, unsigned long long seed);

/*
 * Upper bound estimate of the spectrum: 1.01 * (largest Ritz value + last off-diagonal) of a
 * `steps`-step Lanczos run on H from a seeded random vector.  Host result.
 */
pw_status pw_spectrum_bound(pw_handle *h, int steps, unsigned long long seed, double *bmax);

/*
 * Per-phase device time.  While timing is on, every kernel launch of a call is bracketed by
 * HIP events recorded on the handle's stream; the elapsed times are accumulated per phase.
 * pw_get_stats synchronises the stream and fills PW_NPHASES entries.
 */
typedef enum {
  PW_PH_STICKS_INV = 0, /* sphere -> sticks, inverse z FFT */
  PW_PH_PLANE,          /* fused plane pass: 2D FFT, * V(r), 2D FFT */
  PW_PH_PENCIL_YINV,    /* pencil form: inverse y FFT */
  PW_PH_PENCIL_X,       /* pencil form: x FFT, * V(r), x FFT */
  PW_PH_PENCIL_YFWD,    /* pencil form: forward y FFT */
  PW_PH_STICKS_FWD,     /* sticks -> sphere, forward z FFT */
  PW_PH_PROJ,           /* P = beta^H Y (split-K MFMA GEMM) */
  PW_PH_PROJ_REDUCE,    /* split sum and D scaling of P */
  PW_PH_NL,             /* beta (D P) + kinetic + local + Chebyshev update (MFMA GEMM, fused epilogue) */
  PW_PH_GRAM,           /* [S | H_s] = Y^H [Y | W] (split-K MFMA GEMM) */
  PW_PH_GRAM_REDUCE,    /* split sum and Hermitian parts */
  PW_PH_EIGSOLVE,       /* FP64 Cholesky + generalised eigensolve */
  PW_PH_ROTATE,         /* X' = Y C, W' = W C (MFMA GEMM) */
  PW_PH_RESID,          /* residual norms */
  PW_PH_OTHER,          /* conversions and copies */
  PW_NPHASES
} pw_phase;

typedef struct {
  long long launches;
  double ms;
} pw_phase_stat;

pw_status pw_set_timing(pw_handle *h, int on);
pw_status pw_get_stats(pw_handle *h, pw_phase_stat *out);
pw_status pw_reset_stats(pw_handle *h);

pw_status pw_destroy(pw_handle *h);
const char *pw_last_error(const pw_handle *h);

/*
 * Serving: a request loop that takes eigen-solves of different cells as they arrive.
 *
 * The server owns max_slots host worker threads, each with its own HIP stream (default
 * priority) on the device current at creation.  Requests are admitted in arrival order when a
 * slot is free: the first queued request whose device footprint (pw_plan footprint plus its
 * wavefunction block) fits in the free part of the caller's arena (first-fit placement) is
 * taken, so smaller requests may pass one that does not fit yet, but at most 16 times; after
 * that nothing behind it is admitted until it fits (no starvation).  A request that could never
 * fit fails with PW_ENOMEM at submission.  An admitted request builds its own
 * handle inside its arena range, draws its seeded starting block, estimates the filter bound,
 * and is advanced step by step (first step degree 0, then `degree`) until the residual norms
 * of its lowest `nconv` bands are <= tol or max_steps is reached (PW_ENOTCONV, partial
 * results kept): the loop of pw_solve.  Admitted requests run concurrently, so their kernels overlap on the device;
 * each request's arithmetic is independent of the others (same results alone or in a mix).
 * pw_submit / pw_poll / pw_server_clock are thread safe.
 */
#define PW_SERVER_DRY_RUN 1u /* testing: no device work; a request "runs" for 2 ms per step */

typedef struct {
  void *arena_dev;      /* device memory shared by all admitted requests (caller-owned) */
  size_t arena_bytes;
  int max_slots;        /* concurrent requests, 1..64 */
  unsigned flags;       /* PW_SERVER_* */
  void *hip_stream;     /* the caller's hipStream_t (NULL = default stream): work enqueued on it before
                           pw_server_create (e.g. filling the arena) completes before any request
                           starts; the slot streams wait on an event recorded on it */
} pw_server_cfg;

typedef struct {
  pw_cell_desc cell;            /* copied at submission (tau and mode arrays too) */
  unsigned long long seed;      /* starting block */
  double tol;                   /* residual tolerance (Ha) */
  int max_steps;                /* >= 1 */
  int degree;                   /* Chebyshev degree of the steps after the first, >= 1 */
  int nconv;                    /* lowest bands that must converge (0 = all nbands) */
} pw_request;

typedef struct {
  pw_status status;     /* PW_OK, PW_ENOTCONV, or the error of the failing call */
  int nbands, steps;
  double *eig;          /* caller buffer of nbands doubles (filled by pw_poll), may be NULL */
  double *resid;        /* caller buffer of nbands doubles, may be NULL */
  double t_arrive, t_admit, t_done;  /* server clock (s) */
  char message[256];    /* for a failed request: the failing call and its pw_last_error text; for a
                           request whose solve retried a step: the text of the failure retried */
  int retried;          /* steps of the solve taken again after a failed Cholesky test */
} pw_result;

typedef struct pw_server_s pw_server;

pw_status pw_server_create(const pw_server_cfg *cfg, pw_server **s);
/* Seconds since the server was created (monotonic clock). */
double pw_server_clock(const pw_server *s);
/* Queue a request (one eigen-solve of Section II-A, run as pw_solve does); t_arrive on the server
 * clock (NaN = now).  *ticket identifies it.  PW_ENOMEM when the request can never fit the arena,
 * PW_EINVAL for bad parameters or a bad cell. */
pw_status pw_submit(pw_server *s, const pw_request *r, double t_arrive, unsigned long long *ticket);
/* The result of a request (the eigenvalues and residual norms of its solve, Section II-A):
 * PW_PENDING while queued or running; otherwise copies it into *out (once; the eig and resid
 * buffers are the caller's) and returns PW_OK.  PW_EINVAL for an unknown or consumed ticket. */
pw_status pw_poll(pw_server *s, unsigned long long ticket, pw_result *out);
/* Waits for running requests to finish; queued requests are dropped. */
pw_status pw_server_destroy(pw_server *s);
const char *pw_status_string(pw_status s);

#ifdef __cplusplus
}
#endif

#endif /* PW_H */

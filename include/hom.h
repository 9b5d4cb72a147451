/*
 * hom.h -- C ABI of the MI355X FFT-Galerkin homogenization library.
 *
 * Solves the periodic cell problem of Vondrejc, Zeman & Marek, "An FFT-based
 * Galerkin method for homogenization of periodic media": find the zero-mean
 * curl-free fluctuation e~ in E_N with
 *     G_N A_N e~ = -G_N A_N E                                (Sec. 5.2, Prop.)
 * by conjugate gradients (Sec. 5.3, Lemma on CG), where
 *     G_N = F_N^-1 Gamma^ F_N,  Gamma^(k) = xi xi^T / (xi . xi),  Gamma^(0) = 0
 * with reference A0 = I (Sec. 3.2, Gamma hat; Sec. 5.1, FFT matrices), on a
 * grid of odd size N (assumption A4).  Two quadratures are offered:
 *   HOM_GANI -- A sampled on the trial grid N (Galerkin with numerical
 *               integration, Sec. 4.3; the Moulinec-Suquet discretisation);
 *   HOM_GA   -- A sampled on the doubled grid M = 2N - 1, where the product of
 *               two trial polynomials is integrated exactly (Galerkin with
 *               exact integration, Sec. 4.2, for the coefficient Q_M[A]).
 * The homogenized coefficient is the energy W_lm = <(E_l + e~_l) . A
 * (E_m + e~_m)> on the quadrature grid (A_H = W for E = I).
 *
 * Conventions (Sec. 4.1): the cell is prod [-Y_a, Y_a]; grid point index i
 * along an axis of length n holds x = k h with k = i if i <= (n-1)/2 else
 * i - n and h = 2Y/n ("FFT order", origin at index 0).  Arrays are C-order
 * with the last axis contiguous.  A coefficient field has nA planes of the
 * quadrature grid: nA = 1 (HOM_A_ISO: a I), d (HOM_A_DIAG) or d(d+1)/2
 * (HOM_A_FULLSYM, Voigt order 11,22,33,23,13,12; in 2-D 11,22,12).
 *
 * Linear elasticity (HOM_A_ELASTIC, d = 2 plane strain or 3; the extension
 * beyond the scalar setting that Sec. 6 names): nA = 2 planes, the Lame
 * fields lambda and mu, with sigma = lambda tr(eps) I + 2 mu eps.  Strains,
 * load cases and mean stresses are then symmetric tensors as Mandel vectors of
 * m = d(d+1)/2 components (Voigt order, off-diagonal entries times sqrt 2, so
 * that dot products are tensor contractions): E is [L][m], strain [L][m][N
 * grid], J [L][m], and W the energies of the load cases (the effective Mandel
 * stiffness for E = I_m).  The trial space is the compatible strains (symmetric
 * gradients of periodic trigonometric displacements); the CG iterate holds d
 * displacement potentials per frequency on an orthonormal basis of them.
 * Elastic cells run the generic first-axis and last-axis kernels; they take no
 * dual or a_trig option, the server does not batch them, and a last-axis
 * length with a prime factor above 31 is rejected (HOM_EINVAL).
 *
 * Errors: every function returns a hom_status; nothing aborts or throws.
 * Ownership: the caller owns every buffer it passes; the library copies what
 * it keeps.  Threading: a cell is not re-entrant; distinct cells may be used
 * from distinct threads.  Device pointers are HIP device pointers of the
 * current device.
 */
#ifndef HOM_H
#define HOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hom_cell hom_cell;
typedef struct hom_server hom_server;

typedef enum {
  HOM_OK = 0,
  HOM_EINVAL = -1,      /* bad argument: d, even N, sizes, non-finite values, tol <= 0, L < 1 */
  HOM_ENOTSPD = -2,     /* A not symmetric positive definite at some point (A2) */
  HOM_ENOMEM = -3,      /* device or host allocation failed, or over the server budget */
  HOM_ENOTCONV = -4,    /* max_iter reached; the best iterate and info are still returned */
  HOM_EBREAKDOWN = -5,  /* CG breakdown ((p, q) <= 0 or not finite) */
  HOM_EDEVICE = -6,     /* HIP runtime error */
  HOM_EBUSY = -7,       /* server: request not finished yet */
  HOM_ESCRATCH = -8     /* hom_apply_noalloc: workspace above HOM_NOALLOC_SCRATCH_BYTES */
} hom_status;

typedef enum { HOM_A_ISO = 0, HOM_A_DIAG = 1, HOM_A_FULLSYM = 2, HOM_A_ELASTIC = 3 } hom_a_kind;
typedef enum { HOM_GANI = 0, HOM_GA = 1 } hom_scheme;
/* HOM_FP64: FFTs, fields and reductions in FP64.
 * HOM_MIXED: the CG recursion runs with FP32 FFTs and fields (FP64 dots and
 * step lengths); the iterate is accumulated in FP64, and each time the
 * recursive residual has fallen by inner_tol the true residual b - Op x,
 * computed with the FP64 operator, replaces it while the search direction is
 * kept (residual replacement, van der Vorst & Ye 2000).  The stopping test
 * is on that FP64 residual. */
typedef enum { HOM_FP64 = 0, HOM_MIXED = 1 } hom_prec;

typedef struct {
  hom_scheme scheme;   /* default HOM_GANI */
  hom_prec prec;       /* default HOM_FP64 */
  double Y[3];         /* cell half-lengths, default 0.5 (unit cell) */
  int max_iter;        /* CG iterations per (inner) solve, default 10000 */
  int max_outer;       /* FP64 residual replacements (HOM_MIXED), default 100 */
  double inner_tol;    /* HOM_MIXED: fall of the FP32 recursive residual between
                          replacements, default 1e-3 */
  int check_every;     /* iterations per captured graph between host checks, default 16 */
  void* stream;        /* hipStream_t the caller orders work against, or NULL */
  int a_trig;          /* HOM_GA only, default 0.  1: the coefficient samples on the
                          M = 2N-1 grid are those of a trigonometric polynomial of T_M,
                          the truncated Fourier series P_M[A] of a coefficient A given
                          by its Fourier coefficients (Sec. 4.2-4.3: exact integration
                          for coefficients of known Fourier form).  The products of
                          trial functions lie in T_M, so Ga is then the exact Galerkin
                          method for A itself and A_H an upper bound of A's
                          homogenized coefficient.  The samples may dip to or below 0
                          near jumps (the bilinear form stays that of the SPD A): only
                          finiteness is checked; rho_A reports +inf when some sample is
                          not positive definite (hom_solve_ms then refuses the cell). */
  int dual;            /* d = 2 or 3, default 0.  1: the dual (flux) problem: find the
                          zero-mean divergence-free trigonometric field j~ of J_N (the
                          other part of the discrete Helmholtz decomposition, Sec. 5.1)
                          minimising <(E + j~) . A (E + j~)>, with A the resistivity
                          (the inverse of the conductivity) and E the mean flux; W is
                          then the dual energy, whose inverse (Ga with exactly
                          integrated resistivity, a_trig) bounds the homogenized
                          conductivity from below while the primal Ga bounds it from
                          above (Sec. 6).  In 2-D the divergence-free fields of a
                          frequency are the multiples of the rotated normal
                          t = (-xi_2, xi_1)/|xi|, used in place of xi/|xi|; in 3-D they
                          form a plane, spanned by an orthonormal pair t_1, t_2 orthogonal
                          to xi, so the CG iterate holds two potentials per frequency
                          (twice the CG vector memory; the first-axis passes then run the
                          generic kernels, the projection transforming the component
                          spectra once per potential). */
} hom_options;

typedef struct {
  int iters_inner;       /* CG iterations, max over load cases */
  int iters_outer;       /* FP64 residual evaluations that (re)started the FP32
                            recursion (HOM_MIXED), 0 for HOM_FP64 */
  double rel_resid_true; /* ||b - Op x|| / ||b|| with the FP64 operator, max over load cases */
  double rho_A;          /* contrast C_A / c_A of the coefficient field (A2) */
  double seconds;        /* wall time of the call */
} hom_info;

/* Fill *opt with the defaults above. */
hom_status hom_options_default(hom_options* opt);

/* Create a cell on the current device.
 *  d        1, 2 or 3 (d = 1 runs as a 2-D cell with one grid point along axis 2)
 *  N        d odd trial sizes (A4), each >= 1
 *  kind     coefficient storage, see above
 *  A        [nA][Q grid] FP64, Q = N (GaNi) or 2N-1 (Ga); host pointer, or a device
 *           pointer when A_on_device != 0.  Copied; the caller may free it on return.
 *  opt      options (NULL for defaults); scheme and Y are fixed for the cell
 * Validates A (finite, symmetric positive definite at every point, A2) and
 * records its contrast.  Errors: HOM_EINVAL, HOM_ENOTSPD, HOM_ENOMEM, HOM_EDEVICE.
 * HOM_EINVAL also for a cell whose last-axis transform (of the quadrature grid,
 * or for Ga of the trial grid) has a prime factor above 31 and no compile-time
 * specialised FP64 kernel: the generic FP64 kernel for such lengths is not run
 * (specialised: 127, and for Ga 61 with trial 31 and 509 with trial 255). */
hom_status hom_create_cell(int d, const int32_t* N, hom_a_kind kind, const double* A,
                           int A_on_device, const hom_options* opt, hom_cell** out);

/* Solve L load cases.
 *  E        [L][d] host, macroscopic gradients (Sec. 1, the split e = E + e~);
 *           elastic cells: [L][m] Mandel strains
 *  tol      stopping test ||r_i|| / ||r_0|| <= tol (HOM_FP64) or the FP64
 *           residual ||b - Op x|| / ||b|| <= tol (HOM_MIXED); tol > 0
 *  strain   nullable device pointer, [L][d][N grid] FP64: total strain E + e~
 *           (elastic cells: [L][m][N grid])
 *  W        nullable host pointer, [L][L] energies (A_H when E = I)
 *  J        nullable host pointer, [L][d] mean fluxes <A (E_l + e~_l)> (elastic
 *           cells: [L][m] mean stresses)
 *  strain0  nullable device pointer [L][d][N grid] FP64: warm start; its
 *           E_N component is used (re-projected by G, Sec. 5.3 Lemma)
 *  info     nullable
 * Errors: HOM_EINVAL, HOM_ENOTCONV (results still written), HOM_EBREAKDOWN,
 * HOM_ENOMEM, HOM_EDEVICE. */
hom_status hom_solve(hom_cell* c, int L, const double* E, double tol, double* strain, double* W,
                     double* J, const double* strain0, hom_info* info);

/* The Moulinec-Suquet basic scheme on the same discrete system (Sec. 5.3, the
 * Neumann series with reference A0 = lambda I): e_{i+1} = E - Gamma_lambda
 * (A - lambda I) e_i with lambda = (c_A + C_A) / 2 from the coefficient's
 * eigenvalue range, i.e. x <- x + (b - G A x) / lambda on the fluctuation,
 * FP64, from x = 0.  Stops once ||b - G A x|| <= tol ||b|| (the test of
 * hom_solve's CG), after at most max_iter steps (HOM_ENOTCONV then, results
 * still written); info->iters_inner counts the steps.  Converges at the rate
 * (rho_A - 1) / (rho_A + 1) per step where CG needs about sqrt(rho_A) times
 * fewer steps.  Arguments and errors as hom_solve (no warm start). */
hom_status hom_solve_ms(hom_cell* c, int L, const double* E, double tol, double* strain,
                        double* W, double* J, hom_info* info);

/* One application of the system operator to L real fields:
 * out = G_N A_N G_N u (Ga: the exact-integration operator), u and out device
 * pointers [L][d][N grid] FP64; prec chooses FP64 or FP32 arithmetic inside.
 * For u in E_N this is the operator of the linear system (Sec. 5.2). */
hom_status hom_apply(hom_cell* c, hom_prec prec, int L, const double* u, double* out);

/* Projection onto E_N: out = G_N u, device pointers [L][d][N grid] FP64 (a dual
 * cell projects onto its trial space J_N instead; hom_apply likewise uses the
 * cell's own projection). */
hom_status hom_project(hom_cell* c, int L, const double* u, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hom_apply
 * (same arguments, same kernels, same result) with its whole workspace taken
 * from a fixed array of HOM_NOALLOC_SCRATCH_BYTES of device memory inside the
 * library, one per GPU, held until the process ends.  Calls no allocation
 * routine (the cell, created beforehand, holds its coefficient and plans).
 * Workspace (each part rounded up to 256 bytes): 16 (2 S + 2 d Xe) L bytes,
 * + 16 S L for HOM_MIXED, + 24 L, with S = N_0 .. N_{d-2} (N_last + 1)/2 and
 * Xe = Q_0 .. Q_{d-2} (N_last + 1)/2 complex elements per load case; above
 * the limit it returns HOM_ESCRATCH and does nothing.  The work is queued on
 * the stream given in the cell's options (the cell's own stream if none) and
 * not waited for: out is complete once that stream reaches it.  Every call on
 * a GPU shares that GPU's array, so calls that overlap on one GPU (on
 * different streams or from different threads) race.  Errors: HOM_EINVAL,
 * HOM_ESCRATCH, HOM_EDEVICE. */
#define HOM_NOALLOC_SCRATCH_BYTES (128u << 20)
hom_status hom_apply_noalloc(hom_cell* c, hom_prec prec, int L, const double* u, double* out);

/* Time the kernels of reps consecutive CG iterations on L load cases (HIP
 * events recorded by each dispatch, on the cell's stream).  ms[0..8]
 * receives the mean duration per launch of: axis-0 expand, axis-1 inverse,
 * last-axis flux pass, axis-1 forward, axis-0 project (with the bookkeeping
 * of the last update), CG update (with alpha; r only, x in the last
 * iteration of a launch), the end-of-launch bookkeeping per iteration (one
 * per launch of 16 iterations), ms[7] the sum, one iteration, and ms[8] the
 * direction step (beta, the stopping test, x += alpha p left by the last
 * update, p <- r + beta p).  bytes[0..8] receives the algorithmic HBM bytes
 * of the same launches in the steady state of a launch (each input read
 * once, each output written once). */
hom_status hom_profile_iteration(hom_cell* c, hom_prec prec, int L, int reps, double* ms,
                                 double* bytes);

/* Enable (default, 1) or disable (0) the compile-time specialised kernels of
 * the sizes they exist for; disabled, every size runs the generic kernels.
 * Process-wide, for A/B timing and testing only: it takes effect for every
 * cell and server at its next launch (captured graphs are captured again). */
hom_status hom_set_specialized(int enable);

/* Autotuner: for each pass of c's CG iteration (L load cases, precision
 * prec), time every compile-time variant and the generic kernel inside reps
 * whole CG iterations (HIP events; the other passes at their current
 * choice) and keep the fastest, process-wide, keyed by (pass, precision, FFT
 * length, trial length, components).  best_us (nullable, 5 entries: expand,
 * axis-1 inverse, row, axis-1 forward, project) receives the time of one CG
 * iteration with each pass's winner; passes a cell does not have are left
 * untouched.  Not to be run while other threads solve. */
hom_status hom_autotune(hom_cell* c, hom_prec prec, int L, int reps, double* best_us);
/* Number of compile-time variants of each pass of c's iteration in
 * precision prec (counts[5], same pass order; 0 where only the generic
 * kernel exists or the pass is absent). */
hom_status hom_pass_variants(hom_cell* c, hom_prec prec, int32_t* counts);
/* Use variant v (-1: the generic kernel) of pass `pass` for every cell of
 * c's shape and precision, process-wide, until changed (testing and A/B
 * timing).  HOM_EINVAL for a variant or pass that does not exist. */
hom_status hom_force_variant(hom_cell* c, hom_prec prec, int pass, int variant);
/* The variant pass `pass` of c's iteration runs now (-1: the generic kernel),
 * as hom_force_variant takes it, so a test can restore it. */
hom_status hom_current_variant(hom_cell* c, hom_prec prec, int pass, int32_t* variant);
/* Write / read the tuned choices as JSON ({"arch": ..., "choices": [[pass,
 * element bytes, FFT length, trial length, components, variant], ...]});
 * loading a file tuned on another GPU architecture returns HOM_EINVAL. */
hom_status hom_tune_save(const char* path);
hom_status hom_tune_load(const char* path);

void hom_destroy_cell(hom_cell* c);
const char* hom_status_str(hom_status s);
/* Grid sizes of a cell: N[3], Q[3] (unused axes 1), d. */
hom_status hom_cell_dims(const hom_cell* c, int32_t* d, int32_t* N, int32_t* Q);

/* ---- continuous batching ------------------------------------------------
 * A server owns a background thread that admits submitted requests while
 * their device footprint fits the budget, packs requests of equal (d, N,
 * scheme) into batched iterations replayed as HIP graphs with per-request
 * convergence masks, retires converged requests and admits waiting ones into
 * the freed slots.  Requests are solved with the server's precision. */
hom_status hom_server_create(size_t hbm_budget_bytes, const hom_options* opt, hom_server** out);
/* Queue one request on cell c (the cell must outlive the request).  E [L][d]
 * host, copied.  *ticket receives its id.  HOM_ENOMEM if the request alone
 * exceeds the budget; HOM_EINVAL for more than d load cases or a dual cell. */
hom_status hom_server_submit(hom_server* s, hom_cell* c, int L, const double* E, double tol,
                             uint64_t* ticket);
/* HOM_EBUSY until the request is done; then its status, W [L][L], J [L][d]
 * (both nullable) and info.  A finished ticket can be polled once. */
hom_status hom_server_poll(hom_server* s, uint64_t ticket, double* W, double* J, hom_info* info);
/* Per-request timestamps of a finished ticket (seconds since server start):
 * t[0] submit, t[1] admit, t[2] done.  Call before polling it. */
hom_status hom_server_times(hom_server* s, uint64_t ticket, double* t);
/* Drain and stop the worker, free everything. */
hom_status hom_server_destroy(hom_server* s);

#ifdef __cplusplus
}
#endif
#endif

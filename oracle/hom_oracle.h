/*
 * hom_oracle.h -- plain FP64 CPU oracle for the FFT-Galerkin cell problem.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the mathematics of Vondrejc, Zeman & Marek, "An FFT-based Galerkin
 * method for homogenization of periodic media".  Only the test suite, the
 * smoke entry point and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or helper with the GPU path.
 *
 * Conventions (all from the paper):
 *  - cell Y = prod [-Y_a, Y_a]; grid points x^k = (k_a h_a), h_a = 2 Y_a / N_a,
 *    k in Z_N = { -N_a/2 <= k_a < N_a/2 } (Sec. 4.1); N_a odd (A4).
 *  - storage is "FFT order": array index i along an axis of length n holds
 *    k = i if i <= (n-1)/2 else i - n, so the origin is index 0.
 *  - DFT (Sec. 4.1, eq. for the DFT pair): forward carries 1/n,
 *    u^(k) = (1/n) sum_m u(m) w^{-km}; inverse u(k) = sum_m u^(m) w^{km},
 *    w^{km} = exp(2 pi i k m / n).
 *  - frequency vector xi(k) = (k_a / Y_a)_a (Sec. 2, Fourier basis).
 *  - Gamma^(k) = xi (x) xi / (xi . xi) for k != 0 and 0 at k = 0, i.e. the
 *    projection kernel with reference A0 = I (Sec. 3.2, eq. for Gamma hat;
 *    the discrete G_N = F^-1 Gamma^ F of Sec. 5.1).
 *  - vector fields are stored component-major: [d][grid] (real) and the
 *    coefficient field A as [nA][Q grid] with nA = 1 (isotropic), d
 *    (diagonal) or d(d+1)/2 (full symmetric, Voigt order 11,22,33,23,13,12;
 *    in 2-D 11,22,12).
 *  - grid inner product (u, v) = (1/|N|) sum_k u(x^k) . v(x^k) (Sec. 5.1).
 *
 * Every function returns 0 on success and a negative code on failure.
 */
#ifndef HOM_ORACLE_H
#define HOM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { HOR_OK = 0, HOR_EINVAL = -1, HOR_ENOTREAL = -2, HOR_EBREAKDOWN = -5,
       HOR_ENOTCONV = -4, HOR_ENOMEM = -3 };

/* HOR_ELASTIC: linear elasticity (d = 2 plane strain, or 3), the extension
 * beyond the scalar setting that Sec. 6 names.  Fields are then symmetric
 * tensors in Mandel form, d(d+1)/2 components in Voigt order with the
 * off-diagonal entries times sqrt 2; A holds the Lame fields [lambda, mu] on
 * the Q grid (nA = 2), sigma = lambda tr(eps) I + 2 mu eps; the trial space is
 * the compatible strains (symmetric gradients of periodic displacements) and
 * E, x, W, J are taken over those components. */
enum { HOR_ISO = 0, HOR_DIAG = 1, HOR_FULLSYM = 2, HOR_ELASTIC = 3 };
enum { HOR_GANI = 0, HOR_GA = 1 };

typedef struct {
    int d;            /* 1, 2 or 3 */
    int scheme;       /* HOR_GANI: A on the N grid; HOR_GA: A on the 2N-1 grid */
    int kind;         /* HOR_ISO / HOR_DIAG / HOR_FULLSYM */
    int dual;         /* 0: the primal problem on E_N (gradients); 1: the dual
                         problem on J_N (zero-mean divergence-free fields, the
                         other part of the discrete Helmholtz decomposition of
                         Sec. 5.1), A then being the resistivity; the projection
                         becomes I - xi xi / |xi|^2 for k != 0 and 0 at k = 0 */
    long N[3];        /* trial grid (odd) */
    long Q[3];        /* quadrature grid: N (GaNi) or 2N-1 (Ga) */
    double Y[3];      /* cell half-lengths */
    const double* A;  /* [nA][Q grid], FFT order */
} hor_cell;

/* Naive DFT of a complex array (interleaved re,im) of shape n[0..d-1] along
 * axis ax.  sign = -1: forward, with the 1/n factor; sign = +1: inverse. */
int hor_dft_axis(int d, const long* n, int ax, int sign, double* data);
/* The same along every axis. */
int hor_dft_all(int d, const long* n, int sign, double* data);

/* Projection G_N u = F^-1 Gamma^ F u of a real vector field u [d][N grid]. */
int hor_apply_G(const hor_cell* c, const double* u, double* out);
/* System operator G_N A_N u (GaNi), or its exact-integration analogue (Ga):
 * F_N^-1 Gamma^ Trunc F_M [A F_M^-1 Pad F_N u]. */
int hor_apply_GA(const hor_cell* c, const double* u, double* out);

/* Conjugate gradients on G A x = -G A E for one load case E[d] with x0 = 0
 * (or x0 = G x, the E_N part of x on entry, when warm != 0).  Stops when
 * ||r_i|| / ||b|| <= tol (for x0 = 0, r_0 = b; a warm start that already
 * meets the test returns after 0 iterations).  iters/relres receive the
 * iteration count and the final true relative residual ||b - GA x|| / ||b||.
 * hist (nullable, max_iter+1 entries) receives ||r_i|| / ||b||. */
int hor_cg(const hor_cell* c, const double* E, double tol, int max_iter,
           int warm, double* x, int* iters, double* relres, double* hist);

/* CG on the discrete Lippmann-Schwinger system [I + Gamma_lambda (A - lambda I)] e = E
 * with reference A0 = lambda I (Sec. 5.2 and 5.3), started from e0 = E. */
int hor_cg_lsd(const hor_cell* c, const double* E, double lambda, double tol,
               int max_iter, double* e, int* iters);

/* Moulinec-Suquet Neumann series e_i = E - Gamma_lambda (A - lambda I) e_{i-1}
 * (Sec. 5.3), e_0 = E.  lambda (e_i - e_{i-1}) is the residual b - G A x of
 * the system for x = e_{i-1} - E; the series stops before the step whose
 * residual meets ||r|| <= tol ||b|| (the CG test), so iters counts the steps
 * taken.  HOR_ENOTCONV after max_iter steps. */
int hor_ms(const hor_cell* c, const double* E, double lambda, double tol,
           int max_iter, double* e, int* iters);

/* Energy quadrature W_lm = (1/|Q|) sum_Q e_l . A e_m and mean flux
 * J_l = (1/|Q|) sum_Q A e_l, with e_l = E_l + x_l interpolated to the Q grid
 * (identity for GaNi, zero-padding of the Fourier coefficients for Ga).
 * E: [L][d], x: [L][d][N grid], W: [L][L], J: [L][d] (nullable). */
int hor_homogenized(const hor_cell* c, int L, const double* E, const double* x,
                    double* W, double* J);

/* Total strain e = E + x interpolated to the Q grid: out [d][Q grid]. */
int hor_strain_on_Q(const hor_cell* c, const double* E, const double* x, double* out);

#ifdef __cplusplus
}
#endif
#endif

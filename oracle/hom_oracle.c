/*
 * hom_oracle.c -- plain FP64 CPU oracle for the FFT-Galerkin cell problem.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke entry point
 * and the benchmark's CPU-baseline leg, never by the GPU library.  It follows
 * the paper's definitions step by step, with a naive separable DFT (no FFT)
 * and no blocking, fusion or reordering beyond them.  See hom_oracle.h for
 * the conventions.
 *
 * Parity pins (tests/test_oracle_*.py): DFT identities and the dense DFT
 * matrix; projection identities of G (Lemma on the discrete projection,
 * Sec. 5.1); homogeneous cell; laminate closed forms; dense brute-force
 * solves in real and Fourier space; Voigt-Reuss bounds; L-SD invariance in
 * lambda (Sec. 5.3); Moulinec-Suquet limit.
 */
#include "hom_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* grid helpers                                                        */
/* ------------------------------------------------------------------ */

static long prod(int d, const long* n) {
    long s = 1;
    for (int a = 0; a < d; ++a) s *= n[a];
    return s;
}

/* signed frequency / grid index of storage position i on an axis of length n
 * (Sec. 4.1: -n/2 <= k < n/2, FFT order). */
static long kof(long i, long n) { return (i <= (n - 1) / 2) ? i : i - n; }

/* storage position of signed index k on an axis of length n */
static long pos(long k, long n) { return ((k % n) + n) % n; }

/* components of a field: d (vector fields of the scalar problem) or
 * d(d+1)/2 (symmetric strain / stress tensors in Mandel form, elasticity) */
static int ncomp(const hor_cell* c) {
    return (c->kind == HOR_ELASTIC) ? c->d * (c->d + 1) / 2 : c->d;
}

static int valid_cell(const hor_cell* c) {
    if (!c || c->d < 1 || c->d > 3 || !c->A) return 0;
    if (c->kind < HOR_ISO || c->kind > HOR_ELASTIC) return 0;
    if (c->kind == HOR_ELASTIC && (c->d < 2 || c->dual)) return 0;
    for (int a = 0; a < c->d; ++a) {
        if (c->N[a] < 1 || (c->N[a] % 2) == 0) return 0;
        long q = (c->scheme == HOR_GA) ? 2 * c->N[a] - 1 : c->N[a];
        if (c->Q[a] != q) return 0;
        if (!(c->Y[a] > 0)) return 0;
    }
    return 1;
}

/* Voigt position of the symmetric entry (a, b). */
static int voigt(int d, int a, int b) {
    if (a == b) return a;
    if (d == 2) return 2;
    /* d == 3: 23 -> 3, 13 -> 4, 12 -> 5 */
    int s = a + b;  /* 1+2=3 -> 3, 0+2=2 -> 4, 0+1=1 -> 5 */
    return (s == 3) ? 3 : (s == 2) ? 4 : 5;
}

/* entry A_ab at grid point p of a coefficient field with np points */
static double A_entry(const hor_cell* c, long np, long p, int a, int b) {
    if (c->kind == HOR_ISO) return (a == b) ? c->A[p] : 0.0;
    if (c->kind == HOR_DIAG) return (a == b) ? c->A[(long)a * np + p] : 0.0;
    return c->A[(long)voigt(c->d, a, b) * np + p];
}

/* ------------------------------------------------------------------ */
/* naive DFT (Sec. 4.1, the DFT pair)                                  */
/* ------------------------------------------------------------------ */

int hor_dft_axis(int d, const long* n, int ax, int sign, double* data) {
    if (d < 1 || d > 3 || ax < 0 || ax >= d || (sign != 1 && sign != -1) || !data)
        return HOR_EINVAL;
    long len = n[ax];
    long inner = 1, outer = 1;
    for (int a = ax + 1; a < d; ++a) inner *= n[a];
    for (int a = 0; a < ax; ++a) outer *= n[a];
    /* w^t = exp(sign * 2 pi i t / len), t = (k m) mod len */
    double* cs = (double*)malloc(sizeof(double) * 2 * (size_t)len);
    if (!cs) return HOR_ENOMEM;
    for (long t = 0; t < len; ++t) {
        double th = 2.0 * M_PI * (double)t / (double)len;
        cs[2 * t] = cos(th);
        cs[2 * t + 1] = (double)sign * sin(th);
    }
    const double scale = (sign < 0) ? 1.0 / (double)len : 1.0;
    long nlines = outer * inner;
    int err = 0;
#pragma omp parallel
    {
        double* in = (double*)malloc(sizeof(double) * 2 * (size_t)len);
        double* out = (double*)malloc(sizeof(double) * 2 * (size_t)len);
        if (!in || !out) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (long line = 0; line < nlines; ++line) {
                long o = line / inner, i0 = line % inner;
                double* base = data + 2 * (o * len * inner + i0);
                for (long m = 0; m < len; ++m) {
                    in[2 * m] = base[2 * m * inner];
                    in[2 * m + 1] = base[2 * m * inner + 1];
                }
                for (long k = 0; k < len; ++k) {
                    double sr = 0.0, si = 0.0;
                    long t = 0;
                    for (long m = 0; m < len; ++m) {
                        double xr = in[2 * m], xi = in[2 * m + 1];
                        double wr = cs[2 * t], wi = cs[2 * t + 1];
                        sr += xr * wr - xi * wi;
                        si += xr * wi + xi * wr;
                        t += k;
                        if (t >= len) t -= len;
                    }
                    out[2 * k] = sr * scale;
                    out[2 * k + 1] = si * scale;
                }
                for (long k = 0; k < len; ++k) {
                    base[2 * k * inner] = out[2 * k];
                    base[2 * k * inner + 1] = out[2 * k + 1];
                }
            }
        }
        free(in);
        free(out);
    }
    free(cs);
    return err ? HOR_ENOMEM : HOR_OK;
}

int hor_dft_all(int d, const long* n, int sign, double* data) {
    for (int a = 0; a < d; ++a) {
        int s = hor_dft_axis(d, n, a, sign, data);
        if (s) return s;
    }
    return HOR_OK;
}

/* ------------------------------------------------------------------ */
/* Fourier-space pieces                                                */
/* ------------------------------------------------------------------ */

/* complex [d][grid] <- real [d][grid] (d: the component count) */
static double* to_complex(int d, long np, const double* u) {
    double* z = (double*)calloc(2 * (size_t)d * (size_t)np, sizeof(double));
    if (!z) return NULL;
    for (long i = 0; i < (long)d * np; ++i) z[2 * i] = u[i];
    return z;
}

/* real part of complex [d][grid] into out, after checking that the imaginary
 * part is negligible (a real input gives a real output, Lemma 1 (i)). */
static int to_real(int d, long np, const double* z, double* out) {
    double nr = 0.0, ni = 0.0;
    for (long i = 0; i < (long)d * np; ++i) {
        nr = fmax(nr, fabs(z[2 * i]));
        ni = fmax(ni, fabs(z[2 * i + 1]));
    }
    if (ni > 1e-12 * (nr > 1.0 ? nr : 1.0) && ni > 1e-300) return HOR_ENOTREAL;
    for (long i = 0; i < (long)d * np; ++i) out[i] = z[2 * i];
    return HOR_OK;
}

/* Elasticity (the extension of the scheme beyond the scalar setting named in
 * Sec. 6): strain and stress fields are symmetric d x d tensors, stored as
 * Mandel vectors z [d(d+1)/2][grid] (order 11, 22, 33, 23, 13, 12 as in
 * voigt(), off-diagonal entries times sqrt 2, so that z . z' = Z : Z').  The
 * trial space is the compatible strains, symmetric gradients of periodic
 * displacements: at frequency k != 0 the tensors sym(xi (x) u), u in C^d.
 * The orthogonal projection of Z onto them is sym(xi (x) u) with u the
 * least-squares solution of sym(xi (x) u) = Z, i.e. K u = Z xi with
 * K = (|xi|^2 I + xi xi^T) / 2, whose inverse is (2 / |xi|^2)(I - xi xi^T /
 * (2 |xi|^2)); k = 0 (the mean) is removed.  In place on z. */
static void project_compatible(int d, const long* N, const double* Y, double* z) {
    const int m = d * (d + 1) / 2;
    long np = prod(d, N);
    const double r2 = sqrt(2.0);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        long rem = p;
        double xi[3] = {0, 0, 0};
        int zero = 1;
        for (int a = d - 1; a >= 0; --a) {
            long i = rem % N[a];
            rem /= N[a];
            long k = kof(i, N[a]);
            if (k != 0) zero = 0;
            xi[a] = (double)k / Y[a];
        }
        if (zero) {
            for (int q = 0; q < m; ++q) z[2 * ((long)q * np + p)] = z[2 * ((long)q * np + p) + 1] = 0.0;
            continue;
        }
        /* Z from its Mandel vector (real and imaginary parts) */
        double Zr[3][3], Zi[3][3];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                int q = voigt(d, a, b);
                double f = (a == b) ? 1.0 : 1.0 / r2;
                Zr[a][b] = f * z[2 * ((long)q * np + p)];
                Zi[a][b] = f * z[2 * ((long)q * np + p) + 1];
            }
        double xx = 0.0;
        for (int a = 0; a < d; ++a) xx += xi[a] * xi[a];
        /* t = Z xi, then u = K^-1 t */
        double tr[3] = {0, 0, 0}, ti[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                tr[a] += Zr[a][b] * xi[b];
                ti[a] += Zi[a][b] * xi[b];
            }
        double xtr = 0.0, xti = 0.0;
        for (int a = 0; a < d; ++a) {
            xtr += xi[a] * tr[a];
            xti += xi[a] * ti[a];
        }
        double ur[3], ui[3];
        for (int a = 0; a < d; ++a) {
            ur[a] = (2.0 / xx) * (tr[a] - xi[a] * xtr / (2.0 * xx));
            ui[a] = (2.0 / xx) * (ti[a] - xi[a] * xti / (2.0 * xx));
        }
        /* sym(xi (x) u) back to Mandel form */
        for (int a = 0; a < d; ++a)
            for (int b = a; b < d; ++b) {
                int q = voigt(d, a, b);
                double f = (a == b) ? 1.0 : r2;
                z[2 * ((long)q * np + p)] = f * 0.5 * (xi[a] * ur[b] + ur[a] * xi[b]);
                z[2 * ((long)q * np + p) + 1] = f * 0.5 * (xi[a] * ui[b] + ui[a] * xi[b]);
            }
    }
}

/* Apply Gamma^(k) = xi (x) xi / (xi . xi), Gamma^(0) = 0 (reference A0 = I),
 * in place on the complex vector spectrum z [d][N grid]; with dual != 0 the
 * complementary projection onto J_N, I - Gamma^(k) for k != 0 and 0 at k = 0
 * (G + G_dual + mean = I, the discrete Helmholtz decomposition, Sec. 5.1). */
static void project_fourier(int d, const long* N, const double* Y, double* z, int dual,
                            int elastic) {
    if (elastic) {
        project_compatible(d, N, Y, z);
        return;
    }
    long np = prod(d, N);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        long rem = p;
        double xi[3] = {0, 0, 0};
        int zero = 1;
        for (int a = d - 1; a >= 0; --a) {
            long i = rem % N[a];
            rem /= N[a];
            long k = kof(i, N[a]);
            if (k != 0) zero = 0;
            xi[a] = (double)k / Y[a];
        }
        if (zero) {
            for (int a = 0; a < d; ++a) z[2 * ((long)a * np + p)] = z[2 * ((long)a * np + p) + 1] = 0.0;
            continue;
        }
        double xx = 0.0, sr = 0.0, si = 0.0;
        for (int a = 0; a < d; ++a) {
            xx += xi[a] * xi[a];
            sr += xi[a] * z[2 * ((long)a * np + p)];
            si += xi[a] * z[2 * ((long)a * np + p) + 1];
        }
        if (!dual) {
            for (int a = 0; a < d; ++a) {
                z[2 * ((long)a * np + p)] = xi[a] * sr / xx;
                z[2 * ((long)a * np + p) + 1] = xi[a] * si / xx;
            }
            continue;
        }
        /* (I - xi xi / xx) z as sum_b (xx delta_ab - xi_a xi_b) z_b / xx: a
           field along an axis-aligned xi is removed exactly */
        double orr[3] = {0, 0, 0}, oi[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                double m = ((a == b) ? xx : 0.0) - xi[a] * xi[b];
                orr[a] += m * z[2 * ((long)b * np + p)];
                oi[a] += m * z[2 * ((long)b * np + p) + 1];
            }
        for (int a = 0; a < d; ++a) {
            z[2 * ((long)a * np + p)] = orr[a] / xx;
            z[2 * ((long)a * np + p) + 1] = oi[a] / xx;
        }
    }
}

/* pointwise flux j = A e on a grid of np points: e, j real [d][np] */
static void flux(const hor_cell* c, long np, const double* e, double* j) {
    int d = c->d;
    if (c->kind == HOR_ELASTIC) {
        /* isotropic Hooke law sigma = lambda tr(eps) I + 2 mu eps, Mandel form:
           the first d components are the normal ones */
        const int m = d * (d + 1) / 2;
#pragma omp parallel for schedule(static)
        for (long p = 0; p < np; ++p) {
            double lam = c->A[p], mu = c->A[np + p], tr = 0.0;
            for (int a = 0; a < d; ++a) tr += e[(long)a * np + p];
            for (int q = 0; q < m; ++q)
                j[(long)q * np + p] = 2.0 * mu * e[(long)q * np + p] + ((q < d) ? lam * tr : 0.0);
        }
        return;
    }
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        for (int a = 0; a < d; ++a) {
            double s = 0.0;
            for (int b = 0; b < d; ++b) s += A_entry(c, np, p, a, b) * e[(long)b * np + p];
            j[(long)a * np + p] = s;
        }
    }
}

/* zero-padding of Fourier coefficients from Z_N to Z_M (trigonometric
 * polynomial of T_N seen on the finer grid); zin [d][N], zout [d][M] */
static void pad_spectrum(int d, int nc, const long* N, const long* M, const double* zin,
                         double* zout) {
    long nN = prod(d, N), nM = prod(d, M);
    memset(zout, 0, sizeof(double) * 2 * (size_t)nc * (size_t)nM);
    for (long p = 0; p < nN; ++p) {
        long rem = p, q = 0, stride = 1;
        long idx[3] = {0, 0, 0};
        for (int a = d - 1; a >= 0; --a) {
            idx[a] = rem % N[a];
            rem /= N[a];
        }
        for (int a = d - 1; a >= 0; --a) {
            q += pos(kof(idx[a], N[a]), M[a]) * stride;
            stride *= M[a];
        }
        for (int c = 0; c < nc; ++c) {
            zout[2 * ((long)c * nM + q)] = zin[2 * ((long)c * nN + p)];
            zout[2 * ((long)c * nM + q) + 1] = zin[2 * ((long)c * nN + p) + 1];
        }
    }
}

/* truncation P_N of Fourier coefficients from Z_M to Z_N (Sec. 4.1) */
static void trunc_spectrum(int d, int nc, const long* N, const long* M, const double* zin,
                           double* zout) {
    long nN = prod(d, N), nM = prod(d, M);
    for (long p = 0; p < nN; ++p) {
        long rem = p, q = 0, stride = 1;
        long idx[3] = {0, 0, 0};
        for (int a = d - 1; a >= 0; --a) {
            idx[a] = rem % N[a];
            rem /= N[a];
        }
        for (int a = d - 1; a >= 0; --a) {
            q += pos(kof(idx[a], N[a]), M[a]) * stride;
            stride *= M[a];
        }
        for (int c = 0; c < nc; ++c) {
            zout[2 * ((long)c * nN + p)] = zin[2 * ((long)c * nM + q)];
            zout[2 * ((long)c * nN + p) + 1] = zin[2 * ((long)c * nM + q) + 1];
        }
    }
}

/* ------------------------------------------------------------------ */
/* operators                                                           */
/* ------------------------------------------------------------------ */

int hor_apply_G(const hor_cell* c, const double* u, double* out) {
    if (!valid_cell(c) || !u || !out) return HOR_EINVAL;
    int d = c->d, nc = ncomp(c);
    long np = prod(d, c->N);
    double* z = to_complex(nc, np, u);
    if (!z) return HOR_ENOMEM;
    int s = 0;
    for (int comp = 0; comp < nc && !s; ++comp) s = hor_dft_all(d, c->N, -1, z + 2 * (long)comp * np);
    if (!s) project_fourier(d, c->N, c->Y, z, c->dual, c->kind == HOR_ELASTIC);
    for (int comp = 0; comp < nc && !s; ++comp) s = hor_dft_all(d, c->N, +1, z + 2 * (long)comp * np);
    if (!s) s = to_real(nc, np, z, out);
    free(z);
    return s;
}

/* Interpolate a real field u [d][N] (grid values of a T_N polynomial) to the
 * Q grid: identity for GaNi, Fourier zero-padding for Ga.  out [d][Q]. */
static int interp_to_Q(const hor_cell* c, const double* u, double* out) {
    int d = c->d, nc = ncomp(c);
    long nN = prod(d, c->N), nQ = prod(d, c->Q);
    if (c->scheme == HOR_GANI) {
        memcpy(out, u, sizeof(double) * (size_t)nc * (size_t)nN);
        return HOR_OK;
    }
    double* z = to_complex(nc, nN, u);
    double* zq = (double*)malloc(sizeof(double) * 2 * (size_t)nc * (size_t)nQ);
    if (!z || !zq) { free(z); free(zq); return HOR_ENOMEM; }
    int s = 0;
    for (int comp = 0; comp < nc && !s; ++comp) s = hor_dft_all(d, c->N, -1, z + 2 * (long)comp * nN);
    if (!s) pad_spectrum(d, nc, c->N, c->Q, z, zq);
    for (int comp = 0; comp < nc && !s; ++comp) s = hor_dft_all(d, c->Q, +1, zq + 2 * (long)comp * nQ);
    if (!s) s = to_real(nc, nQ, zq, out);
    free(z);
    free(zq);
    return s;
}

int hor_apply_GA(const hor_cell* c, const double* u, double* out) {
    if (!valid_cell(c) || !u || !out) return HOR_EINVAL;
    int d = c->d, nc = ncomp(c);
    long nN = prod(d, c->N), nQ = prod(d, c->Q);
    double* uq = (double*)malloc(sizeof(double) * (size_t)nc * (size_t)nQ);
    double* jq = (double*)malloc(sizeof(double) * (size_t)nc * (size_t)nQ);
    double* zn = (double*)malloc(sizeof(double) * 2 * (size_t)nc * (size_t)nN);
    if (!uq || !jq || !zn) { free(uq); free(jq); free(zn); return HOR_ENOMEM; }
    int s = interp_to_Q(c, u, uq);            /* u on the quadrature grid */
    double* zq = NULL;
    if (!s) {
        flux(c, nQ, uq, jq);                  /* A_Q u */
        zq = to_complex(nc, nQ, jq);
        if (!zq) s = HOR_ENOMEM;
    }
    for (int comp = 0; comp < nc && !s; ++comp) s = hor_dft_all(d, c->Q, -1, zq + 2 * (long)comp * nQ);
    if (!s) {
        if (c->scheme == HOR_GA) trunc_spectrum(d, nc, c->N, c->Q, zq, zn);
        else memcpy(zn, zq, sizeof(double) * 2 * (size_t)nc * (size_t)nN);
        project_fourier(d, c->N, c->Y, zn, c->dual, c->kind == HOR_ELASTIC);
    }
    for (int comp = 0; comp < nc && !s; ++comp) s = hor_dft_all(d, c->N, +1, zn + 2 * (long)comp * nN);
    if (!s) s = to_real(nc, nN, zn, out);
    free(uq); free(jq); free(zn); free(zq);
    return s;
}

/* ------------------------------------------------------------------ */
/* conjugate gradients (Sec. 5.3, the Lemma on CG for the system)      */
/* ------------------------------------------------------------------ */

static double gdot(long n, long np, const double* a, const double* b) {
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s / (double)np;   /* grid mean, Sec. 5.1 */
}

typedef int (*op_fn)(const hor_cell*, const void*, const double*, double*);

static int op_GA(const hor_cell* c, const void* ctx, const double* u, double* out) {
    (void)ctx;
    return hor_apply_GA(c, u, out);
}

/* L-SD operator M e = e + Gamma_lambda (A - lambda I) e, Gamma_lambda = G / lambda */
static int op_LSD(const hor_cell* c, const void* ctx, const double* u, double* out) {
    double lam = *(const double*)ctx;
    long n = (long)ncomp(c) * prod(c->d, c->N);
    double* t = (double*)malloc(sizeof(double) * (size_t)n);
    double* g = (double*)malloc(sizeof(double) * (size_t)n);
    if (!t || !g) { free(t); free(g); return HOR_ENOMEM; }
    int s = hor_apply_GA(c, u, t);        /* G A u */
    if (!s) s = hor_apply_G(c, u, g);     /* G u   */
    if (!s)
        for (long i = 0; i < n; ++i) out[i] = u[i] + (t[i] - lam * g[i]) / lam;
    free(t); free(g);
    return s;
}

/* Hestenes-Stiefel CG for M x = b from x (as given).  The stopping test is
 * ||r_i|| <= tol ||r_ref|| with ref2 = (r_ref, r_ref); ref2 <= 0 takes the
 * initial residual r_0 (for x0 = 0 the two agree, since r_0 = b). */
static int cg_core(const hor_cell* c, op_fn M, const void* ctx, const double* b, double tol,
                   int max_iter, double ref2, double* x, int* iters, double* relres,
                   double* hist) {
    long np = prod(c->d, c->N);
    long n = (long)ncomp(c) * np;
    double* r = (double*)malloc(sizeof(double) * (size_t)n);
    double* p = (double*)malloc(sizeof(double) * (size_t)n);
    double* q = (double*)malloc(sizeof(double) * (size_t)n);
    if (!r || !p || !q) { free(r); free(p); free(q); return HOR_ENOMEM; }
    int s = M(c, ctx, x, q);
    for (long i = 0; i < n && !s; ++i) r[i] = b[i] - q[i];
    double rho = s ? 0.0 : gdot(n, np, r, r);
    double bb = gdot(n, np, b, b);
    double rho0 = (ref2 > 0.0) ? ref2 : rho;
    int it = 0;
    if (hist && !s) hist[0] = (rho0 > 0.0) ? sqrt(rho / rho0) : 0.0;
    if (!s && rho > 0.0 && sqrt(rho / rho0) > tol) {
        memcpy(p, r, sizeof(double) * (size_t)n);
        for (it = 0; it < max_iter;) {
            s = M(c, ctx, p, q);
            if (s) break;
            double gam = gdot(n, np, p, q);
            if (!(gam > 0.0)) { s = HOR_EBREAKDOWN; break; }
            double alpha = rho / gam;
            for (long i = 0; i < n; ++i) {
                x[i] += alpha * p[i];
                r[i] -= alpha * q[i];
            }
            double rho1 = gdot(n, np, r, r);
            ++it;
            if (hist) hist[it] = sqrt(rho1 / rho0);
            if (sqrt(rho1 / rho0) <= tol) { rho = rho1; break; }
            double beta = rho1 / rho;
            for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
            rho = rho1;
        }
        if (!s && it >= max_iter && sqrt(rho / rho0) > tol) s = HOR_ENOTCONV;
    }
    if (iters) *iters = it;
    if (relres && (s == HOR_OK || s == HOR_ENOTCONV)) {
        int s2 = M(c, ctx, x, q);
        double rr = 0.0;
        if (!s2) {
            for (long i = 0; i < n; ++i) r[i] = b[i] - q[i];
            rr = gdot(n, np, r, r);
        }
        *relres = (bb > 0.0) ? sqrt(rr / bb) : sqrt(rr);
    }
    free(r); free(p); free(q);
    return s;
}

static double* const_field(int d, long np, const double* E) {
    double* f = (double*)malloc(sizeof(double) * (size_t)d * (size_t)np);
    if (!f) return NULL;
    for (int a = 0; a < d; ++a)
        for (long p = 0; p < np; ++p) f[(long)a * np + p] = E[a];
    return f;
}

int hor_cg(const hor_cell* c, const double* E, double tol, int max_iter,
           int warm, double* x, int* iters, double* relres, double* hist) {
    if (!valid_cell(c) || !E || !x || !(tol > 0.0) || max_iter < 0) return HOR_EINVAL;
    int d = c->d, nc = ncomp(c);
    long np = prod(d, c->N), n = (long)nc * np;
    double* Ef = const_field(nc, np, E);
    double* b = (double*)malloc(sizeof(double) * (size_t)n);
    if (!Ef || !b) { free(Ef); free(b); return HOR_ENOMEM; }
    int s = hor_apply_GA(c, Ef, b);           /* b = -G A E */
    for (long i = 0; i < n; ++i) b[i] = -b[i];
    if (!warm) memset(x, 0, sizeof(double) * (size_t)n);
    else if (!s) {
        /* a warm start must lie in E_N: re-project it (Sec. 5.3 Lemma) */
        double* t = (double*)malloc(sizeof(double) * (size_t)n);
        if (!t) s = HOR_ENOMEM;
        else { s = hor_apply_G(c, x, t); memcpy(x, t, sizeof(double) * (size_t)n); free(t); }
    }
    /* the stopping test is relative to ||b||, the initial residual of a cold
       start, so a warm start aims at the residual a cold solve reaches */
    double bb = gdot(n, np, b, b);
    if (!s) s = cg_core(c, op_GA, NULL, b, tol, max_iter, bb, x, iters, relres, hist);
    free(Ef); free(b);
    return s;
}

int hor_cg_lsd(const hor_cell* c, const double* E, double lambda, double tol,
               int max_iter, double* e, int* iters) {
    if (!valid_cell(c) || !E || !e || !(lambda > 0.0) || !(tol > 0.0)) return HOR_EINVAL;
    int d = c->d, nc = ncomp(c);
    long np = prod(d, c->N);
    double* Ef = const_field(nc, np, E);
    if (!Ef) return HOR_ENOMEM;
    memcpy(e, Ef, sizeof(double) * (size_t)nc * (size_t)np);   /* e0 = E */
    int s = cg_core(c, op_LSD, &lambda, Ef, tol, max_iter, 0.0, e, iters, NULL, NULL);
    free(Ef);
    return s;
}

int hor_ms(const hor_cell* c, const double* E, double lambda, double tol,
           int max_iter, double* e, int* iters) {
    if (!valid_cell(c) || !E || !e || !(lambda > 0.0) || !(tol > 0.0)) return HOR_EINVAL;
    int d = c->d, nc = ncomp(c);
    long np = prod(d, c->N), n = (long)nc * np;
    double* Ef = const_field(nc, np, E);
    double* t = (double*)malloc(sizeof(double) * (size_t)n);
    double* g = (double*)malloc(sizeof(double) * (size_t)n);
    if (!Ef || !t || !g) { free(Ef); free(t); free(g); return HOR_ENOMEM; }
    memcpy(e, Ef, sizeof(double) * (size_t)n);
    /* ||b|| of the system G A x = b = -G A E (the CG stopping reference) */
    int s = hor_apply_GA(c, Ef, t);
    double bb = s ? 0.0 : gdot(n, np, t, t);
    int it = 0;
    for (;;) {
        /* e_new = E - Gamma_lambda (A - lambda I) e, Gamma_lambda = G / lambda;
           lambda (e_new - e) = b - G A x for x = e - E, the residual of the
           system, whose norm is the stopping test */
        s = hor_apply_GA(c, e, t);
        if (!s) s = hor_apply_G(c, e, g);
        if (s) break;
        double rr = 0.0;
        for (long i = 0; i < n; ++i) {
            double en = Ef[i] - (t[i] - lambda * g[i]) / lambda;
            rr += lambda * lambda * (en - e[i]) * (en - e[i]);
            t[i] = en;
        }
        rr /= (double)np;
        if (!(bb > 0.0) || sqrt(rr / bb) <= tol) break;
        if (it >= max_iter) { s = HOR_ENOTCONV; break; }
        memcpy(e, t, sizeof(double) * (size_t)n);
        ++it;
    }
    if (iters) *iters = it;
    free(Ef); free(t); free(g);
    return s;
}

/* ------------------------------------------------------------------ */
/* homogenized coefficient by energy quadrature                        */
/* ------------------------------------------------------------------ */

int hor_strain_on_Q(const hor_cell* c, const double* E, const double* x, double* out) {
    if (!valid_cell(c) || !E || !x || !out) return HOR_EINVAL;
    int d = c->d, nc = ncomp(c);
    long nQ = prod(d, c->Q);
    int s = interp_to_Q(c, x, out);
    if (!s)
        for (int a = 0; a < nc; ++a)
            for (long p = 0; p < nQ; ++p) out[(long)a * nQ + p] += E[a];
    return s;
}

int hor_homogenized(const hor_cell* c, int L, const double* E, const double* x,
                    double* W, double* J) {
    if (!valid_cell(c) || L < 1 || !E || !x || !W) return HOR_EINVAL;
    int d = c->d, nc = ncomp(c);
    long nN = prod(d, c->N), nQ = prod(d, c->Q);
    double* e = (double*)malloc(sizeof(double) * (size_t)L * (size_t)nc * (size_t)nQ);
    double* j = (double*)malloc(sizeof(double) * (size_t)L * (size_t)nc * (size_t)nQ);
    if (!e || !j) { free(e); free(j); return HOR_ENOMEM; }
    int s = 0;
    for (int l = 0; l < L && !s; ++l) {
        s = hor_strain_on_Q(c, E + (long)l * nc, x + (long)l * nc * nN, e + (long)l * nc * nQ);
        if (!s) flux(c, nQ, e + (long)l * nc * nQ, j + (long)l * nc * nQ);
    }
    if (!s) {
        for (int l = 0; l < L; ++l)
            for (int m = 0; m < L; ++m)
                W[l * L + m] = gdot((long)nc * nQ, nQ, e + (long)l * nc * nQ, j + (long)m * nc * nQ);
        if (J)
            for (int l = 0; l < L; ++l)
                for (int a = 0; a < nc; ++a) {
                    double sum = 0.0;
                    const double* jj = j + (long)l * nc * nQ + (long)a * nQ;
                    for (long p = 0; p < nQ; ++p) sum += jj[p];
                    J[l * nc + a] = sum / (double)nQ;
                }
    }
    free(e); free(j);
    return s;
}

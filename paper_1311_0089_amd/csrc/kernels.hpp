// kernels.hpp -- argument blocks and launchers of the hot-path kernels.
//
// The solver iterates on the scalar potential c(k) of the fluctuation,
// e^(k) = n(k) c(k) with n = xi / |xi| (n(0) = 0).  The map c -> F^-1[n c]
// is an isometry onto E_N (grid product on the real side, Hermitian-weighted
// sum on the Fourier side, Sec. 4.1), so conjugate gradients on
//     Op(c) = n . Trunc F_Q [ A F_Q^-1 Pad (n c) ]
// produce exactly the iterates of CG on G_N A_N e = -G_N A_N E (Sec. 5.2-5.3),
// with the projection Gamma^ = n (x) n applied on the way in and out.
//
// Spectra are half spectra along the last axis: [k_0]..[k_{d-2}][h],
// h in [0, (N_{d-1}+1)/2), other axes in FFT order.  Real fields are
// [x_0]..[x_{d-1}] in FFT order.  Components are outermost per item, items
// (load cases / served cells) outermost overall.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <vector>

#include "fft_device.hpp"

namespace hom {

constexpr int kThreads = 256;
// the FP32 recursion of the mixed solver aims at this fraction of the outer
// tolerance, so the FP64 residual that replaces it usually passes the test
constexpr double kTolSafety = 0.5;

// a CG iteration's fused scalar work: the (r, r) partials of the last update
// (rr, rr_n per item, stride P) from which the direction step derives beta and
// the stopping test and the projection does the bookkeeping
struct CgFuse {
  const double* rr;
  int rr_n;
  // the last update left x to the direction step: x += alpha p (old p) there
  int xdef;
  // the (p, q) partials of this iteration's last-axis pass: the projection's
  // first workgroup sums them into ItemScal::pq for the update
  const double* pq;
  int pq_n;
};

// per-item solver scalars, device resident
struct ItemScal {
  double rho, rho0, gamma, alpha, beta, tol;
  int active;    // 1 while the item iterates; kernels skip inactive items
  int iters;     // iterations done
  int status;    // 0, or -5 on breakdown
  int conv;      // 1 once the stopping test passed
  int max_iter;
  int fresh;     // 1: beta and the stopping test are current (set at a (re)start and by
                 // the end-of-launch bookkeeping); 0: the next expansion derives them
  // Stop flags of the captured iterations.  Inside a graph no kernel writes a
  // field that other workgroups of the same launch read: the projection's
  // first workgroup books the last update and raises `halt` (read from the
  // update on, never by the projection); the update's first workgroup copies
  // `halt` into `stopped` (read by the projections of later iterations) and
  // raises `broke` on breakdown (read by the passes of later iterations,
  // never by the update).  `active` changes only outside the iterations: the
  // end-of-launch bookkeeping clears it once `halt` or `broke` is raised.
  int halt;
  int stopped;
  int broke;
  // Moulinec-Suquet step 1 / lambda, kept here rather than in a captured
  // kernel argument: cells of one shape share an engine and its graphs
  double step;
  // (p, q) of the current CG iteration, summed by the projection's first
  // workgroup from the last-axis pass's partials; read by the update
  double pq;
};

// an item the passes of a CG iteration still work on (the projection tests
// `stopped` instead of `halt`, which it raises itself)
__host__ __device__ inline bool item_live(const ItemScal& q) {
  return q.active && !q.halt && !q.broke;
}
__host__ __device__ inline bool item_live_project(const ItemScal& q) {
  return q.active && !q.stopped && !q.broke;
}

enum { EPI_STORE = 0, EPI_RHS = 1, EPI_RESID = 2 };
enum { ROW_APPLY = 0, ROW_CONST = 1, ROW_SYNTH = 2, ROW_FWD = 3 };

// geometry of the unit normal n(k): column index -> (k_1, h) or h
struct NormalGeo {
  int d;
  int N1;        // trial size of axis 1 (3-D only)
  int H;         // half-spectrum bins of the last axis
  int dual;      // dual problem on J_N (2-D: the rotated normal t = (-n_1, n_0))
  int npot;      // potentials per frequency: 1; 2 (3-D dual); d (elasticity)
  long pot_stride;   // elements between the potentials of an item
  int nf;        // field components: d, or d(d+1)/2 Mandel components (elasticity)
  int elastic;   // linear elasticity: compatible strains, potentials = displacements
  double invY[3];
};

// pass along axis 0 from the scalar potential: X_a = F_0^-1 Pad(n_a c)
template <class T>
struct ColExpandArgs {
  // scalar spectra: element (axis-0 index i, column) at i * si + column * sc
  // (row-major: si = inner, sc = 1; column-major: si = 1, sc = n_in)
  const cpx<T>* c;  // scalar spectrum
  cpx<T>* X;        // [item][d][n_fft][inner]
  long c_stride, X_stride, X_cstride;
  int n_in, n_fft, inner, W;
  int si, sc_;      // scalar strides (see above); si == 1 maps axis 0 across threads
  NormalGeo g;
  FftPlan plan;
  const cpx<T>* tw;
  ItemScal* sc;     // nullable
};

// plain complex pass along a middle axis (3-D axis 1), per component
template <class T>
struct ColPlainArgs {
  const cpx<T>* in;  // [item][d][outer][n_in][inner]
  cpx<T>* out;       // [item][d][outer][n_out][inner]
  long in_stride, in_cstride, out_stride, out_cstride;
  int outer, n_in, n_fft, n_out, inner, W, d;
  T scale;           // 1/n on forward passes
  // k_col_mid2 only: xi_1 = k_1 xi1_step along the pass, xi_2 = h xi2_step
  double xi1_step, xi2_step;
  FftPlan plan;
  const cpx<T>* tw;
  ItemScal* sc;
};

// forward pass along axis 0 with truncation and projection on n:
// q = n . Trunc F_0 [X] (then one of the epilogues)
template <class T>
struct ColProjectArgs {
  const cpx<T>* X;   // [item][d][n_fft][inner]
  long X_stride, X_cstride;
  cpx<T>* q;         // scalar spectrum, layout as in ColExpandArgs (si, sc_)
  long s_stride;     // item stride of all scalar spectra below
  const cpx<T>* p;   // EPI_STORE: partial (p, q) when non-null
  cpx<T>* r;         // EPI_RHS: r = p = q = -n.F[..]; x = 0   EPI_RESID: r = b - q
  cpx<T>* pp;
  cpx<T>* x;
  const cpx<T>* b;
  double* partials;  // [item][P]
  int P;
  int n_fft, n_out, inner, W, epi, d;
  int si, sc_;
  // CG bookkeeping in workgroup 0 (rr_part non-null): iteration count,
  // stopping test and rho from the (r, r) partials of the last update
  const double* rr_part;
  int rr_n;
  // the (p, q) partials to sum into ItemScal::pq in workgroup 0 (nullable)
  const double* pq_part;
  int pq_n;
  T scale;
  NormalGeo g;
  FftPlan plan;
  const cpx<T>* tw;
  ItemScal* sc;
};

// contiguous (last) axis: c2r -> pointwise -> r2c, in LDS
template <class T>
struct RowArgs {
  const cpx<T>* in;     // [item][d][rows][H]
  cpx<T>* out;          // [item][d][rows][H]
  long in_stride, in_cstride, out_stride, out_cstride;
  const double* ureal;  // ROW_FWD input  [item][d][rows][n]
  double* oreal;        // ROW_SYNTH output [item][d][rows][n]
  long real_stride, real_cstride;
  const T* A;           // [block][nA][rows][n]; item i uses block i / A_group
  long A_stride, A_cstride;
  int A_group;          // items sharing one coefficient block (>= 1)
  int kind;             // 0 iso, 1 diag, 2 full symmetric (Voigt)
  const double* E;      // [item][d] (ROW_CONST, ROW_SYNTH)
  int d, rows, n, H, RP;
  int items;            // items of the launch (set by the launcher)
  FftPlan plan;
  const cpx<T>* tw;
  ItemScal* sc;
  // ROW_APPLY: when non-null, the partial sums of e . (A e) over the real
  // points of each workgroup, times pscale, at [item][P] (slot: row tile)
  double* partials;
  int P;
  double pscale;
};

template <class T>
struct CgUpdateArgs {
  cpx<T>* x;
  cpx<T>* r;
  const cpx<T>* p;
  const cpx<T>* q;
  long stride, count;   // item stride and elements per item
  int H;                // weight 1 for h = 0, 2 otherwise
  int n0;               // column = e / n0 (column-major scalars; 1 for row-major)
  double* partials;
  int P;
  ItemScal* sc;
  // partials of (p, q) left by the projection: every workgroup derives
  // alpha = rho / (p, q) itself; pq_sc: (p, q) is ItemScal::pq instead
  const double* pq_part;
  int pq_n;
  int pq_sc;
  // 1: x += alpha p here; 0: the next expansion does it (it reads p anyway)
  int xupd;
};

// the direction step of a CG iteration, a streaming kernel ahead of the
// expansion: beta and the stopping test from the (r, r) partials of the last
// update (unless the scalars are fresh), x += alpha p with the old p when the
// last update left it (xdef), then p <- r + beta p
template <class T>
struct CgDirArgs {
  cpx<T>* x;
  const cpx<T>* r;
  cpx<T>* p;
  long stride, count;
  ItemScal* sc;
  const double* rr_part;
  int rr_n, P;
  int xdef;
};

// compile-time specialised pass kernels, registered by kernels_static*.hip
enum { KK_EXPAND = 0, KK_PROJECT = 1, KK_PLAIN_INV = 2, KK_PLAIN_FWD = 3, KK_ROW = 4,
       KK_ROW_CONST = 5, KK_ROW_SYNTH = 6,
       // 3-D cells with two spectra between the first- and middle-axis passes
       KK_EXPAND2 = 7, KK_PROJECT2 = 8, KK_MID2_INV = 9, KK_MID2_FWD = 10,
       // 3-D elasticity: first-axis expansion with the basis map fused in
       KK_BEXPAND = 11 };
struct StaticKernel {
  int kind, esz, n, ntrial, d;  // d: component count (row kernels), else 0
  const void* fn;
  int W;                        // tile width (column kernels) or row pairs (row kernels)
  int NT;                       // workgroup size
  size_t lds;                   // dynamic LDS bytes
  int len, blue, nst, rad[kMaxStages];  // the compile-time FFT plan
  int ilv;                      // row kernels: items interleaved on a 1-D grid
  int ipw;                      // row kernels: items per workgroup (0: one)
};
std::vector<StaticKernel>& static_registry();
void register_static(const StaticKernel& k);
void set_static_enabled(bool on);
bool static_enabled();
// bumped by every change of the kernel choices (set_choice, set_static_enabled)
unsigned tune_version();
// entry for (kind, element size, FFT length, trial length, d) whose plan
// matches p, or nullptr (then the generic kernel runs); follows the tuned
// choice when one is recorded, else the first registered variant
const StaticKernel* find_static(int kind, int esz, int n, int ntrial, int d, const FftPlan& p);
std::vector<const StaticKernel*> static_variants(int kind, int esz, int n, int ntrial, int d,
                                                 const FftPlan& p);
struct TuneKey {
  int kind, esz, n, ntrial, d;
  bool operator<(const TuneKey& o) const {
    if (kind != o.kind) return kind < o.kind;
    if (esz != o.esz) return esz < o.esz;
    if (n != o.n) return n < o.n;
    if (ntrial != o.ntrial) return ntrial < o.ntrial;
    return d < o.d;
  }
};
void set_choice(const TuneKey& key, int v);  // -1 generic, v >= 0 the v-th variant
bool get_choice(const TuneKey& key, int* v);
std::map<TuneKey, int> all_choices();

// launchers (defined in kernels.hip); sk selects a specialised kernel (its W /
// row pairs must already be in the arguments); all return the launch status
template <class T>
hipError_t launch_col_expand(const ColExpandArgs<T>& a, int items, size_t lds, hipStream_t s,
                             const StaticKernel* sk = nullptr);
template <class T>
hipError_t launch_col_plain(const ColPlainArgs<T>& a, int items, int sign, size_t lds,
                            hipStream_t s, const StaticKernel* sk = nullptr);
template <class T>
hipError_t launch_col_project(const ColProjectArgs<T>& a, int items, size_t lds, hipStream_t s,
                              const StaticKernel* sk = nullptr);
template <class T>
hipError_t launch_row(const RowArgs<T>& a, int items, int mode, size_t lds, hipStream_t s,
                      const StaticKernel* sk = nullptr);
template <class T>
hipError_t launch_cg_update(const CgUpdateArgs<T>& a, int items, int blocks, hipStream_t s);
template <class T>
hipError_t launch_cg_direction(const CgDirArgs<T>& a, int items, int blocks, hipStream_t s);

// The potentials of real fields obey c(-k) = sigma conj(c(k)) on the h = 0
// plane of the half spectrum, where k and -k are both stored (sigma = -1 for
// an odd basis vector: n, the 2-D rotated normal, t_1 of the 3-D dual; +1 for
// the even t_2).  The last-axis inverse transform keeps only the real part of
// that plane, so the operator annihilates a component of the other symmetry.
// Rounding leaves one in a computed right-hand side; where the exact
// right-hand side vanishes (a load case the cell does not perturb) it is all
// there is, and CG cannot reduce it.  SymArgs names up to three vectors of
// one layout that are given the exact symmetry.
template <class T>
struct SymArgs {
  cpx<T>* v[3];         // vectors (null: unused)
  long stride;          // item stride
  long pot_stride;      // between the potentials of an item
  int npot;             // potentials per frequency
  int even_pot;         // the potential whose basis vector is even in k (-1: none)
  int N0, N1;           // extents of the plane (2-D cells: N1 = 1)
  long s0, s1;          // element strides of the plane's two axes
  const ItemScal* sc;   // selection (null: every item; else item_live_project)
};
template <class T>
hipError_t launch_sym_h0(const SymArgs<T>& a, int items, hipStream_t s);

// Cells with several potentials per frequency (3-D dual, elasticity) split
// each first-axis pass into a per-frequency basis map on the trial rows and a
// plain column transform (the compile-time kernels of the shape):
//   expand:  X_a(k) = sum_p b_p[a](k) c_p(k), then F_0^-1 with padding;
//   project: F_0 with truncation, then q_p(k) = sum_a b_p[a](k) X^_a(k) and
//            the epilogue of the projection pass (store with (p, q), right-hand
//            side, residual; the bookkeeping of the last update in workgroup 0).
// X holds component spectra on the trial rows: [item][nf][N0][inner] with the
// component stride X_cstride; the potentials use the scalar layout (si, sc_).
template <class T>
struct BasisArgs {
  const cpx<T>* c;     // expand: potentials
  cpx<T>* Xo;          // expand: component spectra written
  const cpx<T>* Xi;    // project: transformed component spectra read
  long c_stride, X_stride, X_cstride;
  int N0, inner, si, sc_;
  // project epilogue (as ColProjectArgs)
  cpx<T>* q;
  const cpx<T>* p;
  cpx<T>* r;
  cpx<T>* pp;
  cpx<T>* x;
  const cpx<T>* b;
  double* partials;
  int P, epi;
  const double* rr_part;
  int rr_n;
  const double* pq_part;
  int pq_n;
  NormalGeo g;
  ItemScal* sc;
};
template <class T>
hipError_t launch_basis_expand(const BasisArgs<T>& a, int items, int blocks, hipStream_t s);
template <class T>
hipError_t launch_basis_project(const BasisArgs<T>& a, int items, int blocks, hipStream_t s);
// part[item][b] for b < blocks: the Hermitian-weighted (v, v) of a share of
// the item's count elements (weight 1 where h = (e / n0) % H is 0, else 2)
template <class T>
hipError_t launch_norm_parts(const cpx<T>* v, long stride, long count, int n0, int H,
                             double* part, int P, int blocks, int items, const ItemScal* sc,
                             hipStream_t s);

// Eigenvalue range [lo, hi] of the coefficient at one point (v holds its
// nA values: kind 0 a I, kind 1 diagonal, kind 2 symmetric in Voigt order);
// false if a value is not finite or the matrix is not positive definite.
__host__ __device__ inline int coef_values(int kind, int d) {
  return kind == 0 ? 1 : kind == 1 ? d : kind == 3 ? 2 : d * (d + 1) / 2;
}

__host__ __device__ inline bool point_range(int d, int kind, const double* v, double* lo, double* hi) {
  for (int t = 0; t < coef_values(kind, d); ++t)
    if (!isfinite(v[t])) return false;
  if (kind == 3) {
    // isotropic elasticity (lambda, mu) in d dimensions: the Mandel stiffness
    // has the eigenvalues 2 mu and d lambda + 2 mu
    const double a = 2.0 * v[1], b = d * v[0] + 2.0 * v[1];
    *lo = fmin(a, b);
    *hi = fmax(a, b);
    return *lo > 0;
  }
  if (kind == 0) {
    *lo = *hi = v[0];
    return v[0] > 0;
  }
  if (kind == 1) {
    *lo = *hi = v[0];
    for (int a = 0; a < d; ++a) {
      *lo = fmin(*lo, v[a]);
      *hi = fmax(*hi, v[a]);
    }
    return *lo > 0;
  }
  if (d == 1) {
    *lo = *hi = v[0];
    return v[0] > 0;
  }
  if (d == 2) {
    const double a = v[0], b = v[1], c = v[2];
    const double m = 0.5 * (a + b), r = sqrt(0.25 * (a - b) * (a - b) + c * c);
    *lo = m - r;
    *hi = m + r;
    return *lo > 0;
  }
  // 3x3 symmetric: closed-form eigenvalues (trigonometric method)
  const double a00 = v[0], a11 = v[1], a22 = v[2], a12 = v[3], a02 = v[4], a01 = v[5];
  const double p1 = a01 * a01 + a02 * a02 + a12 * a12;
  const double q = (a00 + a11 + a22) / 3.0;
  if (p1 == 0.0) {
    *lo = fmin(a00, fmin(a11, a22));
    *hi = fmax(a00, fmax(a11, a22));
    return *lo > 0;
  }
  const double p2 = (a00 - q) * (a00 - q) + (a11 - q) * (a11 - q) + (a22 - q) * (a22 - q) + 2 * p1;
  const double p = sqrt(p2 / 6.0);
  const double b00 = (a00 - q) / p, b11 = (a11 - q) / p, b22 = (a22 - q) / p;
  const double b01 = a01 / p, b02 = a02 / p, b12 = a12 / p;
  const double detB = b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) +
                      b02 * (b01 * b12 - b11 * b02);
  double rr = detB / 2.0;
  rr = fmax(-1.0, fmin(1.0, rr));
  const double phi = acos(rr) / 3.0;
  const double e1 = q + 2 * p * cos(phi);
  const double e3 = q + 2 * p * cos(phi + 2.0 * M_PI / 3.0);
  *lo = e3;
  *hi = e1;
  // Sylvester criterion as the definiteness test (robust against rounding of e3)
  const double m1 = a00, m2 = a00 * a11 - a01 * a01;
  const double m3 = a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) +
                    a02 * (a01 * a12 - a11 * a02);
  return m1 > 0 && m2 > 0 && m3 > 0 && e3 > 0;
}

// Range of the whole field A [nA][npts] (device pointer): lo, hi and flags
// (bit 0: a value not finite, bit 1: a point not positive definite).
// scratch: device buffer of kQuadScratch doubles; host: pinned host buffer
// of at least 3 * 1024 doubles.
constexpr int kQuadBlocks = 2048;   // workgroups of the energy quadrature
constexpr int kQuadSlots = 27;      // per workgroup: 3 x 3 W slots and 3 x (up to 6) J sums
constexpr long kQuadScratch = (long)kQuadBlocks * kQuadSlots + 64;
hipError_t a_field_range(const double* A, int d, int kind, long npts, double* scratch,
                         double* host, hipStream_t s, double* lo, double* hi, int* flags);

// Arm HIP events for the next `launches` kernels launched by this thread
// through the launchers below: hipExtLaunchKernel records the start event from
// the first dispatch and the stop event from the last one.
void arm_launch_events(hipEvent_t start, hipEvent_t stop, int launches = 1);

// CG start: rho = (r_0, r_0) from partials; the stopping test is relative to
// (b, b) from ref (nullable: to rho itself, the cold start where r_0 = b); an
// item already meeting it does not iterate.  mask (nullable): only items
// active in the mask are touched
hipError_t launch_cg_init(ItemScal* sc, const double* partials, int P, int nparts, int items,
                          hipStream_t s, const ItemScal* mask = nullptr,
                          const double* ref = nullptr);
// end-of-launch bookkeeping of the last update: iteration count, stopping
// test, beta and rho from its (r, r) partials; marks the scalars fresh
hipError_t launch_cg_finalize(ItemScal* sc, const double* partials, int P, int nparts, int items,
                              hipStream_t s);
// outer (FP64 refinement) residual check: rho = sum partials; stop when
// sqrt(rho / rho0) <= tol or after max_iter refinement steps; the first call
// (init != 0) sets rho0.
hipError_t launch_outer_check(ItemScal* sc, const double* partials, int P, int nparts, int items,
                              int init, hipStream_t s, const ItemScal* mask = nullptr);
// FP32 recursion (re)started from the FP64 residual: r32 = r64 / ||b|| (one
// scale per solve, ||b||^2 = rho0 of the outer scalars), x32 = 0 and partials
// of (r32, r32).  keep_dir = 0 is a fresh start (p32 = r32, iteration count
// reset); keep_dir = 1 replaces the recursive residual and keeps p32.  The
// outer counter of residual evaluations is incremented.
hipError_t launch_inner_start(const cpx<double>* r64, cpx<float>* r32, cpx<float>* p32,
                              cpx<float>* x32, long stride, long count, int H, int n0,
                              ItemScal* outer,
                              ItemScal* inner, int max_iter, int keep_dir, double* partials, int P,
                              int blocks, int items, hipStream_t s, const ItemScal* mask = nullptr);
// inner scalars after launch_inner_start: rho = (r32, r32); a kept direction
// continues with beta scaled to the new residual (a fresh start, or a true
// residual more than twice the recursive one, restarts with p = r).  The
// recursion stops once its residual fell by max(eta, theta tol_out /
// rel_out), where the host replaces it again.  An item whose iteration budget
// is spent also stops its outer loop.
hipError_t launch_inner_init(ItemScal* inner, const double* partials, int P, int nparts, int items,
                             ItemScal* outer, double eta, double theta, hipStream_t s,
                             const ItemScal* mask = nullptr);
// x64 += ||b|| * x32
hipError_t launch_inner_accumulate(cpx<double>* x64, const cpx<float>* x32, long stride, long count,
                                   const ItemScal* outer, int blocks, int items, hipStream_t s,
                                   const ItemScal* mask = nullptr);
// Moulinec-Suquet iteration (Sec. 5.3): book the residual of the step
// (partials of (r, r) from the projection): stop at ||r|| <= tol ||b|| or the
// budget, else count the step; then x += step * r for items still iterating
hipError_t launch_ms_book(ItemScal* sc, const double* partials, int P, int nparts, int items,
                          hipStream_t s);
hipError_t launch_ms_axpy(cpx<double>* x, const cpx<double>* r, long stride, long count,
                          const ItemScal* sc, int blocks, int items, hipStream_t s);
// x = 0, active flags etc.
hipError_t launch_set_scal(ItemScal* sc, int items, double tol, int max_iter, int active,
                           hipStream_t s, double step = 0.0);
// energy quadrature over a grid of npts points for load-case groups
// (l0..l0+nl) x (m0..m0+nm), nl, nm <= 3; e: [L][d][npts], A: [nA][npts]
hipError_t launch_quad(const double* e, long e_stride, long e_cstride, const double* A,
                       long A_cstride, int kind, int d, long npts, int l0, int nl, int m0, int nm,
                       double* partials, int blocks, hipStream_t s);
hipError_t launch_quad_final(const double* partials, int blocks, int nl, int nm, int d,
                             long npts, double* out, hipStream_t s);
// FP64 <-> FP32 element copies
hipError_t launch_convert(const double* in, float* out, long n, hipStream_t s);
hipError_t launch_widen(const float* in, double* out, long n, hipStream_t s);
// p[0..n) = 0 by a kernel (no memset node where a caller captures a graph)
hipError_t launch_zero(double* p, long n, hipStream_t s);

// largest dynamic LDS size a kernel may use (set at library init)
hipError_t configure_kernels(size_t max_lds);

}  // namespace hom

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

// per-item solver scalars, device resident
struct ItemScal {
  double rho, rho0, gamma, alpha, beta, tol;
  int active;    // 1 while the item iterates; kernels skip inactive items
  int iters;     // iterations done
  int status;    // 0, or -5 on breakdown
  int conv;      // 1 once the stopping test passed
  int max_iter;
  int pad;
};

enum { EPI_STORE = 0, EPI_RHS = 1, EPI_RESID = 2 };
enum { ROW_APPLY = 0, ROW_CONST = 1, ROW_SYNTH = 2, ROW_FWD = 3 };

// geometry of the unit normal n(k): column index -> (k_1, h) or h
struct NormalGeo {
  int d;
  int N1;        // trial size of axis 1 (3-D only)
  int H;         // half-spectrum bins of the last axis
  double invY[3];
};

// pass along axis 0 from the scalar potential: X_a = F_0^-1 Pad(n_a c)
template <class T>
struct ColExpandArgs {
  const cpx<T>* c;  // scalar spectrum [item][n_in][inner]
  const cpx<T>* r;  // fuse: p <- r + beta p, then expand p (c must equal p)
  cpx<T>* p;
  cpx<T>* X;        // [item][d][n_fft][inner]
  long c_stride, X_stride, X_cstride;
  int n_in, n_fft, inner, W, fuse;
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
  cpx<T>* q;         // [item][n_out][inner]
  long s_stride;     // item stride of all scalar spectra below
  const cpx<T>* p;   // EPI_STORE: partial (p, q) when non-null
  cpx<T>* r;         // EPI_RHS: r = p = q = -n.F[..]; x = 0   EPI_RESID: r = b - q
  cpx<T>* pp;
  cpx<T>* x;
  const cpx<T>* b;
  double* partials;  // [item][P]
  int P;
  int n_fft, n_out, inner, W, epi, d;
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
  FftPlan plan;
  const cpx<T>* tw;
  ItemScal* sc;
};

template <class T>
struct CgUpdateArgs {
  cpx<T>* x;
  cpx<T>* r;
  const cpx<T>* p;
  const cpx<T>* q;
  long stride, count;   // item stride and elements per item
  int H;                // weight 1 for h = 0, 2 otherwise
  double* partials;
  int P;
  ItemScal* sc;
};

// compile-time specialised pass kernels, registered by kernels_static*.hip
enum { KK_EXPAND = 0, KK_PROJECT = 1, KK_PLAIN_INV = 2, KK_PLAIN_FWD = 3, KK_ROW = 4 };
struct StaticKernel {
  int kind, esz, n, ntrial, d;  // d: component count (row kernels), else 0
  const void* fn;
  int W;                        // tile width (column kernels) or row pairs (row kernels)
  int NT;                       // workgroup size
  size_t lds;                   // dynamic LDS bytes
  int len, blue, nst, rad[kMaxStages];  // the compile-time FFT plan
};
std::vector<StaticKernel>& static_registry();
void register_static(const StaticKernel& k);
void set_static_enabled(bool on);
bool static_enabled();
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

// mask (nullable): only items active in the mask are touched
hipError_t launch_cg_init(ItemScal* sc, const double* partials, int P, int nparts, int items,
                          hipStream_t s, const ItemScal* mask = nullptr);
hipError_t launch_cg_alpha(ItemScal* sc, const double* partials, int P, int nparts, int items,
                           hipStream_t s);
hipError_t launch_cg_beta(ItemScal* sc, const double* partials, int P, int nparts, int items,
                          hipStream_t s);
// outer (FP64 refinement) residual check: rho = sum partials; stop when
// sqrt(rho / rho0) <= tol or after max_iter refinement steps; the first call
// (init != 0) sets rho0.
hipError_t launch_outer_check(ItemScal* sc, const double* partials, int P, int nparts, int items,
                              int init, hipStream_t s, const ItemScal* mask = nullptr);
// inner FP32 start: r32 = p32 = r64 / sqrt(rho_out), x32 = 0, inner scalars
// reset, outer step counter incremented
hipError_t launch_inner_start(const cpx<double>* r64, cpx<float>* r32, cpx<float>* p32,
                              cpx<float>* x32, long stride, long count, int H, ItemScal* outer,
                              ItemScal* inner, double eta, int max_iter, double* partials, int P,
                              int blocks, int items, hipStream_t s, const ItemScal* mask = nullptr);
// x64 += sqrt(rho_out) * x32
hipError_t launch_inner_accumulate(cpx<double>* x64, const cpx<float>* x32, long stride, long count,
                                   const ItemScal* outer, int blocks, int items, hipStream_t s,
                                   const ItemScal* mask = nullptr);
// x = 0, active flags etc.
hipError_t launch_set_scal(ItemScal* sc, int items, double tol, int max_iter, int active,
                           hipStream_t s);
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

// largest dynamic LDS size a kernel may use (set at library init)
hipError_t configure_kernels(size_t max_lds);

}  // namespace hom

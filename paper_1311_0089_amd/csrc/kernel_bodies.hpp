// kernel_bodies.hpp -- the FFT pass kernels, written once over a size policy.
//
// A column policy (ColGen / ColStat) supplies the workgroup size NT, the tile
// width W, the FFT length and the trial length, and the line transform: the
// generic policy reads them from the kernel arguments and runs the runtime-
// planned transform of fft_device.hpp; the static policy makes them
// compile-time constants and runs the specialised transform of
// fft_static.hpp.  Row policies (RowGen / RowStat) do the same for the
// last-axis pass (component count D, row pairs per workgroup RP).
#pragma once
#include "fft_static.hpp"
#include "kernels.hpp"

namespace hom {


// Workgroups are dispatched round-robin over the 8 XCDs of the chip (block b
// goes to XCD b mod 8).  Give each XCD a contiguous run of tiles so that
// neighbouring tiles, which share cache lines, meet in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  if (n % 8) return b;
  return (b % 8) * (n / 8) + b / 8;
}

// loads in flight per thread for n elements over NT threads (n known at
// compile time, else 0: the default cap)
__host__ __device__ constexpr int rounds_ch(int n, int NT, int cap = 8) {
  return (n <= 0) ? cap : ((n + NT - 1) / NT < cap ? (n + NT - 1) / NT : cap);
}

// SL: layout of the scalar spectra (0: given at run time by the strides,
// 1: column-major, 2: row-major); fixed at compile time in the specialised
// kernels, so only one thread mapping is built
struct ColGen {
  static constexpr int NT = kThreads;
  static constexpr int CP = 1;   // components per transform call
  static constexpr bool PRE = false;
  static constexpr int SL = 0;
  static constexpr int WC = 0;   // tile width when known at compile time
  static constexpr int NF = 0;   // FFT length when known at compile time
  static constexpr int WPE = 1;  // waves per SIMD the register allocation must allow
  __device__ static int W(int w) { return w; }
  __device__ static int nfft(int n) { return n; }
  __device__ static int ntrial(int n) { return n; }
  // LDS row length of the expand / project tiles ([row][component][column])
  __device__ static int rowlen(int lw) { return lw; }
  template <class T, int S>
  __device__ static void fft(cpx<T>* lds, const FftPlan& P, int W, const cpx<T>* tw) {
    line_fft<T, S>(lds, P, LdsLines{W, 1, W, true}, tw);
  }
  template <class T, int S>
  __device__ static void fft_rows(cpx<T>* lds, const FftPlan& P, int W, const cpx<T>* tw) {
    line_fft<T, S>(lds, P, LdsLines{W, 1, W, true}, tw);
  }
};

// an even row length of 8-byte or 16-byte elements is padded to the next odd
// one where the expand / project tiles are written and read with axis 0
// across the threads of a wave (column-major scalars): an even stride folds
// those accesses onto few LDS banks
__host__ __device__ constexpr int odd_rowlen(int lw) { return (lw > 1 && lw % 2 == 0) ? lw + 1 : lw; }

template <class SP, int NTRIAL, int W_, int NT_, int SL_ = 0, bool MF_ = false, int WPE_ = 1,
          bool PRE_ = false>
struct ColStat {
  static constexpr int NT = NT_;
  static constexpr int CP = 1;
  // projection pass: every component's tile loads go out before the first
  // transform (held in registers), instead of one component at a time
  static constexpr bool PRE = PRE_;
  static constexpr int SL = SL_;
  static constexpr int WC = W_;
  static constexpr int NF = SP::n;
  static constexpr int WPE = WPE_;
  // only the column-major mapping (axis 0 across the threads) needs the pad
  static constexpr int RL = (SL_ == 1) ? odd_rowlen(W_) : W_;
  __device__ static constexpr int W(int) { return W_; }
  __device__ static constexpr int nfft(int) { return SP::n; }
  __device__ static constexpr int ntrial(int) { return NTRIAL; }
  __device__ static constexpr int rowlen(int) { return RL; }
  template <class T, int S>
  __device__ __forceinline__ static void fft(cpx<T>* lds, const FftPlan& P, int, const cpx<T>* tw) {
    sfft<T, S, SP, W_, true, 1, W_, NT_, MF_>(lds, tw, P);
  }
  template <class T, int S>
  __device__ __forceinline__ static void fft_rows(cpx<T>* lds, const FftPlan& P, int,
                                                  const cpx<T>* tw) {
    sfft<T, S, SP, W_, true, 1, RL, NT_, MF_>(lds, tw, P);
  }
};

// all D_ components of a W_-column tile side by side in one LDS tile
// ([row][component][column]) and transformed by one call, so the block's
// threads share the stages of every component and its loads are issued together
template <class SP, int NTRIAL, int W_, int D_, int NT_, bool MF_ = false>
struct ColStatCP {
  static constexpr int NT = NT_;
  static constexpr int CP = D_;
  static constexpr bool PRE = false;
  static constexpr int WC = W_;
  static constexpr int NF = SP::n;
  static constexpr int WPE = 1;
  static constexpr int SL = (D_ == 2) ? 1 : 2;   // the layout cells with D_ components use
  static constexpr int RL = (SL == 1) ? odd_rowlen(D_ * W_) : D_ * W_;
  __device__ static constexpr int W(int) { return W_; }
  __device__ static constexpr int nfft(int) { return SP::n; }
  __device__ static constexpr int ntrial(int) { return NTRIAL; }
  __device__ static constexpr int rowlen(int) { return RL; }
  template <class T, int S>
  __device__ __forceinline__ static void fft_rows(cpx<T>* lds, const FftPlan& P, int,
                                                  const cpx<T>* tw) {
    sfft<T, S, SP, D_ * W_, true, 1, RL, NT_, MF_>(lds, tw, P);
  }
};

struct RowGen {
  static constexpr int NT = kThreads;
  static constexpr bool ILV = false;
  // loads per thread in flight in the load / store phases for n elements (the
  // generic FP64 kernel, already short of registers, keeps one)
  template <class T>
  static constexpr int CH(int) { return (sizeof(T) == 8) ? 1 : 8; }
  static constexpr int NN = 0, HH = 0, DD = 0, RPP = 0;   // sizes known at compile time
  __device__ static int D(int d) { return d; }
  __device__ static int RP(int rp) { return rp; }
  __device__ static int n(int n_) { return n_; }
  __device__ static int H(int h) { return h; }
  __device__ static int ls(int len) { return len; }
  template <class T, int S>
  __device__ static void fft(cpx<T>* lds, const FftPlan& P, int lines, int ls_, const cpx<T>* tw) {
    line_fft<T, S>(lds, P, LdsLines{lines, ls_, 1, false}, tw);
  }
};

template <class SP, int NTRIAL, int D_, int RP_, int NT_, bool MF_ = false, bool ILV_ = false>
struct RowStat {
  static constexpr int NT = NT_;
  // one-dimensional grid with the items of a row tile on consecutive
  // workgroups: they run together, so the coefficient rows they share come
  // from the cache after the first read
  static constexpr bool ILV = ILV_;
  template <class T>
  static constexpr int CH(int n) { return rounds_ch(n, NT_); }
  static constexpr int NN = SP::n, HH = (NTRIAL + 1) / 2, DD = D_, RPP = RP_;
  __device__ static constexpr int D(int) { return D_; }
  __device__ static constexpr int RP(int) { return RP_; }
  __device__ static constexpr int n(int) { return SP::n; }
  __device__ static constexpr int H(int) { return (NTRIAL + 1) / 2; }
  __device__ static constexpr int ls(int) { return SP::len; }
  template <class T, int S>
  __device__ __forceinline__ static void fft(cpx<T>* lds, const FftPlan& P, int, int,
                                             const cpx<T>* tw) {
    sfft<T, S, SP, D_ * RP_, false, SP::len, 1, NT_, MF_>(lds, tw, P);
  }
};

__device__ __forceinline__ int kof(int i, int n) { return (i <= (n - 1) / 2) ? i : i - n; }
__device__ __forceinline__ int posk(int k, int n) { return k < 0 ? k + n : k; }

// unit normal n(k) = xi / |xi| (0 at k = 0), split into the part that depends
// on the column only (column index -> (k1, h) in 3-D, h in 2-D), evaluated once
// per column, and the axis-0 wavenumber k0 of each position
template <class T>
struct ColXi {
  T x1, x2, c;   // xi_1, xi_2, xi_1^2 + xi_2^2
};

template <class T>
__device__ __forceinline__ ColXi<T> col_xi(const NormalGeo& g, int col) {
  T xi1, xi2 = T(0);
  if (g.d == 3) {
    const int k1 = kof(col / g.H, g.N1);
    const int h = col % g.H;
    xi1 = T(k1) * T(g.invY[1]);
    xi2 = T(h) * T(g.invY[2]);
  } else {
    xi1 = T(col) * T(g.invY[1]);
  }
  return ColXi<T>{xi1, xi2, xi1 * xi1 + xi2 * xi2};
}

__device__ __forceinline__ float inv_sqrt(float s) { return rsqrtf(s); }
__device__ __forceinline__ double inv_sqrt(double s) { return 1.0 / sqrt(s); }

// component comp of n(k) (only the components a pass uses are formed, so a
// compiler hoisting them out of the component loop keeps few registers live)
template <class T>
__device__ __forceinline__ T normal_comp(const NormalGeo& g, int k0, const ColXi<T>& cx, int comp) {
  const T xi0 = T(k0) * T(g.invY[0]);
  const T s = xi0 * xi0 + cx.c;
  const T inv = s > T(0) ? inv_sqrt(s) : T(0);
  // dual (2-D): the divergence-free fields of frequency k are the multiples of
  // t = (-xi_1, xi_0) / |xi|, the primal ones of n = xi / |xi|
  if (g.dual) return (comp == 0 ? -cx.x1 : xi0) * inv;
  return (comp == 0 ? xi0 : comp == 1 ? cx.x1 : cx.x2) * inv;
}

// 3-D dual problem: the divergence-free fields of frequency k != 0 are
// t_1 c_1 + t_2 c_2 with t_1, t_2 an orthonormal basis of the plane
// orthogonal to xi.  With j the axis of the smallest |xi_j| (the first on
// ties, decided in FP64 so that both precisions take the same basis):
// t_1 = e_j x xi / |e_j x xi| and t_2 = n x t_1 = (|xi|^2 e_j - xi_j xi) /
// (|xi| |e_j x xi|).  t_1 is odd and t_2 even in k, so the two potentials of
// a real field keep fixed symmetries.  Component comp of t_(pot+1); 0 at k = 0.
template <class T>
__device__ __forceinline__ T dual3_comp(const NormalGeo& g, int k0, int col, int comp, int pot) {
  const int k1 = kof(col / g.H, g.N1), h = col % g.H;
  const double d0 = fabs(k0 * g.invY[0]), d1 = fabs(k1 * g.invY[1]), d2 = fabs(h * g.invY[2]);
  const int j = (d0 <= d1 && d0 <= d2) ? 0 : (d1 <= d2) ? 1 : 2;
  const T x0 = T(k0 * g.invY[0]), x1 = T(k1 * g.invY[1]), x2 = T(h * g.invY[2]);
  const T s = x0 * x0 + x1 * x1 + x2 * x2;
  const T xj = (j == 0) ? x0 : (j == 1) ? x1 : x2;
  const T m = s - xj * xj;
  if (!(m > T(0))) return T(0);
  const T xc = (comp == 0) ? x0 : (comp == 1) ? x1 : x2;
  if (pot == 0) {
    // (e_j x xi)_c = eps_(c j l) xi_l with l the third axis
    if (comp == j) return T(0);
    const int l = 3 - j - comp;
    const T xl = (l == 0) ? x0 : (l == 1) ? x1 : x2;
    return ((j == (comp + 1) % 3) ? xl : -xl) * inv_sqrt(m);
  }
  return ((comp == j ? s : T(0)) - xc * xj) * inv_sqrt(s * m);
}

// Elasticity: the compatible strains of frequency k != 0 are the Mandel
// vectors of sym(xi (x) u), u in C^d.  With K = (|xi|^2 I + xi xi^T) / 2
// (|sym(xi (x) u)|^2 = u^T K u), the columns b_p = sym(xi (x) K^-1/2 e_p),
// K^-1/2 = (sqrt 2 (I - n n^T) + n n^T) / |xi|, are an orthonormal basis;
// in terms of n = xi / |xi| alone:
//   b_p[aa] = sqrt 2 n_a [a = p] + (1 - sqrt 2) n_p n_a^2,
//   b_p[ab] = n_a [b = p] + n_b [a = p] + (sqrt 2 - 2) n_p n_a n_b  (a != b),
// Mandel order 11, 22, (33, 23, 13,) 12.  Every b_p is odd in k.  Component
// comp of b_pot; 0 at k = 0.
template <class T>
__device__ __forceinline__ T elastic_comp(const NormalGeo& g, int k0, int col, int comp, int pot) {
  T x[3] = {T(k0 * g.invY[0]), T(0), T(0)};
  if (g.d == 3) {
    x[1] = T(kof(col / g.H, g.N1) * g.invY[1]);
    x[2] = T((col % g.H) * g.invY[2]);
  } else {
    x[1] = T(col * g.invY[1]);
  }
  const T s = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  if (!(s > T(0))) return T(0);
  const T r = inv_sqrt(s);
  const T n[3] = {x[0] * r, x[1] * r, x[2] * r};
  // Mandel pair (a, b) of component comp
  int a, b;
  if (g.d == 2) {
    a = (comp == 1) ? 1 : 0;
    b = (comp == 0) ? 0 : 1;
  } else {
    a = (comp < 3) ? comp : (comp == 3) ? 1 : 0;
    b = (comp < 3) ? comp : (comp == 5) ? 1 : 2;
  }
  const T sq2 = T(1.4142135623730951);
  if (a == b) return (a == pot ? sq2 * n[a] : T(0)) + (T(1) - sq2) * n[pot] * n[a] * n[a];
  return (b == pot ? n[a] : T(0)) + (a == pot ? n[b] : T(0)) + (sq2 - T(2)) * n[pot] * n[a] * n[b];
}

// basis component of a cell with several potentials per frequency
template <class T>
__device__ __forceinline__ T pot_comp(const NormalGeo& g, int k0, int col, int comp, int pot) {
  return g.elastic ? elastic_comp<T>(g, k0, col, comp, pot) : dual3_comp<T>(g, k0, col, comp, pot);
}

// 1 / |xi| (0 at k = 0): in 3-D, xi_1 and xi_2 are constant along a first-axis
// line, so n_1 F[X_1] + n_2 F[X_2] = F[xi_1 X_1 + xi_2 X_2] / |xi| and the
// expansion's X_1, X_2 are xi_1, xi_2 times one transform of c / |xi|: the
// first-axis passes of 3-D cells run two transforms per tile instead of three
template <class T>
__device__ __forceinline__ T inv_xi(const NormalGeo& g, int k0, const ColXi<T>& cx) {
  const T xi0 = T(k0) * T(g.invY[0]);
  const T s = xi0 * xi0 + cx.c;
  return s > T(0) ? inv_sqrt(s) : T(0);
}

template <int NT>
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[NT / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (wid == 0) {
    v = (lane < NT / 64) ? red[lane] : 0.0;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  }
  __syncthreads();
  return v;
}

// Fixed-order sum of nparts partials, computed by every wave on its own: lane l
// adds p[l], p[l + 64], p[l + 128], ... in turn (eight loads in flight at a
// time), then the 64 lane sums meet in a butterfly, which leaves the same value
// in every lane (each pairwise addition sees the same two operands on both
// sides).  Every workgroup that needs a CG scalar derives it identically,
// whatever its size, and without a barrier.  Split in two so that a kernel can
// issue the first eight loads per lane (partials_head) ahead of its own loads
// and add them up afterwards (partials_finish).
__device__ __forceinline__ void partials_head(const double* p, int nparts, double* t) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int u = 0; u < 8; ++u) t[u] = p[max(min(lane + u * 64, nparts - 1), 0)];
}

__device__ __forceinline__ double partials_finish(const double* p, int nparts, const double* t) {
  const int lane = threadIdx.x & 63;
  double v = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u) v += (lane + u * 64 < nparts) ? t[u] : 0.0;
  for (int i0 = lane + 8 * 64; i0 < nparts; i0 += 8 * 64) {
    double r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) r[u] = (i0 + u * 64 < nparts) ? p[i0 + u * 64] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) v += r[u];
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double sum_partials_wave(const double* p, int nparts) {
  double t[8];
  partials_head(p, nparts, t);
  return partials_finish(p, nparts, t);
}

// f = threadIdx.x + k NT for every f < n, in rounds of CH per thread: a round
// issues all of its loads (ld) before the first use (use), so a thread keeps CH
// memory requests in flight instead of waiting for each in turn.  The loads are
// unconditional (an index past the end reads element n - 1 again, unused):
// a load under a branch is waited for inside that branch.  Callers that know
// n at compile time pass CH no larger than the rounds n needs (rounds_ch).
template <int NT, int CH, class Ld, class Use>
__device__ __forceinline__ void in_rounds(int n, const Ld& ld, const Use& use) {
  using V = decltype(ld(0));
  for (int f0 = threadIdx.x; f0 < n; f0 += CH * NT) {
    V v[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) v[u] = ld(min(f0 + u * NT, n - 1));
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (f0 + u * NT < n) use(f0 + u * NT, v[u]);
  }
}

template <class T>
struct cpx2 {
  cpx<T> a, b;
};

// CG bookkeeping of one completed update from the sum s = (r, r): iteration
// count, stopping test (relative residual or budget), beta and rho; a stop
// raises `halt`.  One thread of one workgroup per item runs it, in a kernel
// whose other workgroups do not read these fields.
__device__ __forceinline__ void cg_book(ItemScal& q, double s) {
  q.iters += 1;
  if (!isfinite(s)) {
    q.status = -5;
    q.halt = 1;
    return;
  }
  // beta is kept also when the item stops: a residual replacement of the
  // mixed solver rescales it and carries the search direction on
  q.beta = s / q.rho;
  if (sqrt(s / q.rho0) <= q.tol) {
    q.conv = 1;
    q.halt = 1;
  } else if (q.iters >= q.max_iter) {
    q.halt = 1;
  }
  q.rho = s;
}

// (p, q) of this iteration from the last-axis pass's partials, summed in
// fixed order by the first wave of a projection's workgroup 0 for the update
// of the same iteration (no workgroup of the projection reads it)
__device__ __forceinline__ void pq_total(ItemScal& q, const double* part, int n) {
  if (threadIdx.x >= 64) return;
  const double s = sum_partials_wave(part, n);
  if (threadIdx.x == 0) q.pq = s;
}

// the decision cg_book will take, derived by every workgroup of the next
// expansion: 1 if the item stops after its last update
__device__ __forceinline__ bool cg_stops(const ItemScal& q, double s) {
  return !isfinite(s) || sqrt(s / q.rho0) <= q.tol || q.iters + 1 >= q.max_iter;
}

// ---------------------------------------------------------------------------
// axis 0 from the scalar potential: X_a = F_0^-1 Pad(n_a c) for every
// component a
// ---------------------------------------------------------------------------
template <class T, class P, int PMAX>
__global__ __launch_bounds__(P::NT, P::WPE) void k_col_expand(ColExpandArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int NT = P::NT;
  const int item = blockIdx.y;
  if (a.sc && !item_live(a.sc[item])) return;
  const int W = P::W(a.W), n_in = P::ntrial(a.n_in), n_fft = P::nfft(a.n_fft);
  const int col0 = xcd_tile(blockIdx.x, gridDim.x) * W;
  const int ncols = min(W, a.inner - col0);
  const long ibase = (long)item * a.c_stride;
  const int npos = n_in * W;
  const bool colm = (P::SL == 0) ? (a.si == 1) : (P::SL == 1);
  // position it of this thread: (i, w) of the tile; with column-major scalars
  // axis 0 runs across the threads (contiguous loads), else the tile columns do
  auto pos = [=](int it, int& i, int& w) __attribute__((always_inline)) {
    const int f = threadIdx.x + it * NT;
    i = colm ? f % n_in : f / W;
    w = colm ? f / n_in : f % W;
    return f < npos;
  };
  // every load goes out first (unconditional: positions outside the tile read
  // an element inside it again); positions outside the tile contribute 0
  cpx<T> s[PMAX];
#pragma unroll
  for (int it = 0; it < PMAX; ++it) {
    int i, w;
    pos(it, i, w);
    s[it] = a.c[ibase + (long)min(i, n_in - 1) * a.si + (long)(col0 + min(w, ncols - 1)) * a.sc_];
  }
#pragma unroll
  for (int it = 0; it < PMAX; ++it) {
    int i, w;
    if (!pos(it, i, w) || w >= ncols) s[it] = cpx<T>{T(0), T(0)};
  }
  // with row-major positions and NT a multiple of the tile width every
  // position of a thread lies in the same column: its part of xi is evaluated once
  constexpr bool col_fixed = (P::SL == 2) && P::WC > 0 && (NT % P::WC) == 0;
  ColXi<T> cx0{};
  if (col_fixed) cx0 = col_xi<T>(a.g, min(col0 + (int)threadIdx.x % W, a.inner - 1));
  // components in groups of P::CP per transform; LDS tile [row][comp][column]
  constexpr int CPN = P::CP;
  const int LW = P::rowlen(CPN * W);
  // 3-D, one component per transform: transform 0 gives X_0, transform 1 the
  // common part of X_1 and X_2 (see inv_xi)
  // (known at compile time where the scalar layout is: row-major = 3-D)
  constexpr int FOLD = (CPN != 1 || P::SL == 1) ? 0 : (P::SL == 2) ? 1 : -1;
  const bool fold = (FOLD == 1) || (FOLD == -1 && a.g.d == 3);
  const int ntr = fold ? 2 : a.g.nf;
#pragma unroll 1
  for (int al0 = 0; al0 < ntr; al0 += CPN) {
    constexpr int nc = CPN;   // CP > 1 kernels serve only cells with CP components
    if (n_fft != n_in) {
      for (int f = threadIdx.x; f < n_fft * LW; f += NT) lds[f] = cpx<T>{T(0), T(0)};
      __syncthreads();
    }
#pragma unroll
    for (int it = 0; it < PMAX; ++it) {
      int i, w;
      if (pos(it, i, w)) {
        const int row = (n_fft == n_in) ? i : posk(kof(i, n_in), n_fft);
        const ColXi<T> cx = col_fixed ? cx0 : col_xi<T>(a.g, min(col0 + w, a.inner - 1));
        if (fold) {
          const T iv = inv_xi<T>(a.g, kof(i, n_in), cx);
          lds[row * LW + w] = cscale(s[it], al0 == 0 ? T(kof(i, n_in)) * T(a.g.invY[0]) * iv : iv);
        } else {
          for (int c = 0; c < nc; ++c)
            lds[row * LW + c * W + w] = cscale(s[it], normal_comp<T>(a.g, kof(i, n_in), cx, al0 + c));
        }
      }
    }
    __syncthreads();
    P::template fft_rows<T, +1>(lds, a.plan, W, a.tw);
    cpx<T>* X = a.X + (long)item * a.X_stride + (long)al0 * a.X_cstride;
    if (fold && al0 == 1) {
      // xi_1 Z into X_1 and xi_2 Z into X_2
      in_rounds<NT, rounds_ch(P::NF * P::WC * P::CP, NT)>(
          n_fft * W,
          [=](int f) __attribute__((always_inline)) { return lds[(f / W) * LW + f % W]; },
          [=](int f, const cpx<T>& v) __attribute__((always_inline)) {
            const int w = f % W, i = f / W;
            if (w >= ncols) return;
            const ColXi<T> cx = col_fixed ? cx0 : col_xi<T>(a.g, col0 + w);
            const long e = (long)i * a.inner + col0 + w;
            X[e] = cscale(v, cx.x1);
            X[e + a.X_cstride] = cscale(v, cx.x2);
          });
    } else {
      in_rounds<NT, rounds_ch(P::NF * P::WC * P::CP, NT)>(
          n_fft * W * nc,
          [=](int f) __attribute__((always_inline)) {
            const int w = f % W, t = f / W, c = t % nc, i = t / nc;
            return lds[i * LW + c * W + w];
          },
          [=](int f, const cpx<T>& v) __attribute__((always_inline)) {
            const int w = f % W, t = f / W, c = t % nc, i = t / nc;
            if (w < ncols) X[(long)c * a.X_cstride + (long)i * a.inner + col0 + w] = v;
          });
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// plain pass along a middle axis: inverse with zero padding (trial -> fft
// length) or forward with truncation (fft length -> trial), per component
// ---------------------------------------------------------------------------
template <class T, class P, int S>
__global__ __launch_bounds__(P::NT, P::WPE) void k_col_plain(ColPlainArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int NT = P::NT;
  const int item = blockIdx.z / a.d, comp = blockIdx.z % a.d;
  if (a.sc && !item_live(a.sc[item])) return;
  const int W = P::W(a.W), n_fft = P::nfft(a.n_fft);
  const int n_in = (S > 0) ? P::ntrial(a.n_in) : P::nfft(a.n_in);
  const int n_out = (S > 0) ? P::nfft(a.n_out) : P::ntrial(a.n_out);
  const int o = blockIdx.y;
  const int col0 = xcd_tile(blockIdx.x, gridDim.x) * W;
  const int ncols = min(W, a.inner - col0);
  const cpx<T>* in = a.in + (long)item * a.in_stride + (long)comp * a.in_cstride +
                     (long)o * n_in * a.inner + col0;
  cpx<T>* out = a.out + (long)item * a.out_stride + (long)comp * a.out_cstride +
                (long)o * n_out * a.inner + col0;
  if (n_in != n_fft) {
    for (int f = threadIdx.x; f < n_fft * W; f += NT) lds[f] = cpx<T>{T(0), T(0)};
    __syncthreads();
  }
  in_rounds<NT, rounds_ch(P::NF * P::WC * P::CP, NT)>(
      n_in * W,
      [=](int f) __attribute__((always_inline)) {
        const int i = f / W, w = f % W;
        return in[(long)i * a.inner + min(w, ncols - 1)];
      },
      [=](int f, const cpx<T>& v) __attribute__((always_inline)) {
        const int i = f / W, w = f % W;
        const int rrow = (n_in == n_fft) ? i : posk(kof(i, n_in), n_fft);
        lds[rrow * W + w] = (w < ncols) ? v : cpx<T>{T(0), T(0)};
      });
  __syncthreads();
  P::template fft<T, S>(lds, a.plan, W, a.tw);
  in_rounds<NT, rounds_ch(P::NF * P::WC * P::CP, NT)>(
      n_out * W,
      [=](int f) __attribute__((always_inline)) {
        const int i = f / W, w = f % W;
        const int rrow = (n_out == n_fft) ? i : posk(kof(i, n_out), n_fft);
        return lds[rrow * W + w];
      },
      [=](int f, const cpx<T>& v) __attribute__((always_inline)) {
        const int i = f / W, w = f % W;
        if (w < ncols) out[(long)i * a.inner + w] = cscale(v, a.scale);
      });
}

// ---------------------------------------------------------------------------
// plain column pass of a two-stage plan (n = R1 R2) with the first stage's
// operands loaded from global memory straight into registers and the second
// stage's results stored straight to global memory: one LDS exchange and one
// barrier per tile instead of the four round trips of the LDS-staged pass.
// Lanes take consecutive columns of the tile, so both the loads and the
// stores of a wave cover whole row segments.
// ---------------------------------------------------------------------------
template <class R_>
struct TwoRadices;
template <int A, int B>
struct TwoRadices<Rad<A, B>> {
  static constexpr int r1 = A, r2 = B;
};

template <class T, class SP, int NTRIAL, int W, int NT, int S>
__global__ __launch_bounds__(NT) void k_col_reg2(ColPlainArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int R1 = TwoRadices<typename SP::radices>::r1, R2 = TwoRadices<typename SP::radices>::r2;
  constexpr int n = SP::n;
  static_assert(R1 * R2 == n && !SP::blue, "two-stage Stockham plan");
  // inverse: trial rows in, padded to n; forward: n rows in, truncated to trial
  constexpr int n_in = (S > 0) ? NTRIAL : n, n_out = (S > 0) ? n : NTRIAL;
  constexpr int hk = (NTRIAL - 1) / 2;   // |k| of the trial frequencies
  const int item = blockIdx.z / a.d, comp = blockIdx.z % a.d;
  if (a.sc && !item_live(a.sc[item])) return;
  const int o = blockIdx.y;
  const int col0 = xcd_tile(blockIdx.x, gridDim.x) * W;
  const int ncols = min(W, a.inner - col0);
  const cpx<T>* in = a.in + (long)item * a.in_stride + (long)comp * a.in_cstride +
                     (long)o * n_in * a.inner + col0;
  cpx<T>* out = a.out + (long)item * a.out_stride + (long)comp * a.out_cstride +
                (long)o * n_out * a.inner + col0;
  // stage 1 (no twiddles): butterfly (w, j), j < R2, operands at rows j + r R2
  constexpr int T1 = R2 * W, M1 = (T1 + NT - 1) / NT;
  cpx<T> v[M1][R1];
#pragma unroll
  for (int it = 0; it < M1; ++it) {
    const int f = min((int)threadIdx.x + it * NT, T1 - 1);
    const int w = min(f % W, ncols - 1), j = f / W;
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const int t = j + r * R2;
      if constexpr (n_in == n) {
        v[it][r] = in[(long)t * a.inner + w];
      } else {
        const int k = kof(t, n);
        const bool trial = (k >= -hk && k <= hk);
        const cpx<T> x = in[(long)(trial ? posk(k, NTRIAL) : 0) * a.inner + w];
        v[it][r] = trial ? x : cpx<T>{T(0), T(0)};
      }
    }
  }
#pragma unroll
  for (int it = 0; it < M1; ++it) {
    const int f = (int)threadIdx.x + it * NT;
    if (f < T1) {
      const int w = f % W, j = f / W;
      Dft<T, R1, S>::run(v[it]);
#pragma unroll
      for (int r = 0; r < R1; ++r) lds[(j * R1 + r) * W + w] = v[it][r];
    }
  }
  __syncthreads();
  // stage 2 (Ns = R1): butterfly (w, k), k < R1, operands at rows k + r R1,
  // twiddles of the plan's second stage, results at rows k + r R1
  constexpr int T2 = R1 * W, M2 = (T2 + NT - 1) / NT;
#pragma unroll
  for (int it = 0; it < M2; ++it) {
    const int f = (int)threadIdx.x + it * NT;
    if (f >= T2) continue;
    const int w = f % W, k = f / W;
    cpx<T> u[R2];
#pragma unroll
    for (int r = 0; r < R2; ++r) u[r] = lds[(k + r * R1) * W + w];
#pragma unroll
    for (int r = 1; r < R2; ++r) {
      cpx<T> tw = a.tw[k * (R2 - 1) + r - 1];
      if (S > 0) tw.y = -tw.y;
      u[r] = cmul(u[r], tw);
    }
    Dft<T, R2, S>::run(u);
    if (w >= ncols) continue;
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      const int t = k + r * R1;
      if constexpr (n_out == n) {
        out[(long)t * a.inner + w] = cscale(u[r], a.scale);
      } else {
        const int kk = kof(t, n);
        if (kk >= -hk && kk <= hk) out[(long)posk(kk, NTRIAL) * a.inner + w] = cscale(u[r], a.scale);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// first-axis passes of 3-D cells (one potential, row-major scalars: element
// (i, column) at i si + column) with the
// register pipeline of k_col_reg2: per tile two transforms (see inv_xi), each
// with its first-stage operands taken from registers and its second-stage
// results kept in registers, one LDS exchange per transform.  The thread of
// first-stage butterfly (w, j) and of second-stage butterfly (w, k) works on
// tile column w = threadIdx.x mod W throughout (NT a multiple of W), so its
// part of xi is evaluated once.
// ---------------------------------------------------------------------------
// PAIR: the expansion leaves Z in place of X_1 and nothing in X_2, and the
// projection reads xi_1 X_1 + xi_2 X_2, already combined, in place of X_1: the
// middle-axis passes of such cells apply xi_1 and xi_2 (k_col_mid2)
template <class T, class SP, int NTRIAL, int W, int NT, bool PAIR = false>
__global__ __launch_bounds__(NT) void k_col_expand_r2(ColExpandArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int R1 = TwoRadices<typename SP::radices>::r1, R2 = TwoRadices<typename SP::radices>::r2;
  constexpr int n = SP::n;
  static_assert(R1 * R2 == n && !SP::blue, "two-stage Stockham plan");
  static_assert(NT % W == 0, "a thread keeps one tile column");
  constexpr int hk = (NTRIAL - 1) / 2;   // |k| of the trial frequencies
  const int item = blockIdx.y;
  if (a.sc && !item_live(a.sc[item])) return;
  const int col0 = xcd_tile(blockIdx.x, gridDim.x) * W;
  const int ncols = min(W, a.inner - col0);
  const int w = (int)threadIdx.x % W;
  const int wl = min(w, ncols - 1);   // loads of columns past the edge read the last one
  const cpx<T>* c = a.c + (long)item * a.c_stride + col0 + wl;
  cpx<T>* X = a.X + (long)item * a.X_stride + col0 + w;
  const ColXi<T> cx = col_xi<T>(a.g, col0 + wl);
  const T y0 = T(a.g.invY[0]);
  // c / |xi| at the first-stage operand rows t = j + r R2 of every butterfly
  // of this thread (0 outside the trial frequencies)
  constexpr int T1 = R2 * W, M1 = (T1 + NT - 1) / NT;
  cpx<T> pv[M1][R1];
#pragma unroll
  for (int it = 0; it < M1; ++it) {
    const int j = min((int)threadIdx.x + it * NT, T1 - 1) / W;
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const int k = kof(j + r * R2, n);
      const bool trial = (k >= -hk && k <= hk);
      const cpx<T> x = c[(long)(trial ? posk(k, NTRIAL) : 0) * a.si];
      pv[it][r] = trial ? cscale(x, inv_xi<T>(a.g, k, cx)) : cpx<T>{T(0), T(0)};
    }
  }
  constexpr int T2 = R1 * W, M2 = (T2 + NT - 1) / NT;
  // transform 0: xi_0 c / |xi| (X_0); transform 1: c / |xi| (X_1, X_2 = xi_1,
  // xi_2 times it).  Unrolled: as a loop, the compiler keeps the twiddles and
  // addresses it hoists out of it live across both transforms (~190 VGPRs
  // against ~125)
#pragma unroll
  for (int tr = 0; tr < 2; ++tr) {
#pragma unroll
    for (int it = 0; it < M1; ++it) {
      const int f = (int)threadIdx.x + it * NT;
      if (f < T1) {
        const int j = f / W;
        cpx<T> u[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r)
          u[r] = (tr == 0) ? cscale(pv[it][r], T(kof(j + r * R2, n)) * y0) : pv[it][r];
        Dft<T, R1, +1>::run(u);
#pragma unroll
        for (int r = 0; r < R1; ++r) lds[(j * R1 + r) * W + w] = u[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < M2; ++it) {
      const int f = (int)threadIdx.x + it * NT;
      if (f >= T2) continue;
      const int k = f / W;
      cpx<T> u[R2];
#pragma unroll
      for (int r = 0; r < R2; ++r) u[r] = lds[(k + r * R1) * W + w];
#pragma unroll
      for (int r = 1; r < R2; ++r) {
        cpx<T> t = a.tw[k * (R2 - 1) + r - 1];
        t.y = -t.y;
        u[r] = cmul(u[r], t);
      }
      Dft<T, R2, +1>::run(u);
      if (w >= ncols) continue;
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const long e = (long)(k + r * R1) * a.inner;
        if (tr == 0) {
          X[e] = u[r];
        } else if (PAIR) {
          X[a.X_cstride + e] = u[r];
        } else {
          X[a.X_cstride + e] = cscale(u[r], cx.x1);
          X[2 * a.X_cstride + e] = cscale(u[r], cx.x2);
        }
      }
    }
    __syncthreads();
  }
}

template <class T, class SP, int NTRIAL, int W, int NT, bool PAIR = false>
__global__ __launch_bounds__(NT) void k_col_project_r2(ColProjectArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int R1 = TwoRadices<typename SP::radices>::r1, R2 = TwoRadices<typename SP::radices>::r2;
  constexpr int n = SP::n;
  static_assert(R1 * R2 == n && !SP::blue, "two-stage Stockham plan");
  static_assert(NT % W == 0, "a thread keeps one tile column");
  constexpr int hk = (NTRIAL - 1) / 2;
  const int item = blockIdx.y;
  if (a.sc && !item_live_project(a.sc[item])) {
    // an item whose update broke down stops here: the first workgroup raises
    // halt for the update of this iteration (no workgroup here reads it)
    const ItemScal& q0 = a.sc[item];
    if (q0.active && q0.broke && a.rr_part && blockIdx.x == 0 && threadIdx.x == 0)
      a.sc[item].halt = 1;
    return;
  }
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int col0 = tile * W;
  const int ncols = min(W, a.inner - col0);
  const int w = (int)threadIdx.x % W;
  const int wl = min(w, ncols - 1);
  const cpx<T>* X = a.X + (long)item * a.X_stride + col0 + wl;
  const ColXi<T> cx = col_xi<T>(a.g, col0 + wl);
  const T y0 = T(a.g.invY[0]);
  constexpr int T1 = R2 * W, M1 = (T1 + NT - 1) / NT;
  constexpr int T2 = R1 * W, M2 = (T2 + NT - 1) / NT;
  // xi_0 F[X_0] + F[xi_1 X_1 + xi_2 X_2] at the second-stage result rows
  cpx<T> acc[M2][R2];
#pragma unroll
  for (int it = 0; it < M2; ++it)
#pragma unroll
    for (int r = 0; r < R2; ++r) acc[it][r] = cpx<T>{T(0), T(0)};
#pragma unroll
  for (int tr = 0; tr < 2; ++tr) {
#pragma unroll
    for (int it = 0; it < M1; ++it) {
      const int f = (int)threadIdx.x + it * NT;
      const int j = min(f, T1 - 1) / W;
      cpx<T> u[R1];
      if (tr == 0 || PAIR) {
#pragma unroll
        for (int r = 0; r < R1; ++r) u[r] = X[tr * a.X_cstride + (long)(j + r * R2) * a.inner];
      } else {
        cpx<T> u2[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) {
          u[r] = X[a.X_cstride + (long)(j + r * R2) * a.inner];
          u2[r] = X[2 * a.X_cstride + (long)(j + r * R2) * a.inner];
        }
#pragma unroll
        for (int r = 0; r < R1; ++r)
          u[r] = cpx<T>{cx.x1 * u[r].x + cx.x2 * u2[r].x, cx.x1 * u[r].y + cx.x2 * u2[r].y};
      }
      if (f < T1) {
        Dft<T, R1, -1>::run(u);
#pragma unroll
        for (int r = 0; r < R1; ++r) lds[(j * R1 + r) * W + w] = u[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < M2; ++it) {
      const int f = (int)threadIdx.x + it * NT;
      if (f >= T2) continue;
      const int k = f / W;
      cpx<T> u[R2];
#pragma unroll
      for (int r = 0; r < R2; ++r) u[r] = lds[(k + r * R1) * W + w];
#pragma unroll
      for (int r = 1; r < R2; ++r) u[r] = cmul(u[r], a.tw[k * (R2 - 1) + r - 1]);
      Dft<T, R2, -1>::run(u);
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const T f0 = (tr == 0) ? T(kof(k + r * R1, n)) * y0 : T(1);
        acc[it][r].x += f0 * u[r].x;
        acc[it][r].y += f0 * u[r].y;
      }
    }
    __syncthreads();
  }
  // epilogue at the trial rows among this thread's result rows t = k + r R1;
  // its loads (p for (p, q), b for the residual) all go out first
  const long sb = (long)item * a.s_stride + col0 + wl;
  const cpx<T>* ld = (a.epi == EPI_STORE) ? a.p : (a.epi == EPI_RESID) ? a.b : nullptr;
  cpx<T> lv[M2][R2];
#pragma unroll
  for (int it = 0; it < M2; ++it) {
    const int k = min((int)threadIdx.x + it * NT, T2 - 1) / W;
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      const int kk = kof(k + r * R1, n);
      const bool trial = (kk >= -hk && kk <= hk);
      lv[it][r] = cpx<T>{T(0), T(0)};
      if (ld) lv[it][r] = ld[sb + (long)(trial ? posk(kk, NTRIAL) : 0) * a.si];
    }
  }
  // Hermitian weight of the column: 1 on the h = 0 plane, else 2
  const double wt = (((col0 + w) % a.g.H) == 0) ? 1.0 : 2.0;
  double part = 0.0;
#pragma unroll
  for (int it = 0; it < M2; ++it) {
    const int f = (int)threadIdx.x + it * NT;
    const int k = min(f, T2 - 1) / W;
    const bool live = (f < T2) && (w < ncols);
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      const int kk = kof(k + r * R1, n);
      if (!live || kk < -hk || kk > hk) continue;
      const long idx = sb + (long)posk(kk, NTRIAL) * a.si;
      const cpx<T> qv = cscale(cscale(acc[it][r], a.scale), inv_xi<T>(a.g, kk, cx));
      if (a.epi == EPI_STORE) {
        a.q[idx] = qv;
        if (a.p) part += wt * ((double)lv[it][r].x * (double)qv.x + (double)lv[it][r].y * (double)qv.y);
      } else if (a.epi == EPI_RHS) {
        const cpx<T> mq = cpx<T>{-qv.x, -qv.y};
        a.q[idx] = mq;
        if (a.r) a.r[idx] = mq;
        if (a.pp) a.pp[idx] = mq;
        if (a.x) a.x[idx] = cpx<T>{T(0), T(0)};
        part += wt * ((double)mq.x * (double)mq.x + (double)mq.y * (double)mq.y);
      } else {  // EPI_RESID: r = b - q
        const cpx<T> rv = cpx<T>{lv[it][r].x - qv.x, lv[it][r].y - qv.y};
        a.r[idx] = rv;
        part += wt * ((double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y);
      }
    }
  }
  if (a.partials) {
    part = block_sum<NT>(part);
    if (threadIdx.x == 0) a.partials[(long)item * a.P + tile] = part;
  }
  if (a.rr_part && blockIdx.x == 0) {
    // bookkeeping of the update before this iteration's expansion (that
    // expansion has finished reading rho; no other workgroup here reads it)
    const bool fresh = a.sc[item].fresh != 0;
    const double s = fresh ? 0.0 : sum_partials_wave(a.rr_part + (long)item * a.P, a.rr_n);
    if (threadIdx.x == 0) {
      if (fresh) a.sc[item].fresh = 0;
      else cg_book(a.sc[item], s);
    }
  }
  if (a.pq_part && blockIdx.x == 0) pq_total(a.sc[item], a.pq_part + (long)item * a.P, a.pq_n);
}

// ---------------------------------------------------------------------------
// 3-D elasticity, first-axis expansion with the basis map fused in (register
// pipeline): the three displacement potentials of a tile column are loaded
// once into registers, and each of the six Mandel components
//   b_p[aa] = sqrt 2 n_a [a = p] + (1 - sqrt 2) n_p n_a^2,
//   b_p[ab] = n_a [b = p] + n_b [a = p] + (sqrt 2 - 2) n_p n_a n_b
// (see elastic_comp) is formed from them at the first-stage operand rows and
// transformed in turn: the potentials are read once and the components
// written once, where the basis map plus plain transform wrote and read the
// components in between
// ---------------------------------------------------------------------------
template <class T, class SP, int NTRIAL, int W, int NT>
__global__ __launch_bounds__(NT) void k_col_bexpand_r2(ColExpandArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int R1 = TwoRadices<typename SP::radices>::r1, R2 = TwoRadices<typename SP::radices>::r2;
  constexpr int n = SP::n;
  static_assert(R1 * R2 == n && !SP::blue, "two-stage Stockham plan");
  static_assert(NT % W == 0, "a thread keeps one tile column");
  constexpr int hk = (NTRIAL - 1) / 2;
  const int item = blockIdx.y;
  if (a.sc && !item_live(a.sc[item])) return;
  const int col0 = xcd_tile(blockIdx.x, gridDim.x) * W;
  const int ncols = min(W, a.inner - col0);
  const int w = (int)threadIdx.x % W;
  const int wl = min(w, ncols - 1);
  const cpx<T>* c = a.c + (long)item * a.c_stride + col0 + wl;
  cpx<T>* X = a.X + (long)item * a.X_stride + col0 + w;
  const ColXi<T> cx = col_xi<T>(a.g, col0 + wl);
  const T y0 = T(a.g.invY[0]);
  constexpr int T1 = R2 * W, M1 = (T1 + NT - 1) / NT;
  constexpr int T2 = R1 * W, M2 = (T2 + NT - 1) / NT;
  static_assert(M1 == 1, "one first-stage butterfly per thread");
  const int j = min((int)threadIdx.x, T1 - 1) / W;
  cpx<T> pv[3][R1];
#pragma unroll
  for (int r = 0; r < R1; ++r) {
    const int k = kof(j + r * R2, n);
    const bool trial = (k >= -hk && k <= hk);
    const long row = (long)(trial ? posk(k, NTRIAL) : 0) * a.si;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const cpx<T> x = c[p * a.g.pot_stride + row];
      pv[p][r] = trial ? x : cpx<T>{T(0), T(0)};
    }
  }
  const T sq2 = T(1.4142135623730951);
#pragma unroll 1
  for (int comp = 0; comp < 6; ++comp) {
    // Mandel pair (a, b) of the component: 11, 22, 33, 23, 13, 12
    const int ca = (comp < 3) ? comp : (comp == 3) ? 1 : 0;
    const int cb = (comp < 3) ? comp : (comp == 5) ? 1 : 2;
    if ((int)threadIdx.x < T1) {
      cpx<T> u[R1];
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int k = kof(j + r * R2, n);
        const T iv = inv_xi<T>(a.g, k, cx);
        const T nv[3] = {T(k) * y0 * iv, cx.x1 * iv, cx.x2 * iv};
        // n . u over the potentials
        const cpx<T> s = {nv[0] * pv[0][r].x + nv[1] * pv[1][r].x + nv[2] * pv[2][r].x,
                          nv[0] * pv[0][r].y + nv[1] * pv[1][r].y + nv[2] * pv[2][r].y};
        // selects, not indexing: the arrays stay in registers
        const T na = (ca == 0) ? nv[0] : (ca == 1) ? nv[1] : nv[2];
        const T nb = (cb == 0) ? nv[0] : (cb == 1) ? nv[1] : nv[2];
        const cpx<T> ua = (ca == 0) ? pv[0][r] : (ca == 1) ? pv[1][r] : pv[2][r];
        const cpx<T> ub = (cb == 0) ? pv[0][r] : (cb == 1) ? pv[1][r] : pv[2][r];
        if (ca == cb) {
          const T f = (T(1) - sq2) * na * na;
          u[r] = {sq2 * na * ua.x + f * s.x, sq2 * na * ua.y + f * s.y};
        } else {
          const T f = (sq2 - T(2)) * na * nb;
          u[r] = {na * ub.x + nb * ua.x + f * s.x, na * ub.y + nb * ua.y + f * s.y};
        }
      }
      Dft<T, R1, +1>::run(u);
#pragma unroll
      for (int r = 0; r < R1; ++r) lds[(j * R1 + r) * W + w] = u[r];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < M2; ++it) {
      const int f = (int)threadIdx.x + it * NT;
      if (f >= T2) continue;
      const int k = f / W;
      cpx<T> u[R2];
#pragma unroll
      for (int r = 0; r < R2; ++r) u[r] = lds[(k + r * R1) * W + w];
#pragma unroll
      for (int r = 1; r < R2; ++r) {
        cpx<T> t = a.tw[k * (R2 - 1) + r - 1];
        t.y = -t.y;
        u[r] = cmul(u[r], t);
      }
      Dft<T, R2, +1>::run(u);
      if (w >= ncols) continue;
#pragma unroll
      for (int r = 0; r < R2; ++r) X[comp * a.X_cstride + (long)(k + r * R1) * a.inner] = u[r];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// middle-axis (3-D axis 1) passes between PAIR first-axis passes, register
// pipeline as in k_col_reg2.  Inverse: part 0 transforms X_0; part 1 reads Z
// once and gives X_1 = F^-1[xi_1 Z] and X_2 = xi_2 F^-1[Z] (xi_1 varies along
// this axis, xi_2 = h / Y_2 is constant on a tile column).  Forward: part 0
// transforms X_0; part 1 gives xi_1 F[X_1] + xi_2 F[X_2] into the X_1 slot.
// The grid's z index is item * 2 + part.
// ---------------------------------------------------------------------------
template <class T, class SP, int NTRIAL, int W, int NT, int S>
__global__ __launch_bounds__(NT) void k_col_mid2(ColPlainArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int R1 = TwoRadices<typename SP::radices>::r1, R2 = TwoRadices<typename SP::radices>::r2;
  constexpr int n = SP::n;
  static_assert(R1 * R2 == n && !SP::blue, "two-stage Stockham plan");
  static_assert(NT % W == 0, "a thread keeps one tile column");
  constexpr int n_in = (S > 0) ? NTRIAL : n, n_out = (S > 0) ? n : NTRIAL;
  constexpr int hk = (NTRIAL - 1) / 2;
  const int item = blockIdx.z >> 1, part = blockIdx.z & 1;
  if (a.sc && !item_live(a.sc[item])) return;
  const int o = blockIdx.y;
  const int col0 = xcd_tile(blockIdx.x, gridDim.x) * W;
  const int ncols = min(W, a.inner - col0);
  const int w = (int)threadIdx.x % W;
  const int wl = min(w, ncols - 1);
  const cpx<T>* in = a.in + (long)item * a.in_stride + (long)o * n_in * a.inner + col0 + wl;
  cpx<T>* out = a.out + (long)item * a.out_stride + (long)o * n_out * a.inner + col0 + w;
  const T x1s = T(a.xi1_step), xi2 = T((col0 + wl) * a.xi2_step);
  const int ntr = part ? 2 : 1;
  constexpr int T1 = R2 * W, M1 = (T1 + NT - 1) / NT;
  constexpr int T2 = R1 * W, M2 = (T2 + NT - 1) / NT;
  // inverse: the trial rows of X_0 or Z at this thread's first-stage operand rows
  cpx<T> pv[M1][R1];
  if (S > 0) {
    const cpx<T>* src = in + (part ? a.in_cstride : 0);
#pragma unroll
    for (int it = 0; it < M1; ++it) {
      const int j = min((int)threadIdx.x + it * NT, T1 - 1) / W;
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int k = kof(j + r * R2, n);
        const bool trial = (k >= -hk && k <= hk);
        const cpx<T> x = src[(long)(trial ? posk(k, NTRIAL) : 0) * a.inner];
        pv[it][r] = trial ? x : cpx<T>{T(0), T(0)};
      }
    }
  }
  // forward, part 1: xi_1 F[X_1] + xi_2 F[X_2] at the second-stage result rows
  cpx<T> acc[M2][R2];
#pragma unroll
  for (int it = 0; it < M2; ++it)
#pragma unroll
    for (int r = 0; r < R2; ++r) acc[it][r] = cpx<T>{T(0), T(0)};
#pragma unroll
  for (int tr = 0; tr < 2; ++tr) {
    if (tr >= ntr) break;
#pragma unroll
    for (int it = 0; it < M1; ++it) {
      const int f = (int)threadIdx.x + it * NT;
      const int j = min(f, T1 - 1) / W;
      cpx<T> u[R1];
      if (S > 0) {
        // part 1, transform 0: xi_1 Z
#pragma unroll
        for (int r = 0; r < R1; ++r)
          u[r] = (part && tr == 0) ? cscale(pv[it][r], T(kof(j + r * R2, n)) * x1s) : pv[it][r];
      } else {
        const cpx<T>* src = in + (long)(part + tr) * a.in_cstride;
#pragma unroll
        for (int r = 0; r < R1; ++r) u[r] = src[(long)(j + r * R2) * a.inner];
      }
      if (f < T1) {
        Dft<T, R1, S>::run(u);
#pragma unroll
        for (int r = 0; r < R1; ++r) lds[(j * R1 + r) * W + w] = u[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < M2; ++it) {
      const int f = (int)threadIdx.x + it * NT;
      if (f >= T2) continue;
      const int k = f / W;
      cpx<T> u[R2];
#pragma unroll
      for (int r = 0; r < R2; ++r) u[r] = lds[(k + r * R1) * W + w];
#pragma unroll
      for (int r = 1; r < R2; ++r) {
        cpx<T> t = a.tw[k * (R2 - 1) + r - 1];
        if (S > 0) t.y = -t.y;
        u[r] = cmul(u[r], t);
      }
      Dft<T, R2, S>::run(u);
      if (S > 0) {
        if (w >= ncols) continue;
        // X_0 (part 0), X_1 (part 1, transform 0), X_2 = xi_2 F^-1[Z] (transform 1)
        cpx<T>* dst = out + (long)(part + tr) * a.out_cstride;
        const T sc = (part && tr == 1) ? xi2 : T(1);
#pragma unroll
        for (int r = 0; r < R2; ++r) dst[(long)(k + r * R1) * a.inner] = cscale(u[r], sc);
      } else if (part == 0) {
        if (w >= ncols) continue;
#pragma unroll
        for (int r = 0; r < R2; ++r) {
          const int kk = kof(k + r * R1, n);
          if (kk >= -hk && kk <= hk) out[(long)posk(kk, NTRIAL) * a.inner] = cscale(u[r], a.scale);
        }
      } else {
#pragma unroll
        for (int r = 0; r < R2; ++r) {
          const T fr = (tr == 0) ? T(kof(k + r * R1, n)) * x1s : xi2;
          acc[it][r].x += fr * u[r].x;
          acc[it][r].y += fr * u[r].y;
        }
      }
    }
    __syncthreads();
  }
  if (S < 0 && part) {
#pragma unroll
    for (int it = 0; it < M2; ++it) {
      const int f = (int)threadIdx.x + it * NT;
      if (f >= T2 || w >= ncols) continue;
      const int k = f / W;
      cpx<T>* dst = out + a.out_cstride;
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int kk = kof(k + r * R1, n);
        if (kk >= -hk && kk <= hk) dst[(long)posk(kk, NTRIAL) * a.inner] = cscale(acc[it][r], a.scale);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// axis 0 forward + truncation + projection q = n . F_0[X], CG epilogues
// ---------------------------------------------------------------------------
template <class T, class P, int PMAX>
__global__ __launch_bounds__(P::NT, P::WPE) void k_col_project(ColProjectArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int NT = P::NT;
  const int item = blockIdx.y;
  if (a.sc && !item_live_project(a.sc[item])) {
    // an item whose update broke down stops here: the first workgroup raises
    // halt for the update of this iteration (no workgroup here reads it)
    const ItemScal& q0 = a.sc[item];
    if (q0.active && q0.broke && a.rr_part && blockIdx.x == 0 && threadIdx.x == 0)
      a.sc[item].halt = 1;
    return;
  }
  const int W = P::W(a.W), n_fft = P::nfft(a.n_fft), n_out = P::ntrial(a.n_out);
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int col0 = tile * W;
  const int ncols = min(W, a.inner - col0);
  const int npos = n_out * W;
  const bool colm = (P::SL == 0) ? (a.si == 1) : (P::SL == 1);
  auto pos = [=](int it, int& i, int& w) __attribute__((always_inline)) {
    const int f = threadIdx.x + it * NT;
    i = colm ? f % n_out : f / W;
    w = colm ? f / n_out : f % W;
    return f < npos;
  };
  // with row-major positions and NT a multiple of the tile width every
  // position of a thread lies in the same column: its part of xi is evaluated once
  constexpr bool col_fixed = (P::SL == 2) && P::WC > 0 && (NT % P::WC) == 0;
  ColXi<T> cx0{};
  if (col_fixed) cx0 = col_xi<T>(a.g, min(col0 + (int)threadIdx.x % W, a.inner - 1));
  // components in groups of P::CP per transform; LDS tile [row][comp][column]
  constexpr int CPN = P::CP;
  const int LW = P::rowlen(CPN * W);
  // 3-D, one component per transform: two transforms, X_0 and xi_1 X_1 +
  // xi_2 X_2, the sum divided by |xi| at the end (see inv_xi).  Cells with
  // several potentials per frequency do not come here (basis map + plain pass)
  constexpr int FOLD = (CPN != 1 || P::SL == 1) ? 0 : (P::SL == 2) ? 1 : -1;
  const bool fold = (FOLD == 1) || (FOLD == -1 && a.g.d == 3);
  double part = 0.0;
  {
    cpx<T> acc[PMAX];
#pragma unroll
    for (int it = 0; it < PMAX; ++it) acc[it] = cpx<T>{T(0), T(0)};
    if constexpr (P::PRE) {
      // 3-D cells, one component per transform, sizes known at compile time:
      // all three tiles are loaded before the first transform
      constexpr int NL = (P::NF * P::WC + NT - 1) / NT;
      cpx<T> pre[3][NL];
      const cpx<T>* X0 = a.X + (long)item * a.X_stride + col0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int u = 0; u < NL; ++u) {
          const int f = min((int)threadIdx.x + u * NT, P::NF * P::WC - 1);
          const int i = f / P::WC, w = f % P::WC;
          pre[c][u] = X0[(long)c * a.X_cstride + (long)i * a.inner + min(w, ncols - 1)];
        }
      }
      // two transforms: X_0, and xi_1 X_1 + xi_2 X_2 (see inv_xi)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int u = 0; u < NL; ++u) {
          const int f = (int)threadIdx.x + u * NT;
          if (f < P::NF * P::WC) {
            const int i = f / P::WC, w = f % P::WC;
            cpx<T> v = pre[0][u];
            if (c == 1) {
              const ColXi<T> cx = col_fixed ? cx0 : col_xi<T>(a.g, min(col0 + w, a.inner - 1));
              v = cpx<T>{cx.x1 * pre[1][u].x + cx.x2 * pre[2][u].x,
                         cx.x1 * pre[1][u].y + cx.x2 * pre[2][u].y};
            }
            lds[i * LW + w] = (w < ncols) ? v : cpx<T>{T(0), T(0)};
          }
        }
        __syncthreads();
        P::template fft_rows<T, -1>(lds, a.plan, W, a.tw);
#pragma unroll
        for (int it = 0; it < PMAX; ++it) {
          int i, w;
          if (pos(it, i, w)) {
            const int row = (n_out == n_fft) ? i : posk(kof(i, n_out), n_fft);
            const cpx<T> v = lds[row * LW + w];
            const T f0 = (c == 0) ? T(kof(i, n_out)) * T(a.g.invY[0]) : T(1);
            acc[it].x += f0 * v.x;
            acc[it].y += f0 * v.y;
          }
        }
        __syncthreads();
      }
    }
#pragma unroll 1
    for (int al0 = 0; al0 < (P::PRE ? 0 : fold ? 2 : a.d); al0 += CPN) {
      constexpr int nc = CPN;   // CP > 1 kernels serve only cells with CP components
      const cpx<T>* X = a.X + (long)item * a.X_stride + (long)al0 * a.X_cstride + col0;
      if (fold && al0 == 1) {
        // xi_1 X_1 + xi_2 X_2, combined as it is loaded
        in_rounds<NT, rounds_ch(P::NF * P::WC * P::CP, NT)>(
            n_fft * W,
            [=](int f) __attribute__((always_inline)) {
              const int w = f % W, i = f / W;
              const long e = (long)i * a.inner + min(w, ncols - 1);
              return cpx2<T>{X[e], X[e + a.X_cstride]};
            },
            [=](int f, const cpx2<T>& v) __attribute__((always_inline)) {
              const int w = f % W, i = f / W;
              const ColXi<T> cx = col_fixed ? cx0 : col_xi<T>(a.g, min(col0 + w, a.inner - 1));
              lds[i * LW + w] = (w < ncols) ? cpx<T>{cx.x1 * v.a.x + cx.x2 * v.b.x,
                                                     cx.x1 * v.a.y + cx.x2 * v.b.y}
                                            : cpx<T>{T(0), T(0)};
            });
      } else
      in_rounds<NT, rounds_ch(P::NF * P::WC * P::CP, NT)>(
          n_fft * W * nc,
          [=](int f) __attribute__((always_inline)) {
            const int w = f % W, t = f / W, c = t % nc, i = t / nc;
            return X[(long)c * a.X_cstride + (long)i * a.inner + min(w, ncols - 1)];
          },
          [=](int f, const cpx<T>& v) __attribute__((always_inline)) {
            const int w = f % W, t = f / W, c = t % nc, i = t / nc;
            lds[i * LW + c * W + w] = (w < ncols) ? v : cpx<T>{T(0), T(0)};
          });
      __syncthreads();
      P::template fft_rows<T, -1>(lds, a.plan, W, a.tw);
#pragma unroll
      for (int it = 0; it < PMAX; ++it) {
        int i, w;
        if (pos(it, i, w)) {
          const int row = (n_out == n_fft) ? i : posk(kof(i, n_out), n_fft);
          const ColXi<T> cx = col_fixed ? cx0 : col_xi<T>(a.g, min(col0 + w, a.inner - 1));
          for (int c = 0; c < nc; ++c) {
            const cpx<T> v = lds[row * LW + c * W + w];
            const T nvc = fold ? (al0 == 0 ? T(kof(i, n_out)) * T(a.g.invY[0]) : T(1))
                               : normal_comp<T>(a.g, kof(i, n_out), cx, al0 + c);
            acc[it].x += nvc * v.x;
            acc[it].y += nvc * v.y;
          }
        }
      }
      __syncthreads();
    }
    const long sb = (long)item * a.s_stride;
    // the epilogue's loads (p for (p, q), b for the residual) all go out first
    const cpx<T>* ld = (a.epi == EPI_STORE) ? a.p : (a.epi == EPI_RESID) ? a.b : nullptr;
    cpx<T> lv[PMAX];
#pragma unroll
    for (int it = 0; it < PMAX; ++it) {
      int i, w;
      pos(it, i, w);
      lv[it] = cpx<T>{T(0), T(0)};
      if (ld) lv[it] = ld[sb + (long)min(i, n_out - 1) * a.si + (long)(col0 + min(w, ncols - 1)) * a.sc_];
    }
    // Hermitian weight of a column: 1 on the h = 0 plane, else 2
    const double wt0 = col_fixed ? (((col0 + (int)threadIdx.x % W) % a.g.H) == 0 ? 1.0 : 2.0) : 0.0;
#pragma unroll
    for (int it = 0; it < PMAX; ++it) {
      int i, w;
      if (pos(it, i, w) && w < ncols) {
        const int col = col0 + w;
        const long idx = sb + (long)i * a.si + (long)col * a.sc_;
        const int h = col_fixed ? 1 : (a.g.d == 3) ? col % a.g.H : col;   // 2-D: column = h
        const double wt = col_fixed ? wt0 : (h == 0 ? 1.0 : 2.0);
        cpx<T> qv = cscale(acc[it], a.scale);
        if (fold) {
          const ColXi<T> cx = col_fixed ? cx0 : col_xi<T>(a.g, col);
          qv = cscale(qv, inv_xi<T>(a.g, kof(i, n_out), cx));
        }
        if (a.epi == EPI_STORE) {
          a.q[idx] = qv;
          if (a.p) {
            const cpx<T> pv = lv[it];
            part += wt * ((double)pv.x * (double)qv.x + (double)pv.y * (double)qv.y);
          }
        } else if (a.epi == EPI_RHS) {
          qv = cpx<T>{-qv.x, -qv.y};
          a.q[idx] = qv;
          if (a.r) a.r[idx] = qv;
          if (a.pp) a.pp[idx] = qv;
          if (a.x) a.x[idx] = cpx<T>{T(0), T(0)};
          part += wt * ((double)qv.x * (double)qv.x + (double)qv.y * (double)qv.y);
        } else {  // EPI_RESID: r = b - q
          const cpx<T> bv = lv[it];
          const cpx<T> rv = cpx<T>{bv.x - qv.x, bv.y - qv.y};
          a.r[idx] = rv;
          part += wt * ((double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y);
        }
      }
    }
  }
  if (a.partials) {
    part = block_sum<NT>(part);
    if (threadIdx.x == 0) a.partials[(long)item * a.P + tile] = part;
  }
  if (a.rr_part && blockIdx.x == 0) {
    // bookkeeping of the update before this iteration's expansion (that
    // expansion has finished reading rho; no other workgroup here reads it)
    const bool fresh = a.sc[item].fresh != 0;
    const double s = fresh ? 0.0 : sum_partials_wave(a.rr_part + (long)item * a.P, a.rr_n);
    if (threadIdx.x == 0) {
      if (fresh) a.sc[item].fresh = 0;
      else cg_book(a.sc[item], s);
    }
  }
  if (a.pq_part && blockIdx.x == 0) pq_total(a.sc[item], a.pq_part + (long)item * a.P, a.pq_n);
}

// ---------------------------------------------------------------------------
// last (contiguous) axis: pairs of rows packed as one complex line
// ---------------------------------------------------------------------------
// stored components of A per point: 1 (isotropic), d (diagonal), d(d+1)/2
// (symmetric, order 00 11 [22 12 02] 01) or 2 (isotropic elasticity: lambda,
// mu; d is then the Mandel component count 3 or 6)
__device__ __forceinline__ int coef_count(int kind, int d) {
  return kind == 0 ? 1 : kind == 1 ? d : kind == 3 ? 2 : d * (d + 1) / 2;
}

template <class T>
__device__ __forceinline__ void load_coef(int kind, int d, const T* A, long Acs, long off, T* c) {
  const int na = coef_count(kind, d), namax = (d >= 3) ? 6 : (d == 2) ? 3 : 1;
#pragma unroll
  for (int q = 0; q < 6; ++q)
    if (q < namax && q < na) c[q] = A[q * Acs + off];
}

// j = A e from the loaded components c of one point
template <class T>
__device__ __forceinline__ void flux_coef(int kind, int d, const T* c, const T* e, T* j) {
  if (kind == 0) {
    for (int q = 0; q < d; ++q) j[q] = c[0] * e[q];
  } else if (kind == 1) {
    for (int q = 0; q < d; ++q) j[q] = c[q] * e[q];
  } else if (kind == 3) {
    // sigma = lambda tr(eps) I + 2 mu eps on Mandel vectors of d = 3 (plane
    // strain) or 6 components, the normal components first
    const int dim = (d == 6) ? 3 : 2;
    T tr = T(0);
    for (int q = 0; q < dim; ++q) tr += e[q];
    for (int q = 0; q < d; ++q) j[q] = T(2) * c[1] * e[q] + (q < dim ? c[0] * tr : T(0));
  } else if (d == 1) {
    j[0] = c[0] * e[0];
  } else if (d == 2) {
    j[0] = c[0] * e[0] + c[2] * e[1];
    j[1] = c[2] * e[0] + c[1] * e[1];
  } else {
    j[0] = c[0] * e[0] + c[5] * e[1] + c[4] * e[2];
    j[1] = c[5] * e[0] + c[1] * e[1] + c[3] * e[2];
    j[2] = c[4] * e[0] + c[3] * e[1] + c[2] * e[2];
  }
}

template <class T>
__device__ __forceinline__ void flux_point(int kind, int d, const T* A, long Acs, long off,
                                           const T* e, T* j) {
  T c[6];
  load_coef<T>(kind, d, A, Acs, off, c);
  flux_coef<T>(kind, d, c, e, j);
}

template <class T>
struct Coef2 {
  T c0[6], c1[6];
};

template <class T, class P, int MODE>
__global__ __launch_bounds__(P::NT) void k_row(RowArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int NT = P::NT;
  // loads in flight: row loads / stores, flux, real rows
  constexpr int CHR = P::template CH<T>(P::DD * P::RPP * P::HH);
  constexpr int CHF = P::template CH<T>(P::RPP * P::NN) > 4 ? 4 : P::template CH<T>(P::RPP * P::NN);
  constexpr int CHN = P::template CH<T>(P::DD * P::RPP * P::NN);
  const int n = P::n(a.n), H = P::H(a.H), RP = P::RP(a.RP), d = P::D(a.d);
  const int ls = P::ls(a.plan.len);
  const int item = P::ILV ? (int)blockIdx.x % a.items : (int)blockIdx.y;
  if (a.sc && !item_live(a.sc[item])) return;
  const int pair0 = (P::ILV ? (int)blockIdx.x / a.items : xcd_tile(blockIdx.x, gridDim.x)) * RP;

  if (MODE == ROW_APPLY || MODE == ROW_SYNTH) {
    // Z(h) = X_a(h) + i X_b(h), Z(n-h) = conj X_a(h) + i conj X_b(h)
    if (n > 2 * H - 1) {
      const int gap = n - (2 * H - 1);
      for (int f = threadIdx.x; f < d * RP * gap; f += NT) {
        const int line = f / gap, x = H + f % gap;
        lds[line * ls + x] = cpx<T>{T(0), T(0)};
      }
    }
    in_rounds<NT, CHR>(
        d * RP * H,
        [=](int f) __attribute__((always_inline)) {
          const int line = f / H, h = f % H;
          const int comp = line / RP, lp = line % RP;
          const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
          const cpx<T>* src = a.in + (long)item * a.in_stride + (long)comp * a.in_cstride;
          return cpx2<T>{src[(long)min(r0, a.rows - 1) * H + h],
                         src[(long)min(r1, a.rows - 1) * H + h]};
        },
        [=](int f, cpx2<T> v) __attribute__((always_inline)) {
          const int line = f / H, h = f % H;
          const int lp = line % RP;
          const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
          if (r0 >= a.rows) v.a = cpx<T>{T(0), T(0)};
          if (r1 >= a.rows) v.b = cpx<T>{T(0), T(0)};
          if (h == 0) {
            // the h = 0 bin of a real line is real: an imaginary part left there
            // by rounding would otherwise leak into the other line of the pair
            v.a.y = T(0);
            v.b.y = T(0);
          }
          lds[line * ls + h] = cpx<T>{v.a.x - v.b.y, v.a.y + v.b.x};
          if (h > 0) lds[line * ls + n - h] = cpx<T>{v.a.x + v.b.y, v.b.x - v.a.y};
        });
    __syncthreads();
    P::template fft<T, +1>(lds, a.plan, d * RP, ls, a.tw);
  } else if (MODE == ROW_FWD) {
    in_rounds<NT, CHN>(
        d * RP * n,
        [=](int f) __attribute__((always_inline)) {
          const int line = f / n, x = f % n;
          const int comp = line / RP, lp = line % RP;
          const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
          cpx<T> u{T(0), T(0)};
          if (r0 < a.rows) {
            const double* src = a.ureal + (long)item * a.real_stride + (long)comp * a.real_cstride;
            u.x = T(src[(long)r0 * n + x]);
            if (r1 < a.rows) u.y = T(src[(long)r1 * n + x]);
          }
          return u;
        },
        [=](int f, const cpx<T>& u) __attribute__((always_inline)) { lds[(f / n) * ls + f % n] = u; });
    __syncthreads();
  }

  if (MODE == ROW_SYNTH) {
    const double* E = a.E + (long)item * d;
    // once per solve: a plain loop
    for (int f = threadIdx.x; f < d * RP * n; f += NT) {
      const int line = f / n, x = f % n;
      const int comp = line / RP, lp = line % RP;
      const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
      if (r0 >= a.rows) continue;
      double* dst = a.oreal + (long)item * a.real_stride + (long)comp * a.real_cstride;
      const cpx<T> z = lds[line * ls + x];
      dst[(long)r0 * n + x] = (double)z.x + E[comp];
      if (r1 < a.rows) dst[(long)r1 * n + x] = (double)z.y + E[comp];
    }
    return;
  }

  if (MODE == ROW_APPLY || MODE == ROW_CONST) {
    const T* A = a.A + (long)(item / a.A_group) * a.A_stride;
    // e . (A e) over this workgroup's real points: the CG's (p, q) by
    // Parseval, with the forward passes' 1 / |Q| in pscale
    double part = 0.0;
    in_rounds<NT, CHF>(
        RP * n,
        [=](int f) __attribute__((always_inline)) {
          const int lp = f / n, x = f % n;
          const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
          Coef2<T> v;
          load_coef<T>(a.kind, d, A, a.A_cstride, (long)min(r0, a.rows - 1) * n + x, v.c0);
          load_coef<T>(a.kind, d, A, a.A_cstride, (long)min(r1, a.rows - 1) * n + x, v.c1);
          return v;
        },
        [=, &part](int f, const Coef2<T>& v) __attribute__((always_inline)) {
          const int lp = f / n, x = f % n;
          const int r0 = 2 * (pair0 + lp);
          if (r0 >= a.rows) return;
          // up to 6 components (elasticity): the compile-time count, else 6
          constexpr int DM = (P::DD > 3) ? P::DD : (P::DD > 0) ? 3 : 6;
          T e0[DM], e1[DM], j0[DM], j1[DM];
          if (MODE == ROW_CONST) {
            const double* E = a.E + (long)item * d;
            for (int q = 0; q < d; ++q) e0[q] = e1[q] = T(E[q]);
          } else {
            for (int q = 0; q < d; ++q) {
              const cpx<T> z = lds[(q * RP + lp) * ls + x];
              e0[q] = z.x;
              e1[q] = z.y;
            }
          }
          flux_coef<T>(a.kind, d, v.c0, e0, j0);
          flux_coef<T>(a.kind, d, v.c1, e1, j1);
          for (int q = 0; q < d; ++q) lds[(q * RP + lp) * ls + x] = cpx<T>{j0[q], j1[q]};
          if (MODE == ROW_APPLY) {
            // the few terms of one point add up in T (for positive definite
            // A without cancellation), the points in FP64
            const bool two = r0 + 1 < a.rows;
            T t = T(0);
            for (int q = 0; q < d; ++q) t += e0[q] * j0[q] + (two ? e1[q] * j1[q] : T(0));
            part += (double)t;
          }
        });
    __syncthreads();
    if (MODE == ROW_APPLY && a.partials) {
      part = block_sum<NT>(part);
      if (threadIdx.x == 0) a.partials[(long)item * a.P + pair0 / RP] = part * a.pscale;
    }
  }

  // forward transform and split of the two packed real lines
  P::template fft<T, -1>(lds, a.plan, d * RP, ls, a.tw);
  const T half = T(0.5) / T(n);
  in_rounds<NT, CHR>(
      d * RP * H,
      [=](int f) __attribute__((always_inline)) {
        const int line = f / H, h = f % H;
        return cpx2<T>{lds[line * ls + h], lds[line * ls + (h == 0 ? 0 : n - h)]};
      },
      [=](int f, const cpx2<T>& z) __attribute__((always_inline)) {
        const int line = f / H, h = f % H;
        const int comp = line / RP, lp = line % RP;
        const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
        if (r0 >= a.rows) return;
        const cpx<T> zh = z.a, zm = z.b;
        // A = (Z(h) + conj Z(n-h)) / 2,  B = (Z(h) - conj Z(n-h)) / (2 i)
        const cpx<T> va = {(zh.x + zm.x) * half, (zh.y - zm.y) * half};
        const cpx<T> vb = {(zh.y + zm.y) * half, (zm.x - zh.x) * half};
        cpx<T>* dst = a.out + (long)item * a.out_stride + (long)comp * a.out_cstride;
        dst[(long)r0 * H + h] = va;
        if (r1 < a.rows) dst[(long)r1 * H + h] = vb;
      });
}

// ---------------------------------------------------------------------------
// last axis, flux pass (ROW_APPLY) with IT items (load cases) per workgroup:
// the d RP lines of every item of a row tile in one LDS tile, so that the
// coefficient rows of the tile are read once for all of them (items of
// another coefficient block, as in the server, read their own)
// ---------------------------------------------------------------------------
template <class SP, int NTRIAL, int D_, int RP_, int NT_, int IT_>
struct RowMulti {
  static constexpr int NT = NT_, IT = IT_, D = D_, RP = RP_, n = SP::n, H = (NTRIAL + 1) / 2;
  static constexpr int LINES = IT_ * D_ * RP_, LS = SP::len;
  template <class T, int S>
  __device__ __forceinline__ static void fft(cpx<T>* lds, const FftPlan& P, const cpx<T>* tw) {
    sfft<T, S, SP, LINES, false, SP::len, 1, NT_, false>(lds, tw, P);
  }
};

template <class T, class P>
__global__ __launch_bounds__(P::NT) void k_row_multi(RowArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int NT = P::NT, IT = P::IT, D = P::D, RP = P::RP, n = P::n, H = P::H;
  constexpr int ls = P::LS;
  constexpr int CHR = rounds_ch(P::LINES * H, NT);
  constexpr int CHF = rounds_ch(RP * n, NT) > 4 ? 4 : rounds_ch(RP * n, NT);
  const int item0 = (int)blockIdx.y * IT;
  const int nit = min(IT, a.items - item0);
  // items still iterating, one bit each
  unsigned lm = 0;
#pragma unroll
  for (int it = 0; it < IT; ++it)
    if (it < nit && (!a.sc || item_live(a.sc[item0 + it]))) lm |= 1u << it;
  if (!lm) return;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int pair0 = tile * RP;
  // Z(h) = X_a(h) + i X_b(h), Z(n-h) = conj X_a(h) + i conj X_b(h); line
  // (it, comp, lp) at ((it D + comp) RP + lp)
  if (n > 2 * H - 1) {
    constexpr int gap = n - (2 * H - 1);
    for (int f = threadIdx.x; f < P::LINES * gap; f += NT) {
      const int line = f / gap, x = H + f % gap;
      lds[line * ls + x] = cpx<T>{T(0), T(0)};
    }
  }
  in_rounds<NT, CHR>(
      P::LINES * H,
      [=](int f) __attribute__((always_inline)) {
        const int line = f / H, h = f % H;
        const int it = min(line / (D * RP), nit - 1), comp = (line / RP) % D, lp = line % RP;
        const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
        const cpx<T>* src = a.in + (long)(item0 + it) * a.in_stride + (long)comp * a.in_cstride;
        return cpx2<T>{src[(long)min(r0, a.rows - 1) * H + h], src[(long)min(r1, a.rows - 1) * H + h]};
      },
      [=](int f, cpx2<T> v) __attribute__((always_inline)) {
        const int line = f / H, h = f % H;
        const int lp = line % RP;
        const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
        if (r0 >= a.rows || line / (D * RP) >= nit) v.a = v.b = cpx<T>{T(0), T(0)};
        if (r1 >= a.rows) v.b = cpx<T>{T(0), T(0)};
        if (h == 0) {
          // the h = 0 bin of a real line is real
          v.a.y = T(0);
          v.b.y = T(0);
        }
        lds[line * ls + h] = cpx<T>{v.a.x - v.b.y, v.a.y + v.b.x};
        if (h > 0) lds[line * ls + n - h] = cpx<T>{v.a.x + v.b.y, v.b.x - v.a.y};
      });
  __syncthreads();
  P::template fft<T, +1>(lds, a.plan, a.tw);
  // flux: the coefficient rows of a point once, applied to every item; (p, q)
  // partials per item as in k_row
  const long blk0 = (long)(item0 / a.A_group);
  const T* A0 = a.A + blk0 * a.A_stride;
  double part[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) part[it] = 0.0;
  in_rounds<NT, CHF>(
      RP * n,
      [=](int f) __attribute__((always_inline)) {
        const int lp = f / n, x = f % n;
        const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
        Coef2<T> v;
        load_coef<T>(a.kind, D, A0, a.A_cstride, (long)min(r0, a.rows - 1) * n + x, v.c0);
        load_coef<T>(a.kind, D, A0, a.A_cstride, (long)min(r1, a.rows - 1) * n + x, v.c1);
        return v;
      },
      [=, &part](int f, const Coef2<T>& v) __attribute__((always_inline)) {
        const int lp = f / n, x = f % n;
        const int r0 = 2 * (pair0 + lp);
        if (r0 >= a.rows) return;
        const bool two = r0 + 1 < a.rows;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
          if (it >= nit) break;
          Coef2<T> cv = v;
          const long blk = (long)((item0 + it) / a.A_group);
          if (blk != blk0) {
            // another coefficient block (items of several cells)
            const T* Ai = a.A + blk * a.A_stride;
            load_coef<T>(a.kind, D, Ai, a.A_cstride, (long)r0 * n + x, cv.c0);
            load_coef<T>(a.kind, D, Ai, a.A_cstride, (long)min(r0 + 1, a.rows - 1) * n + x, cv.c1);
          }
          T e0[D], e1[D], j0[D], j1[D];
#pragma unroll
          for (int q = 0; q < D; ++q) {
            const cpx<T> z = lds[((it * D + q) * RP + lp) * ls + x];
            e0[q] = z.x;
            e1[q] = z.y;
          }
          flux_coef<T>(a.kind, D, cv.c0, e0, j0);
          flux_coef<T>(a.kind, D, cv.c1, e1, j1);
          T t = T(0);
#pragma unroll
          for (int q = 0; q < D; ++q) {
            lds[((it * D + q) * RP + lp) * ls + x] = cpx<T>{j0[q], j1[q]};
            t += e0[q] * j0[q] + (two ? e1[q] * j1[q] : T(0));
          }
          part[it] += (double)t;
        }
      });
  __syncthreads();
  if (a.partials) {
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const double s = block_sum<NT>(part[it]);
      if (threadIdx.x == 0 && ((lm >> it) & 1u)) a.partials[(long)(item0 + it) * a.P + tile] = s * a.pscale;
    }
  }
  P::template fft<T, -1>(lds, a.plan, a.tw);
  const T half = T(0.5) / T(n);
  in_rounds<NT, CHR>(
      P::LINES * H,
      [=](int f) __attribute__((always_inline)) {
        const int line = f / H, h = f % H;
        return cpx2<T>{lds[line * ls + h], lds[line * ls + (h == 0 ? 0 : n - h)]};
      },
      [=](int f, const cpx2<T>& z) __attribute__((always_inline)) {
        const int line = f / H, h = f % H;
        const int it = line / (D * RP), comp = (line / RP) % D, lp = line % RP;
        const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
        if (r0 >= a.rows || !((lm >> it) & 1u)) return;
        const cpx<T> zh = z.a, zm = z.b;
        const cpx<T> va = {(zh.x + zm.x) * half, (zh.y - zm.y) * half};
        const cpx<T> vb = {(zh.y + zm.y) * half, (zm.x - zh.x) * half};
        cpx<T>* dst = a.out + (long)(item0 + it) * a.out_stride + (long)comp * a.out_cstride;
        dst[(long)r0 * H + h] = va;
        if (r1 < a.rows) dst[(long)r1 * H + h] = vb;
      });
}

}  // namespace hom

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

// SL: layout of the scalar spectra (0: given at run time by the strides,
// 1: column-major, 2: row-major); fixed at compile time in the specialised
// kernels, so only one thread mapping is built
struct ColGen {
  static constexpr int NT = kThreads;
  static constexpr int CP = 1;   // components per transform call
  static constexpr int SL = 0;
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

template <class SP, int NTRIAL, int W_, int NT_, int SL_ = 0>
struct ColStat {
  static constexpr int NT = NT_;
  static constexpr int CP = 1;
  static constexpr int SL = SL_;
  // only the column-major mapping (axis 0 across the threads) needs the pad
  static constexpr int RL = (SL_ == 1) ? odd_rowlen(W_) : W_;
  __device__ static constexpr int W(int) { return W_; }
  __device__ static constexpr int nfft(int) { return SP::n; }
  __device__ static constexpr int ntrial(int) { return NTRIAL; }
  __device__ static constexpr int rowlen(int) { return RL; }
  template <class T, int S>
  __device__ __forceinline__ static void fft(cpx<T>* lds, const FftPlan&, int, const cpx<T>* tw) {
    sfft<T, S, SP, W_, true, 1, W_, NT_>(lds, tw);
  }
  template <class T, int S>
  __device__ __forceinline__ static void fft_rows(cpx<T>* lds, const FftPlan&, int,
                                                  const cpx<T>* tw) {
    sfft<T, S, SP, W_, true, 1, RL, NT_>(lds, tw);
  }
};

// all D_ components of a W_-column tile side by side in one LDS tile
// ([row][component][column]) and transformed by one call, so the block's
// threads share the stages of every component and its loads are issued together
template <class SP, int NTRIAL, int W_, int D_, int NT_>
struct ColStatCP {
  static constexpr int NT = NT_;
  static constexpr int CP = D_;
  static constexpr int SL = (D_ == 2) ? 1 : 2;   // the layout cells with D_ components use
  static constexpr int RL = (SL == 1) ? odd_rowlen(D_ * W_) : D_ * W_;
  __device__ static constexpr int W(int) { return W_; }
  __device__ static constexpr int nfft(int) { return SP::n; }
  __device__ static constexpr int ntrial(int) { return NTRIAL; }
  __device__ static constexpr int rowlen(int) { return RL; }
  template <class T, int S>
  __device__ __forceinline__ static void fft_rows(cpx<T>* lds, const FftPlan&, int,
                                                  const cpx<T>* tw) {
    sfft<T, S, SP, D_ * W_, true, 1, RL, NT_>(lds, tw);
  }
};

struct RowGen {
  static constexpr int NT = kThreads;
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

template <class SP, int NTRIAL, int D_, int RP_, int NT_>
struct RowStat {
  static constexpr int NT = NT_;
  __device__ static constexpr int D(int) { return D_; }
  __device__ static constexpr int RP(int) { return RP_; }
  __device__ static constexpr int n(int) { return SP::n; }
  __device__ static constexpr int H(int) { return (NTRIAL + 1) / 2; }
  __device__ static constexpr int ls(int) { return SP::len; }
  template <class T, int S>
  __device__ __forceinline__ static void fft(cpx<T>* lds, const FftPlan&, int, int,
                                             const cpx<T>* tw) {
    sfft<T, S, SP, D_ * RP_, false, SP::len, 1, NT_>(lds, tw);
  }
};

__device__ __forceinline__ int kof(int i, int n) { return (i <= (n - 1) / 2) ? i : i - n; }
__device__ __forceinline__ int posk(int k, int n) { return k < 0 ? k + n : k; }

// unit normal n(k) = xi / |xi| (0 at k = 0); column index -> (k1, h) in 3-D, h in 2-D
template <class T>
__device__ __forceinline__ void unit_normal(const NormalGeo& g, int k0, int col, T* nv) {
  T xi0 = T(k0) * T(g.invY[0]), xi1, xi2 = T(0);
  if (g.d == 3) {
    const int k1 = kof(col / g.H, g.N1);
    const int h = col % g.H;
    xi1 = T(k1) * T(g.invY[1]);
    xi2 = T(h) * T(g.invY[2]);
  } else {
    xi1 = T(col) * T(g.invY[1]);
  }
  const T s = xi0 * xi0 + xi1 * xi1 + xi2 * xi2;
  const T inv = s > T(0) ? T(1) / sqrt(s) : T(0);
  nv[0] = xi0 * inv;
  nv[1] = xi1 * inv;
  nv[2] = xi2 * inv;
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

// fixed-order sum of nparts partials, result valid in thread 0
__device__ __forceinline__ double sum_partials(const double* p, int nparts) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) v += p[i];
  return block_sum<kThreads>(v);
}

// the same fixed-order sum for a workgroup of NT threads, returned to every
// thread (each workgroup that needs a CG scalar derives it identically)
template <int NT>
__device__ __forceinline__ double sum_partials_all(const double* p, int nparts) {
  __shared__ double total;
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += NT) v += p[i];
  v = block_sum<NT>(v);
  if (threadIdx.x == 0) total = v;
  __syncthreads();
  v = total;
  __syncthreads();
  return v;
}

// CG bookkeeping of one completed update from the sum s = (r, r): iteration
// count, stopping test (relative residual or budget), beta and rho.  One
// thread of one workgroup per item runs it, in a kernel whose other
// workgroups do not read these fields.
__device__ __forceinline__ void cg_book(ItemScal& q, double s) {
  q.iters += 1;
  if (!isfinite(s)) {
    q.status = -5;
    q.active = 0;
    return;
  }
  // beta is kept also when the item stops: a residual replacement of the
  // mixed solver rescales it and carries the search direction on
  q.beta = s / q.rho;
  if (sqrt(s / q.rho0) <= q.tol) {
    q.conv = 1;
    q.active = 0;
  } else if (q.iters >= q.max_iter) {
    q.active = 0;
  }
  q.rho = s;
}

// the decision cg_book will take, derived by every workgroup of the next
// expansion: 1 if the item stops after its last update
__device__ __forceinline__ bool cg_stops(const ItemScal& q, double s) {
  return !isfinite(s) || sqrt(s / q.rho0) <= q.tol || q.iters + 1 >= q.max_iter;
}

// ---------------------------------------------------------------------------
// axis 0 from the scalar potential (optionally fusing p <- r + beta p):
// X_a = F_0^-1 Pad(n_a c) for every component a
// ---------------------------------------------------------------------------
template <class T, class P, int PMAX>
__global__ __launch_bounds__(P::NT) void k_col_expand(ColExpandArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int NT = P::NT;
  const int item = blockIdx.y;
  if (a.sc && !a.sc[item].active) return;
  const int W = P::W(a.W), n_in = P::ntrial(a.n_in), n_fft = P::nfft(a.n_fft);
  const int col0 = xcd_tile(blockIdx.x, gridDim.x) * W;
  const int ncols = min(W, a.inner - col0);
  const long ibase = (long)item * a.c_stride;
  T beta = a.fuse ? T(a.sc[item].beta) : T(0);
  if (a.fuse && a.rr_part && !a.sc[item].fresh) {
    // s = (r, r) of the last update; its bookkeeping runs in the projection
    const double s = sum_partials_all<NT>(a.rr_part + (long)item * a.P, a.rr_n);
    const ItemScal q = a.sc[item];
    if (cg_stops(q, s)) return;
    beta = T(s / q.rho);
  }
  const int npos = n_in * W;
  const bool colm = (P::SL == 0) ? (a.si == 1) : (P::SL == 1);
  cpx<T> s[PMAX];
  int row[PMAX];
#pragma unroll
  for (int it = 0; it < PMAX; ++it) {
    const int f = threadIdx.x + it * NT;
    s[it] = cpx<T>{T(0), T(0)};
    row[it] = -1;
    if (f < npos) {
      // with column-major scalars axis 0 runs across the threads (contiguous
      // loads), else the tile columns do
      const int i = colm ? f % n_in : f / W, w = colm ? f / n_in : f % W;
      row[it] = (n_fft == n_in) ? i : posk(kof(i, n_in), n_fft);
      if (w < ncols) {
        const long idx = ibase + (long)i * a.si + (long)(col0 + w) * a.sc_;
        if (a.fuse) {
          const cpx<T> rv = a.r[idx];
          cpx<T> pv = a.p[idx];
          // beta = 0 restarts the direction: p = r exactly, whatever p held
          pv = (beta == T(0)) ? rv : cpx<T>{rv.x + beta * pv.x, rv.y + beta * pv.y};
          a.p[idx] = pv;
          s[it] = pv;
        } else {
          s[it] = a.c[idx];
        }
      }
    }
  }
  // components in groups of P::CP per transform; LDS tile [row][comp][column]
  constexpr int CPN = P::CP;
  const int LW = P::rowlen(CPN * W);
  for (int al0 = 0; al0 < a.g.d; al0 += CPN) {
    constexpr int nc = CPN;   // CP > 1 kernels serve only cells with CP components
    if (n_fft != n_in) {
      for (int f = threadIdx.x; f < n_fft * LW; f += NT) lds[f] = cpx<T>{T(0), T(0)};
      __syncthreads();
    }
#pragma unroll
    for (int it = 0; it < PMAX; ++it) {
      if (row[it] >= 0) {
        const int f = threadIdx.x + it * NT;
        const int i = colm ? f % n_in : f / W, w = colm ? f / n_in : f % W;
        T nv[3];
        unit_normal<T>(a.g, kof(i, n_in), min(col0 + w, a.inner - 1), nv);
        for (int c = 0; c < nc; ++c) lds[row[it] * LW + c * W + w] = cscale(s[it], nv[al0 + c]);
      }
    }
    __syncthreads();
    P::template fft_rows<T, +1>(lds, a.plan, W, a.tw);
    cpx<T>* X = a.X + (long)item * a.X_stride + (long)al0 * a.X_cstride;
    for (int f = threadIdx.x; f < n_fft * W * nc; f += NT) {
      const int w = f % W, t = f / W, c = t % nc, i = t / nc;
      if (w < ncols) X[(long)c * a.X_cstride + (long)i * a.inner + col0 + w] = lds[i * LW + c * W + w];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// plain pass along a middle axis: inverse with zero padding (trial -> fft
// length) or forward with truncation (fft length -> trial), per component
// ---------------------------------------------------------------------------
template <class T, class P, int S>
__global__ __launch_bounds__(P::NT) void k_col_plain(ColPlainArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int NT = P::NT;
  const int item = blockIdx.z / a.d, comp = blockIdx.z % a.d;
  if (a.sc && !a.sc[item].active) return;
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
  for (int f = threadIdx.x; f < n_in * W; f += NT) {
    const int i = f / W, w = f % W;
    const int rrow = (n_in == n_fft) ? i : posk(kof(i, n_in), n_fft);
    lds[rrow * W + w] = (w < ncols) ? in[(long)i * a.inner + w] : cpx<T>{T(0), T(0)};
  }
  __syncthreads();
  P::template fft<T, S>(lds, a.plan, W, a.tw);
  for (int f = threadIdx.x; f < n_out * W; f += NT) {
    const int i = f / W, w = f % W;
    const int rrow = (n_out == n_fft) ? i : posk(kof(i, n_out), n_fft);
    if (w < ncols) out[(long)i * a.inner + w] = cscale(lds[rrow * W + w], a.scale);
  }
}

// ---------------------------------------------------------------------------
// axis 0 forward + truncation + projection q = n . F_0[X], CG epilogues
// ---------------------------------------------------------------------------
template <class T, class P, int PMAX>
__global__ __launch_bounds__(P::NT) void k_col_project(ColProjectArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int NT = P::NT;
  const int item = blockIdx.y;
  if (a.sc && !a.sc[item].active) return;
  const int W = P::W(a.W), n_fft = P::nfft(a.n_fft), n_out = P::ntrial(a.n_out);
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int col0 = tile * W;
  const int ncols = min(W, a.inner - col0);
  const int npos = n_out * W;
  const bool colm = (P::SL == 0) ? (a.si == 1) : (P::SL == 1);
  cpx<T> acc[PMAX];
  int row[PMAX];
#pragma unroll
  for (int it = 0; it < PMAX; ++it) {
    acc[it] = cpx<T>{T(0), T(0)};
    const int f = threadIdx.x + it * NT;
    row[it] = -1;
    if (f < npos) {
      const int i = colm ? f % n_out : f / W;
      row[it] = (n_out == n_fft) ? i : posk(kof(i, n_out), n_fft);
    }
  }
  // components in groups of P::CP per transform; LDS tile [row][comp][column]
  constexpr int CPN = P::CP;
  const int LW = P::rowlen(CPN * W);
  for (int al0 = 0; al0 < a.d; al0 += CPN) {
    constexpr int nc = CPN;   // CP > 1 kernels serve only cells with CP components
    const cpx<T>* X = a.X + (long)item * a.X_stride + (long)al0 * a.X_cstride + col0;
    for (int f = threadIdx.x; f < n_fft * W * nc; f += NT) {
      const int w = f % W, t = f / W, c = t % nc, i = t / nc;
      lds[i * LW + c * W + w] = (w < ncols) ? X[(long)c * a.X_cstride + (long)i * a.inner + w]
                                            : cpx<T>{T(0), T(0)};
    }
    __syncthreads();
    P::template fft_rows<T, -1>(lds, a.plan, W, a.tw);
#pragma unroll
    for (int it = 0; it < PMAX; ++it) {
      if (row[it] >= 0) {
        const int f = threadIdx.x + it * NT;
        const int i = colm ? f % n_out : f / W, w = colm ? f / n_out : f % W;
        T nv[3];
        unit_normal<T>(a.g, kof(i, n_out), min(col0 + w, a.inner - 1), nv);
        for (int c = 0; c < nc; ++c) {
          const cpx<T> v = lds[row[it] * LW + c * W + w];
          acc[it].x += nv[al0 + c] * v.x;
          acc[it].y += nv[al0 + c] * v.y;
        }
      }
    }
    __syncthreads();
  }
  double part = 0.0;
  const long sb = (long)item * a.s_stride;
#pragma unroll
  for (int it = 0; it < PMAX; ++it) {
    const int f = threadIdx.x + it * NT;
    const int i = colm ? f % n_out : f / W, w = colm ? f / n_out : f % W;
    if (row[it] >= 0 && w < ncols) {
      const int col = col0 + w;
      const long idx = sb + (long)i * a.si + (long)col * a.sc_;
      const double wt = ((col % a.g.H) == 0) ? 1.0 : 2.0;
      cpx<T> qv = cscale(acc[it], a.scale);
      if (a.epi == EPI_STORE) {
        a.q[idx] = qv;
        if (a.p) {
          const cpx<T> pv = a.p[idx];
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
        const cpx<T> bv = a.b[idx];
        const cpx<T> rv = cpx<T>{bv.x - qv.x, bv.y - qv.y};
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
    const double s = fresh ? 0.0 : sum_partials_all<NT>(a.rr_part + (long)item * a.P, a.rr_n);
    if (threadIdx.x == 0) {
      if (fresh) a.sc[item].fresh = 0;
      else cg_book(a.sc[item], s);
    }
  }
}

// ---------------------------------------------------------------------------
// last (contiguous) axis: pairs of rows packed as one complex line
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void flux_point(int kind, int d, const T* A, long Acs, long off,
                                           const T* e, T* j) {
  if (kind == 0) {
    const T a = A[off];
    for (int q = 0; q < d; ++q) j[q] = a * e[q];
  } else if (kind == 1) {
    for (int q = 0; q < d; ++q) j[q] = A[q * Acs + off] * e[q];
  } else {
    if (d == 1) {
      j[0] = A[off] * e[0];
    } else if (d == 2) {
      const T a00 = A[off], a11 = A[Acs + off], a01 = A[2 * Acs + off];
      j[0] = a00 * e[0] + a01 * e[1];
      j[1] = a01 * e[0] + a11 * e[1];
    } else {
      const T a00 = A[off], a11 = A[Acs + off], a22 = A[2 * Acs + off];
      const T a12 = A[3 * Acs + off], a02 = A[4 * Acs + off], a01 = A[5 * Acs + off];
      j[0] = a00 * e[0] + a01 * e[1] + a02 * e[2];
      j[1] = a01 * e[0] + a11 * e[1] + a12 * e[2];
      j[2] = a02 * e[0] + a12 * e[1] + a22 * e[2];
    }
  }
}

template <class T, class P, int MODE>
__global__ __launch_bounds__(P::NT) void k_row(RowArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int NT = P::NT;
  const int item = blockIdx.y;
  if (a.sc && !a.sc[item].active) return;
  const int n = P::n(a.n), H = P::H(a.H), RP = P::RP(a.RP), d = P::D(a.d);
  const int ls = P::ls(a.plan.len);
  const int pair0 = xcd_tile(blockIdx.x, gridDim.x) * RP;

  if (MODE == ROW_APPLY || MODE == ROW_SYNTH) {
    // Z(h) = X_a(h) + i X_b(h), Z(n-h) = conj X_a(h) + i conj X_b(h)
    if (n > 2 * H - 1) {
      const int gap = n - (2 * H - 1);
      for (int f = threadIdx.x; f < d * RP * gap; f += NT) {
        const int line = f / gap, x = H + f % gap;
        lds[line * ls + x] = cpx<T>{T(0), T(0)};
      }
    }
    for (int f = threadIdx.x; f < d * RP * H; f += NT) {
      const int line = f / H, h = f % H;
      const int comp = line / RP, lp = line % RP;
      const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
      cpx<T> xa = {T(0), T(0)}, xb = {T(0), T(0)};
      if (r0 < a.rows) {
        const cpx<T>* src = a.in + (long)item * a.in_stride + (long)comp * a.in_cstride;
        xa = src[(long)r0 * H + h];
        if (r1 < a.rows) xb = src[(long)r1 * H + h];
      }
      if (h == 0) {
        // the h = 0 bin of a real line is real: an imaginary part left there by
        // rounding would otherwise leak into the other line of the pair
        xa.y = T(0);
        xb.y = T(0);
      }
      lds[line * ls + h] = cpx<T>{xa.x - xb.y, xa.y + xb.x};
      if (h > 0) lds[line * ls + n - h] = cpx<T>{xa.x + xb.y, xb.x - xa.y};
    }
    __syncthreads();
    P::template fft<T, +1>(lds, a.plan, d * RP, ls, a.tw);
  } else if (MODE == ROW_FWD) {
    for (int f = threadIdx.x; f < d * RP * n; f += NT) {
      const int line = f / n, x = f % n;
      const int comp = line / RP, lp = line % RP;
      const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
      T ua = T(0), ub = T(0);
      if (r0 < a.rows) {
        const double* src = a.ureal + (long)item * a.real_stride + (long)comp * a.real_cstride;
        ua = T(src[(long)r0 * n + x]);
        if (r1 < a.rows) ub = T(src[(long)r1 * n + x]);
      }
      lds[line * ls + x] = cpx<T>{ua, ub};
    }
    __syncthreads();
  }

  if (MODE == ROW_SYNTH) {
    const double* E = a.E + (long)item * d;
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
    for (int f = threadIdx.x; f < RP * n; f += NT) {
      const int lp = f / n, x = f % n;
      const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
      if (r0 >= a.rows) continue;
      T e0[3], e1[3], j0[3], j1[3];
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
      flux_point<T>(a.kind, d, A, a.A_cstride, (long)r0 * n + x, e0, j0);
      flux_point<T>(a.kind, d, A, a.A_cstride, (long)((r1 < a.rows) ? r1 : r0) * n + x, e1, j1);
      for (int q = 0; q < d; ++q) lds[(q * RP + lp) * ls + x] = cpx<T>{j0[q], j1[q]};
    }
    __syncthreads();
  }

  // forward transform and split of the two packed real lines
  P::template fft<T, -1>(lds, a.plan, d * RP, ls, a.tw);
  const T half = T(0.5) / T(n);
  for (int f = threadIdx.x; f < d * RP * H; f += NT) {
    const int line = f / H, h = f % H;
    const int comp = line / RP, lp = line % RP;
    const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
    if (r0 >= a.rows) continue;
    const cpx<T> zh = lds[line * ls + h];
    const cpx<T> zm = lds[line * ls + (h == 0 ? 0 : n - h)];
    // A = (Z(h) + conj Z(n-h)) / 2,  B = (Z(h) - conj Z(n-h)) / (2 i)
    const cpx<T> va = {(zh.x + zm.x) * half, (zh.y - zm.y) * half};
    const cpx<T> vb = {(zh.y + zm.y) * half, (zm.x - zh.x) * half};
    cpx<T>* dst = a.out + (long)item * a.out_stride + (long)comp * a.out_cstride;
    dst[(long)r0 * H + h] = va;
    if (r1 < a.rows) dst[(long)r1 * H + h] = vb;
  }
}

}  // namespace hom

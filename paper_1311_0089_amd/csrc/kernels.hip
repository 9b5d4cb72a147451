// kernels.hip -- hot-path kernels for gfx950: FFT passes with fused pointwise
// stages (flux A e, projection on n(k), CG updates and FP64 partial dots),
// CG scalar kernels and the FP64 energy quadrature.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace hom {

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

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kThreads / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (wid == 0) {
    v = (lane < (int)(blockDim.x >> 6)) ? red[lane] : 0.0;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  }
  __syncthreads();
  return v;
}

// fixed-order sum of nparts partials, result valid in thread 0
__device__ __forceinline__ double sum_partials(const double* p, int nparts) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) v += p[i];
  return block_sum(v);
}

// ---------------------------------------------------------------------------
// axis 0 from the scalar potential (optionally fusing p <- r + beta p)
// ---------------------------------------------------------------------------
template <class T, int PMAX>
__global__ __launch_bounds__(kThreads) void k_col_expand(ColExpandArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  const int item = blockIdx.y;
  if (a.sc && !a.sc[item].active) return;
  const int col0 = blockIdx.x * a.W;
  const int ncols = min(a.W, a.inner - col0);
  const long ibase = (long)item * a.c_stride;
  const T beta = a.fuse ? T(a.sc[item].beta) : T(0);
  const int npos = a.n_in * a.W;
  cpx<T> s[PMAX];
  int row[PMAX];
#pragma unroll
  for (int it = 0; it < PMAX; ++it) {
    const int f = threadIdx.x + it * blockDim.x;
    s[it] = cpx<T>{T(0), T(0)};
    row[it] = -1;
    if (f < npos) {
      const int i = f / a.W, w = f % a.W;
      const int k0 = kof(i, a.n_in);
      row[it] = (a.n_fft == a.n_in) ? i : posk(k0, a.n_fft);
      if (w < ncols) {
        const long idx = ibase + (long)i * a.inner + col0 + w;
        if (a.fuse) {
          cpx<T> rv = a.r[idx], pv = a.p[idx];
          pv = cpx<T>{rv.x + beta * pv.x, rv.y + beta * pv.y};
          a.p[idx] = pv;
          s[it] = pv;
        } else {
          s[it] = a.c[idx];
        }
      }
    }
  }
  const LdsLines L{a.W, 1, a.W, true};
  for (int al = 0; al < a.g.d; ++al) {
    if (a.n_fft != a.n_in) {
      for (int f = threadIdx.x; f < a.n_fft * a.W; f += blockDim.x) lds[f] = cpx<T>{T(0), T(0)};
      __syncthreads();
    }
#pragma unroll
    for (int it = 0; it < PMAX; ++it) {
      if (row[it] >= 0) {
        const int f = threadIdx.x + it * blockDim.x;
        const int w = f % a.W;
        T nv[3];
        unit_normal<T>(a.g, kof(f / a.W, a.n_in), min(col0 + w, a.inner - 1), nv);
        lds[row[it] * a.W + w] = cscale(s[it], nv[al]);
      }
    }
    __syncthreads();
    line_fft<T, +1>(lds, a.plan, L, a.tw);
    cpx<T>* X = a.X + (long)item * a.X_stride + (long)al * a.X_cstride;
    for (int f = threadIdx.x; f < a.n_fft * a.W; f += blockDim.x) {
      const int i = f / a.W, w = f % a.W;
      if (w < ncols) X[(long)i * a.inner + col0 + w] = lds[i * a.W + w];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// plain pass along a middle axis; zero-pad (inverse) or truncate (forward)
// ---------------------------------------------------------------------------
template <class T, int S>
__global__ __launch_bounds__(kThreads) void k_col_plain(ColPlainArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  const int item = blockIdx.z / a.d, comp = blockIdx.z % a.d;
  if (a.sc && !a.sc[item].active) return;
  const int o = blockIdx.y;
  const int col0 = blockIdx.x * a.W;
  const int ncols = min(a.W, a.inner - col0);
  const cpx<T>* in = a.in + (long)item * a.in_stride + (long)comp * a.in_cstride +
                     (long)o * a.n_in * a.inner + col0;
  cpx<T>* out = a.out + (long)item * a.out_stride + (long)comp * a.out_cstride +
                (long)o * a.n_out * a.inner + col0;
  if (a.n_in != a.n_fft) {
    for (int f = threadIdx.x; f < a.n_fft * a.W; f += blockDim.x) lds[f] = cpx<T>{T(0), T(0)};
    __syncthreads();
  }
  for (int f = threadIdx.x; f < a.n_in * a.W; f += blockDim.x) {
    const int i = f / a.W, w = f % a.W;
    const int rrow = (a.n_in == a.n_fft) ? i : posk(kof(i, a.n_in), a.n_fft);
    lds[rrow * a.W + w] = (w < ncols) ? in[(long)i * a.inner + w] : cpx<T>{T(0), T(0)};
  }
  __syncthreads();
  const LdsLines L{a.W, 1, a.W, true};
  line_fft<T, S>(lds, a.plan, L, a.tw);
  for (int f = threadIdx.x; f < a.n_out * a.W; f += blockDim.x) {
    const int i = f / a.W, w = f % a.W;
    const int rrow = (a.n_out == a.n_fft) ? i : posk(kof(i, a.n_out), a.n_fft);
    if (w < ncols) out[(long)i * a.inner + w] = cscale(lds[rrow * a.W + w], a.scale);
  }
}

// ---------------------------------------------------------------------------
// axis 0 forward + truncation + projection, with CG epilogues
// ---------------------------------------------------------------------------
template <class T, int PMAX>
__global__ __launch_bounds__(kThreads) void k_col_project(ColProjectArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  const int item = blockIdx.y;
  if (a.sc && !a.sc[item].active) return;
  const int col0 = blockIdx.x * a.W;
  const int ncols = min(a.W, a.inner - col0);
  const int npos = a.n_out * a.W;
  cpx<T> acc[PMAX];
  int row[PMAX];
#pragma unroll
  for (int it = 0; it < PMAX; ++it) {
    acc[it] = cpx<T>{T(0), T(0)};
    const int f = threadIdx.x + it * blockDim.x;
    row[it] = -1;
    if (f < npos) {
      const int i = f / a.W;
      row[it] = (a.n_out == a.n_fft) ? i : posk(kof(i, a.n_out), a.n_fft);
    }
  }
  const LdsLines L{a.W, 1, a.W, true};
  for (int al = 0; al < a.d; ++al) {
    const cpx<T>* X = a.X + (long)item * a.X_stride + (long)al * a.X_cstride + col0;
    for (int f = threadIdx.x; f < a.n_fft * a.W; f += blockDim.x) {
      const int i = f / a.W, w = f % a.W;
      lds[f] = (w < ncols) ? X[(long)i * a.inner + w] : cpx<T>{T(0), T(0)};
    }
    __syncthreads();
    line_fft<T, -1>(lds, a.plan, L, a.tw);
#pragma unroll
    for (int it = 0; it < PMAX; ++it) {
      if (row[it] >= 0) {
        const int f = threadIdx.x + it * blockDim.x;
        const int i = f / a.W, w = f % a.W;
        T nv[3];
        unit_normal<T>(a.g, kof(i, a.n_out), min(col0 + w, a.inner - 1), nv);
        const cpx<T> v = lds[row[it] * a.W + w];
        acc[it].x += nv[al] * v.x;
        acc[it].y += nv[al] * v.y;
      }
    }
    __syncthreads();
  }
  // epilogue
  double part = 0.0;
  const long sb = (long)item * a.s_stride;
#pragma unroll
  for (int it = 0; it < PMAX; ++it) {
    const int f = threadIdx.x + it * blockDim.x;
    if (row[it] >= 0 && (f % a.W) < ncols) {
      const int i = f / a.W, w = f % a.W;
      const int col = col0 + w;
      const long idx = sb + (long)i * a.inner + col;
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
    part = block_sum(part);
    if (threadIdx.x == 0) a.partials[(long)item * a.P + blockIdx.x] = part;
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

template <class T, int MODE>
__global__ __launch_bounds__(kThreads) void k_row(RowArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  const int item = blockIdx.y;
  if (a.sc && !a.sc[item].active) return;
  const int n = a.n, H = a.H, RP = a.RP, d = a.d;
  const int ls = a.plan.len;
  const int pair0 = blockIdx.x * RP;
  const LdsLines L{d * RP, ls, 1, false};

  if (MODE == ROW_APPLY || MODE == ROW_SYNTH) {
    // Z(h) = X_a(h) + i X_b(h), Z(n-h) = conj X_a(h) + i conj X_b(h)
    if (n > 2 * H - 1) {
      const int gap = n - (2 * H - 1);
      for (int f = threadIdx.x; f < d * RP * gap; f += blockDim.x) {
        const int line = f / gap, x = H + f % gap;
        lds[line * ls + x] = cpx<T>{T(0), T(0)};
      }
    }
    for (int f = threadIdx.x; f < d * RP * H; f += blockDim.x) {
      const int line = f / H, h = f % H;
      const int comp = line / RP, lp = line % RP;
      const int r0 = 2 * (pair0 + lp), r1 = r0 + 1;
      cpx<T> xa = {T(0), T(0)}, xb = {T(0), T(0)};
      if (r0 < a.rows) {
        const cpx<T>* src = a.in + (long)item * a.in_stride + (long)comp * a.in_cstride;
        xa = src[(long)r0 * H + h];
        if (r1 < a.rows) xb = src[(long)r1 * H + h];
      }
      lds[line * ls + h] = cpx<T>{xa.x - xb.y, xa.y + xb.x};
      if (h > 0) lds[line * ls + n - h] = cpx<T>{xa.x + xb.y, xb.x - xa.y};
    }
    __syncthreads();
    line_fft<T, +1>(lds, a.plan, L, a.tw);
  } else if (MODE == ROW_FWD) {
    for (int f = threadIdx.x; f < d * RP * n; f += blockDim.x) {
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
    for (int f = threadIdx.x; f < d * RP * n; f += blockDim.x) {
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
    const T* A = a.A + (long)item * a.A_stride;
    for (int f = threadIdx.x; f < RP * n; f += blockDim.x) {
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
  line_fft<T, -1>(lds, a.plan, L, a.tw);
  const T half = T(0.5) / T(n);
  for (int f = threadIdx.x; f < d * RP * H; f += blockDim.x) {
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

// ---------------------------------------------------------------------------
// CG vector update and scalar kernels
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(kThreads) void k_cg_update(CgUpdateArgs<T> a) {
  const int item = blockIdx.y;
  if (!a.sc[item].active) return;
  const T alpha = T(a.sc[item].alpha);
  const long base = (long)item * a.stride;
  double part = 0.0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < a.count;
       e += (long)gridDim.x * blockDim.x) {
    const cpx<T> pv = a.p[base + e], qv = a.q[base + e];
    cpx<T> xv = a.x[base + e], rv = a.r[base + e];
    xv.x += alpha * pv.x;
    xv.y += alpha * pv.y;
    rv.x -= alpha * qv.x;
    rv.y -= alpha * qv.y;
    a.x[base + e] = xv;
    a.r[base + e] = rv;
    const double wt = ((e % a.H) == 0) ? 1.0 : 2.0;
    part += wt * ((double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y);
  }
  part = block_sum(part);
  if (threadIdx.x == 0) a.partials[(long)item * a.P + blockIdx.x] = part;
}

__global__ __launch_bounds__(kThreads) void k_cg_init(ItemScal* sc, const double* partials, int P,
                                                      int nparts) {
  const int item = blockIdx.x;
  if (!sc[item].active) return;
  const double s = sum_partials(partials + (long)item * P, nparts);
  if (threadIdx.x == 0) {
    ItemScal& q = sc[item];
    q.rho = q.rho0 = s;
    q.iters = 0;
    q.beta = 0.0;
    q.alpha = 0.0;
    q.status = 0;
    q.conv = (s == 0.0) ? 1 : 0;
    q.active = (s > 0.0 && isfinite(s) && q.max_iter > 0) ? 1 : 0;
    if (!isfinite(s)) q.status = -5;
  }
}

__global__ __launch_bounds__(kThreads) void k_cg_alpha(ItemScal* sc, const double* partials, int P,
                                                       int nparts) {
  const int item = blockIdx.x;
  if (!sc[item].active) return;
  const double g = sum_partials(partials + (long)item * P, nparts);
  if (threadIdx.x == 0) {
    ItemScal& q = sc[item];
    q.gamma = g;
    if (!(g > 0.0) || !isfinite(g)) {
      q.status = -5;
      q.active = 0;
      q.alpha = 0.0;
    } else {
      q.alpha = q.rho / g;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_cg_beta(ItemScal* sc, const double* partials, int P,
                                                      int nparts) {
  const int item = blockIdx.x;
  if (!sc[item].active) return;
  const double s = sum_partials(partials + (long)item * P, nparts);
  if (threadIdx.x == 0) {
    ItemScal& q = sc[item];
    q.iters += 1;
    if (!isfinite(s)) {
      q.status = -5;
      q.active = 0;
      return;
    }
    if (sqrt(s / q.rho0) <= q.tol) {
      q.conv = 1;
      q.active = 0;
      q.beta = 0.0;
    } else {
      q.beta = s / q.rho;
      if (q.iters >= q.max_iter) q.active = 0;
    }
    q.rho = s;
  }
}

__global__ __launch_bounds__(kThreads) void k_outer_check(ItemScal* sc, const double* partials,
                                                          int P, int nparts, int init) {
  const int item = blockIdx.x;
  if (!sc[item].active) return;
  const double s = sum_partials(partials + (long)item * P, nparts);
  if (threadIdx.x == 0) {
    ItemScal& q = sc[item];
    if (init) {
      q.rho0 = s;
      q.iters = 0;
      q.status = 0;
    }
    q.rho = s;
    if (!isfinite(s)) {
      q.status = -5;
      q.active = 0;
    } else if (s == 0.0 || sqrt(s / q.rho0) <= q.tol) {
      q.conv = 1;
      q.active = 0;
    } else if (q.iters >= q.max_iter) {
      q.active = 0;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_inner_start(const cpx<double>* r64, cpx<float>* r32,
                                                          cpx<float>* p32, cpx<float>* x32,
                                                          long stride, long count, int H,
                                                          ItemScal* outer, ItemScal* inner,
                                                          double eta, int max_iter,
                                                          double* partials, int P) {
  const int item = blockIdx.y;
  if (!outer[item].active) {
    if (blockIdx.x == 0 && threadIdx.x == 0) inner[item].active = 0;
    return;
  }
  const double sc = 1.0 / sqrt(outer[item].rho);
  const long base = (long)item * stride;
  double part = 0.0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (long)gridDim.x * blockDim.x) {
    const cpx<double> v = r64[base + e];
    const cpx<float> w = {(float)(v.x * sc), (float)(v.y * sc)};
    r32[base + e] = w;
    p32[base + e] = w;
    x32[base + e] = cpx<float>{0.f, 0.f};
    const double wt = ((e % H) == 0) ? 1.0 : 2.0;
    part += wt * ((double)w.x * (double)w.x + (double)w.y * (double)w.y);
  }
  part = block_sum(part);
  if (threadIdx.x == 0) partials[(long)item * P + blockIdx.x] = part;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    inner[item].tol = eta;
    inner[item].max_iter = max_iter;
    inner[item].active = 1;
    outer[item].iters += 1;   // refinement steps started
  }
}

__global__ __launch_bounds__(kThreads) void k_inner_accumulate(cpx<double>* x64,
                                                               const cpx<float>* x32, long stride,
                                                               long count, const ItemScal* outer) {
  const int item = blockIdx.y;
  if (!outer[item].active) return;
  const double sc = sqrt(outer[item].rho);
  const long base = (long)item * stride;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (long)gridDim.x * blockDim.x) {
    const cpx<float> v = x32[base + e];
    cpx<double> xv = x64[base + e];
    xv.x += sc * (double)v.x;
    xv.y += sc * (double)v.y;
    x64[base + e] = xv;
  }
}

__global__ void k_set_scal(ItemScal* sc, int items, double tol, int max_iter, int active) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < items) {
    ItemScal q{};
    q.tol = tol;
    q.max_iter = max_iter;
    q.active = active;
    sc[i] = q;
  }
}

// ---------------------------------------------------------------------------
// FP64 energy quadrature W_lm = <e_l . A e_m>, J_l = <A e_l>
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_quad(const double* e, long es, long ecs,
                                                   const double* A, long Acs, int kind, int d,
                                                   long npts, int l0, int nl, int m0, int nm,
                                                   double* partials) {
  double accW[9], accJ[9];
  for (int t = 0; t < 9; ++t) accW[t] = accJ[t] = 0.0;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npts;
       p += (long)gridDim.x * blockDim.x) {
    double el[3][3], jm[3][3];
    for (int l = 0; l < nl; ++l)
      for (int q = 0; q < d; ++q) el[l][q] = e[(l0 + l) * es + q * ecs + p];
    for (int m = 0; m < nm; ++m) {
      double em[3];
      for (int q = 0; q < d; ++q) em[q] = e[(m0 + m) * es + q * ecs + p];
      flux_point<double>(kind, d, A, Acs, p, em, jm[m]);
      for (int q = 0; q < d; ++q) accJ[m * 3 + q] += jm[m][q];
    }
    for (int l = 0; l < nl; ++l)
      for (int m = 0; m < nm; ++m) {
        double s = 0.0;
        for (int q = 0; q < d; ++q) s += el[l][q] * jm[m][q];
        accW[l * 3 + m] += s;
      }
  }
  for (int t = 0; t < 9; ++t) {
    const double v = block_sum(accW[t]);
    if (threadIdx.x == 0) partials[(long)blockIdx.x * 18 + t] = v;
  }
  for (int t = 0; t < 9; ++t) {
    const double v = block_sum(accJ[t]);
    if (threadIdx.x == 0) partials[(long)blockIdx.x * 18 + 9 + t] = v;
  }
}

__global__ __launch_bounds__(kThreads) void k_quad_final(const double* partials, int blocks,
                                                         long npts, double* out) {
  // out[0..8] = W (3x3 slots), out[9..17] = J sums, each divided by npts
  for (int t = 0; t < 18; ++t) {
    double v = 0.0;
    for (int b = threadIdx.x; b < blocks; b += blockDim.x) v += partials[(long)b * 18 + t];
    v = block_sum(v);
    if (threadIdx.x == 0) out[t] = v / (double)npts;
  }
}

__global__ void k_convert(const double* in, float* out, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

__global__ void k_widen(const float* in, double* out, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

template <class T>
hipError_t launch_col_expand(const ColExpandArgs<T>& a, int items, size_t lds, hipStream_t s) {
  dim3 grid(ceil_div(a.inner, a.W), items);
  const long npos = (long)a.n_in * a.W;
  if (npos <= 8L * kThreads)
    hipLaunchKernelGGL((k_col_expand<T, 8>), grid, dim3(kThreads), lds, s, a);
  else if (npos <= 16L * kThreads)
    hipLaunchKernelGGL((k_col_expand<T, 16>), grid, dim3(kThreads), lds, s, a);
  else if (npos <= 32L * kThreads)
    hipLaunchKernelGGL((k_col_expand<T, 32>), grid, dim3(kThreads), lds, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class T>
hipError_t launch_col_plain(const ColPlainArgs<T>& a, int items, int sign, size_t lds,
                            hipStream_t s) {
  dim3 grid(ceil_div(a.inner, a.W), a.outer, items * a.d);
  if (sign < 0)
    hipLaunchKernelGGL((k_col_plain<T, -1>), grid, dim3(kThreads), lds, s, a);
  else
    hipLaunchKernelGGL((k_col_plain<T, +1>), grid, dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_col_project(const ColProjectArgs<T>& a, int items, size_t lds, hipStream_t s) {
  dim3 grid(ceil_div(a.inner, a.W), items);
  const long npos = (long)a.n_out * a.W;
  if (npos <= 8L * kThreads)
    hipLaunchKernelGGL((k_col_project<T, 8>), grid, dim3(kThreads), lds, s, a);
  else if (npos <= 16L * kThreads)
    hipLaunchKernelGGL((k_col_project<T, 16>), grid, dim3(kThreads), lds, s, a);
  else if (npos <= 32L * kThreads)
    hipLaunchKernelGGL((k_col_project<T, 32>), grid, dim3(kThreads), lds, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class T>
hipError_t launch_row(const RowArgs<T>& a, int items, int mode, size_t lds, hipStream_t s) {
  const long pairs = (a.rows + 1) / 2;
  dim3 grid(ceil_div(pairs, a.RP), items);
  switch (mode) {
    case ROW_APPLY: hipLaunchKernelGGL((k_row<T, ROW_APPLY>), grid, dim3(kThreads), lds, s, a); break;
    case ROW_CONST: hipLaunchKernelGGL((k_row<T, ROW_CONST>), grid, dim3(kThreads), lds, s, a); break;
    case ROW_SYNTH: hipLaunchKernelGGL((k_row<T, ROW_SYNTH>), grid, dim3(kThreads), lds, s, a); break;
    case ROW_FWD: hipLaunchKernelGGL((k_row<T, ROW_FWD>), grid, dim3(kThreads), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_cg_update(const CgUpdateArgs<T>& a, int items, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((k_cg_update<T>), dim3(blocks, items), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_cg_init(ItemScal* sc, const double* partials, int P, int nparts, int items,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_cg_init, dim3(items), dim3(kThreads), 0, s, sc, partials, P, nparts);
  return hipGetLastError();
}
hipError_t launch_cg_alpha(ItemScal* sc, const double* partials, int P, int nparts, int items,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(items), dim3(kThreads), 0, s, sc, partials, P, nparts);
  return hipGetLastError();
}
hipError_t launch_cg_beta(ItemScal* sc, const double* partials, int P, int nparts, int items,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_cg_beta, dim3(items), dim3(kThreads), 0, s, sc, partials, P, nparts);
  return hipGetLastError();
}
hipError_t launch_outer_check(ItemScal* sc, const double* partials, int P, int nparts, int items,
                              int init, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_check, dim3(items), dim3(kThreads), 0, s, sc, partials, P, nparts,
                     init);
  return hipGetLastError();
}
hipError_t launch_inner_start(const cpx<double>* r64, cpx<float>* r32, cpx<float>* p32,
                              cpx<float>* x32, long stride, long count, int H, ItemScal* outer,
                              ItemScal* inner, double eta, int max_iter, double* partials, int P,
                              int blocks, int items, hipStream_t s) {
  hipLaunchKernelGGL(k_inner_start, dim3(blocks, items), dim3(kThreads), 0, s, r64, r32, p32, x32,
                     stride, count, H, outer, inner, eta, max_iter, partials, P);
  return hipGetLastError();
}
hipError_t launch_inner_accumulate(cpx<double>* x64, const cpx<float>* x32, long stride, long count,
                                   const ItemScal* outer, int blocks, int items, hipStream_t s) {
  hipLaunchKernelGGL(k_inner_accumulate, dim3(blocks, items), dim3(kThreads), 0, s, x64, x32,
                     stride, count, outer);
  return hipGetLastError();
}
hipError_t launch_set_scal(ItemScal* sc, int items, double tol, int max_iter, int active,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_set_scal, dim3(ceil_div(items, 64)), dim3(64), 0, s, sc, items, tol,
                     max_iter, active);
  return hipGetLastError();
}
hipError_t launch_quad(const double* e, long e_stride, long e_cstride, const double* A,
                       long A_cstride, int kind, int d, long npts, int l0, int nl, int m0, int nm,
                       double* partials, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_quad, dim3(blocks), dim3(kThreads), 0, s, e, e_stride, e_cstride, A,
                     A_cstride, kind, d, npts, l0, nl, m0, nm, partials);
  return hipGetLastError();
}
hipError_t launch_quad_final(const double* partials, int blocks, int nl, int nm, int d, long npts,
                             double* out, hipStream_t s) {
  (void)nl;
  (void)nm;
  (void)d;
  hipLaunchKernelGGL(k_quad_final, dim3(1), dim3(kThreads), 0, s, partials, blocks, npts, out);
  return hipGetLastError();
}
hipError_t launch_convert(const double* in, float* out, long n, hipStream_t s) {
  int blocks = ceil_div(n, kThreads);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_convert, dim3(blocks), dim3(kThreads), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_widen(const float* in, double* out, long n, hipStream_t s) {
  int blocks = ceil_div(n, kThreads);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_widen, dim3(blocks), dim3(kThreads), 0, s, in, out, n);
  return hipGetLastError();
}

template <class K>
static hipError_t set_lds(K kernel, size_t max_lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds);
}

hipError_t configure_kernels(size_t max_lds) {
  hipError_t e = hipSuccess;
#define HOM_SET(k)                            \
  do {                                        \
    hipError_t e2 = set_lds((k), max_lds);    \
    if (e2 != hipSuccess) e = e2;             \
  } while (0)
  HOM_SET((k_col_expand<float, 8>));
  HOM_SET((k_col_expand<float, 16>));
  HOM_SET((k_col_expand<float, 32>));
  HOM_SET((k_col_expand<double, 8>));
  HOM_SET((k_col_expand<double, 16>));
  HOM_SET((k_col_expand<double, 32>));
  HOM_SET((k_col_project<float, 8>));
  HOM_SET((k_col_project<float, 16>));
  HOM_SET((k_col_project<float, 32>));
  HOM_SET((k_col_project<double, 8>));
  HOM_SET((k_col_project<double, 16>));
  HOM_SET((k_col_project<double, 32>));
  HOM_SET((k_col_plain<float, -1>));
  HOM_SET((k_col_plain<float, 1>));
  HOM_SET((k_col_plain<double, -1>));
  HOM_SET((k_col_plain<double, 1>));
  HOM_SET((k_row<float, ROW_APPLY>));
  HOM_SET((k_row<float, ROW_CONST>));
  HOM_SET((k_row<float, ROW_SYNTH>));
  HOM_SET((k_row<float, ROW_FWD>));
  HOM_SET((k_row<double, ROW_APPLY>));
  HOM_SET((k_row<double, ROW_CONST>));
  HOM_SET((k_row<double, ROW_SYNTH>));
  HOM_SET((k_row<double, ROW_FWD>));
#undef HOM_SET
  return e;
}

template hipError_t launch_col_expand<float>(const ColExpandArgs<float>&, int, size_t, hipStream_t);
template hipError_t launch_col_expand<double>(const ColExpandArgs<double>&, int, size_t, hipStream_t);
template hipError_t launch_col_plain<float>(const ColPlainArgs<float>&, int, int, size_t, hipStream_t);
template hipError_t launch_col_plain<double>(const ColPlainArgs<double>&, int, int, size_t, hipStream_t);
template hipError_t launch_col_project<float>(const ColProjectArgs<float>&, int, size_t, hipStream_t);
template hipError_t launch_col_project<double>(const ColProjectArgs<double>&, int, size_t, hipStream_t);
template hipError_t launch_row<float>(const RowArgs<float>&, int, int, size_t, hipStream_t);
template hipError_t launch_row<double>(const RowArgs<double>&, int, int, size_t, hipStream_t);
template hipError_t launch_cg_update<float>(const CgUpdateArgs<float>&, int, int, hipStream_t);
template hipError_t launch_cg_update<double>(const CgUpdateArgs<double>&, int, int, hipStream_t);

}  // namespace hom

// kernels.hip -- hot-path kernels for gfx950: FFT passes with fused pointwise
// stages (flux A e, projection on n(k), CG updates and FP64 partial dots),
// CG scalar kernels and the FP64 energy quadrature.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "kernel_bodies.hpp"
#include "kernels.hpp"

namespace hom {


// ---------------------------------------------------------------------------
// registry of compile-time specialised kernels
// ---------------------------------------------------------------------------
std::vector<StaticKernel>& static_registry() {
  static std::vector<StaticKernel> v;
  return v;
}
void register_static(const StaticKernel& k) { static_registry().push_back(k); }
// Kernel choices are process-wide (they depend only on the pass and its
// sizes); every change bumps a version that captured graphs are keyed by, so
// a graph captured with the old kernels is never replayed after a change.
static std::atomic<bool> g_static_on{true};
static std::atomic<unsigned> g_tune_version{0};
static size_t g_static_max_lds = 0;
void set_static_enabled(bool on) {
  g_static_on = on;
  ++g_tune_version;
}
bool static_enabled() { return g_static_on; }
unsigned tune_version() { return g_tune_version.load(); }
static std::mutex g_tune_mu;
static std::map<TuneKey, int> g_choice;   // -1: generic kernel, v >= 0: v-th variant

std::vector<const StaticKernel*> static_variants(int kind, int esz, int n, int ntrial, int d,
                                                 const FftPlan& p) {
  std::vector<const StaticKernel*> out;
  for (const StaticKernel& k : static_registry()) {
    // d: components the kernel is built for (0: any)
    if (k.kind != kind || k.esz != esz || k.n != n || k.ntrial != ntrial) continue;
    if (k.d != 0 && k.d != d) continue;
    // the dynamic size a kernel may take (the device limit less 1 KiB for the
    // static LDS of the block reductions)
    if (k.lds > g_static_max_lds) continue;
    // the compile-time plan must describe the same tables the host uploaded
    // (a Rader kernel: the plan's Rader section, lines of n + 1 rows)
    if (k.blue == 2) {
      if (!p.rader || k.len != p.n + 1 || k.nst != p.r_nst) continue;
      bool same = true;
      for (int i = 0; i < p.r_nst; ++i) same = same && (k.rad[i] == p.r_rad[i]);
      if (!same) continue;
      out.push_back(&k);
      continue;
    }
    if (k.len != p.len || k.blue != p.blue || k.nst != p.nst) continue;
    bool same = true;
    for (int i = 0; i < p.nst; ++i) same = same && (k.rad[i] == p.rad[i]);
    if (!same) continue;
    out.push_back(&k);
  }
  return out;
}

void set_choice(const TuneKey& key, int v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_choice[key] = v;
  ++g_tune_version;
}
bool get_choice(const TuneKey& key, int* v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_choice.find(key);
  if (it == g_choice.end()) return false;
  *v = it->second;
  return true;
}
std::map<TuneKey, int> all_choices() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_choice;
}

const StaticKernel* find_static(int kind, int esz, int n, int ntrial, int d, const FftPlan& p) {
  if (!g_static_on) return nullptr;
  std::vector<const StaticKernel*> v = static_variants(kind, esz, n, ntrial, d, p);
  if (v.empty()) return nullptr;
  int c = 0;
  if (get_choice(TuneKey{kind, esz, n, ntrial, d}, &c)) {
    if (c < 0) return nullptr;
    if (c < (int)v.size()) return v[c];
  }
  return v[0];
}

// ---------------------------------------------------------------------------
// CG vector update and scalar kernels
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(kThreads) void k_cg_update(CgUpdateArgs<T> a) {
  const int item = blockIdx.y;
  // the projection's booking is visible to later projections through
  // `stopped` (the projection never reads `halt`, which it raises itself)
  if (blockIdx.x == 0 && threadIdx.x == 0) a.sc[item].stopped = a.sc[item].halt;
  if (!item_live(a.sc[item])) return;
  // rounds of CH elements per thread (grid-stride); the first round's loads go
  // out before alpha is derived
  constexpr int CH = 4;
  const long base = (long)item * a.stride;
  const long step = (long)gridDim.x * blockDim.x;
  cpx<T> pv[CH], qv[CH], xv[CH], rv[CH];
  const bool xupd = a.xupd != 0;
  auto load = [&](long e0) {
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      // unconditional (past the end: element count - 1 again, unused)
      const long e = min(e0 + u * step, a.count - 1);
      qv[u] = a.q[base + e];
      rv[u] = a.r[base + e];
      if (xupd) {
        pv[u] = a.p[base + e];
        xv[u] = a.x[base + e];
      }
    }
  };
  // alpha = rho / (p, q), derived by every workgroup from the (p, q) partials
  // (left by the last-axis pass, or the projection) in the same order (their
  // first loads go out ahead of the data's)
  const double* pq = a.pq_part + (long)item * a.P;
  double ph[8];
  if (!a.pq_sc) partials_head(pq, a.pq_n, ph);
  long e0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  load(e0);
  const double g = a.pq_sc ? a.sc[item].pq : partials_finish(pq, a.pq_n, ph);
  if (!(g > 0.0) || !isfinite(g)) {
    // every workgroup derives the breakdown itself; the first one records it
    // for the passes of later iterations (none of this launch reads it)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.sc[item].gamma = g;
      a.sc[item].status = -5;
      a.sc[item].broke = 1;
    }
    return;
  }
  const double alpha64 = a.sc[item].rho / g;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.sc[item].gamma = g;
    a.sc[item].alpha = alpha64;
  }
  const T alpha = T(alpha64);
  double part = 0.0;
  const bool small = a.count < (1L << 31);
  while (e0 < a.count) {
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const long e = e0 + u * step;
      if (e < a.count) {
        if (xupd) {
          xv[u].x += alpha * pv[u].x;
          xv[u].y += alpha * pv[u].y;
          a.x[base + e] = xv[u];
        }
        rv[u].x -= alpha * qv[u].x;
        rv[u].y -= alpha * qv[u].y;
        a.r[base + e] = rv[u];
        // Hermitian weight; 32-bit division where the indices fit (a 64-bit
        // one costs ~100 instructions per element)
        const int hcol = small ? ((int)e / a.n0) % a.H : (int)((e / a.n0) % a.H);
        const double wt = (hcol == 0) ? 1.0 : 2.0;
        part += wt * ((double)rv[u].x * (double)rv[u].x + (double)rv[u].y * (double)rv[u].y);
      }
    }
    e0 += CH * step;
    if (e0 < a.count) load(e0);
  }
  part = block_sum<kThreads>(part);
  if (threadIdx.x == 0) a.partials[(long)item * a.P + blockIdx.x] = part;
}

// each thread takes one pair (k, -k) of the h = 0 plane and writes both of its
// elements: c(k) <- (c(k) + sigma conj(c(-k))) / 2, c(-k) <- sigma conj(c(k))
template <class T>
__global__ __launch_bounds__(kThreads) void k_sym_h0(SymArgs<T> a) {
  const int item = blockIdx.y;
  if (a.sc && !item_live_project(a.sc[item])) return;
  const long n = (long)a.N0 * a.N1;
  for (long f = (long)blockIdx.x * blockDim.x + threadIdx.x; f < n * a.npot;
       f += (long)gridDim.x * blockDim.x) {
    const int pot = (int)(f / n);
    const long pi = f % n;
    const int i0 = (int)(pi / a.N1), i1 = (int)(pi % a.N1);
    const int m0 = i0 ? a.N0 - i0 : 0, m1 = i1 ? a.N1 - i1 : 0;
    if ((long)m0 * a.N1 + m1 < pi) continue;   // the pair's first element takes it
    const T sg = (pot == a.even_pot) ? T(1) : T(-1);
    const long base = (long)item * a.stride + pot * a.pot_stride;
    const long e = base + i0 * a.s0 + i1 * a.s1, em = base + m0 * a.s0 + m1 * a.s1;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cpx<T>* v = a.v[k];
      if (!v) continue;
      const cpx<T> A = v[e], B = v[em];
      const cpx<T> h{T(0.5) * (A.x + sg * B.x), T(0.5) * (A.y - sg * B.y)};
      v[e] = h;
      v[em] = cpx<T>{sg * h.x, -sg * h.y};
    }
  }
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_basis_expand(BasisArgs<T> a) {
  const int item = blockIdx.y;
  if (a.sc && !item_live(a.sc[item])) return;
  const long n = (long)a.N0 * a.inner;
  const int npot = a.g.npot, nf = a.g.nf;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / a.inner), col = (int)(e % a.inner);
    const int k0 = kof(i, a.N0);
    const long src = (long)item * a.c_stride + (long)i * a.si + (long)col * a.sc_;
    cpx<T> cp[3];
#pragma unroll
    for (int pt = 0; pt < 3; ++pt)
      cp[pt] = (pt < npot) ? a.c[src + pt * a.g.pot_stride] : cpx<T>{T(0), T(0)};
    cpx<T>* X = a.Xo + (long)item * a.X_stride + e;
#pragma unroll
    for (int comp = 0; comp < 6; ++comp) {
      if (comp >= nf) break;
      cpx<T> u{T(0), T(0)};
#pragma unroll
      for (int pt = 0; pt < 3; ++pt) {
        if (pt >= npot) break;
        const T bv = pot_comp<T>(a.g, k0, col, comp, pt);
        u.x += bv * cp[pt].x;
        u.y += bv * cp[pt].y;
      }
      X[(long)comp * a.X_cstride] = u;
    }
  }
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_basis_project(BasisArgs<T> a) {
  const int item = blockIdx.y;
  if (a.sc && !item_live_project(a.sc[item])) {
    // as the projection pass: an item whose update broke down stops here
    const ItemScal& q0 = a.sc[item];
    if (q0.active && q0.broke && a.rr_part && blockIdx.x == 0 && threadIdx.x == 0)
      a.sc[item].halt = 1;
    return;
  }
  const long n = (long)a.N0 * a.inner;
  const int npot = a.g.npot, nf = a.g.nf;
  double part = 0.0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / a.inner), col = (int)(e % a.inner);
    const int k0 = kof(i, a.N0);
    const int h = (a.g.d == 3) ? col % a.g.H : col;   // 2-D: the column is h
    const double wt = (h == 0) ? 1.0 : 2.0;
    const cpx<T>* X = a.Xi + (long)item * a.X_stride + e;
    cpx<T> xv[6];
#pragma unroll
    for (int comp = 0; comp < 6; ++comp)
      xv[comp] = (comp < nf) ? X[(long)comp * a.X_cstride] : cpx<T>{T(0), T(0)};
#pragma unroll
    for (int pt = 0; pt < 3; ++pt) {
      if (pt >= npot) break;
      cpx<T> qv{T(0), T(0)};
#pragma unroll
      for (int comp = 0; comp < 6; ++comp) {
        if (comp >= nf) break;
        const T bv = pot_comp<T>(a.g, k0, col, comp, pt);
        qv.x += bv * xv[comp].x;
        qv.y += bv * xv[comp].y;
      }
      const long idx = (long)item * a.c_stride + pt * a.g.pot_stride + (long)i * a.si +
                       (long)col * a.sc_;
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
    part = block_sum<kThreads>(part);
    if (threadIdx.x == 0) a.partials[(long)item * a.P + blockIdx.x] = part;
  }
  if (a.rr_part && blockIdx.x == 0) {
    // bookkeeping of the update before this iteration's expansion, as the
    // projection pass does it
    const bool fresh = a.sc[item].fresh != 0;
    const double s = fresh ? 0.0 : sum_partials_wave(a.rr_part + (long)item * a.P, a.rr_n);
    if (threadIdx.x == 0) {
      if (fresh) a.sc[item].fresh = 0;
      else cg_book(a.sc[item], s);
    }
  }
  if (a.pq_part && blockIdx.x == 0) pq_total(a.sc[item], a.pq_part + (long)item * a.P, a.pq_n);
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_norm_parts(const cpx<T>* v, long stride, long count,
                                                          int n0, int H, double* part, int P,
                                                          const ItemScal* sc) {
  const int item = blockIdx.y;
  if (sc && !item_live_project(sc[item])) return;
  double s = 0.0;
  const bool small = count < (1L << 31);
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (long)gridDim.x * blockDim.x) {
    const cpx<T> x = v[(long)item * stride + e];
    const int h = small ? ((int)e / n0) % H : (int)((e / n0) % H);
    s += (h == 0 ? 1.0 : 2.0) * ((double)x.x * (double)x.x + (double)x.y * (double)x.y);
  }
  s = block_sum<kThreads>(s);
  if (threadIdx.x == 0) part[(long)item * P + blockIdx.x] = s;
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_cg_direction(CgDirArgs<T> a) {
  const int item = blockIdx.y;
  if (!item_live(a.sc[item])) return;
  constexpr int CH = 4;
  const long base = (long)item * a.stride;
  const long step = (long)gridDim.x * blockDim.x;
  const bool xd = a.xdef != 0;
  cpx<T> rv[CH], pv[CH], xv[CH];
  auto load = [&](long e0) {
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const long e = min(e0 + u * step, a.count - 1);
      rv[u] = a.r[base + e];
      pv[u] = a.p[base + e];
      if (xd) xv[u] = a.x[base + e];
    }
  };
  // beta and the stopping test, derived by every workgroup in the same order
  // from the last update's partials (their first loads go out ahead of the
  // data's); the projection's first workgroup books the same decision later
  const ItemScal q = a.sc[item];
  const bool derive = !q.fresh;
  double ph[8];
  const double* rr = a.rr_part + (long)item * a.P;
  if (derive) partials_head(rr, a.rr_n, ph);
  long e0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  load(e0);
  bool stop = false;
  T beta = T(q.beta);
  if (derive) {
    const double s = partials_finish(rr, a.rr_n, ph);
    stop = cg_stops(q, s);
    beta = T(s / q.rho);
  }
  const T alpha = T(q.alpha);
  while (e0 < a.count) {
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const long e = e0 + u * step;
      if (e < a.count) {
        if (xd) {
          xv[u].x += alpha * pv[u].x;
          xv[u].y += alpha * pv[u].y;
          a.x[base + e] = xv[u];
        }
        // an item that stops keeps p (x is final); beta = 0 restarts: p = r
        if (!stop)
          a.p[base + e] = (beta == T(0)) ? rv[u]
                                         : cpx<T>{rv[u].x + beta * pv[u].x, rv[u].y + beta * pv[u].y};
      }
    }
    e0 += CH * step;
    if (e0 < a.count) load(e0);
  }
}

__global__ __launch_bounds__(kThreads) void k_cg_init(ItemScal* sc, const double* partials, int P,
                                                      int nparts, const ItemScal* mask,
                                                      const double* ref) {
  const int item = blockIdx.x;
  if (!sc[item].active || (mask && !mask[item].active)) return;
  const double s = sum_partials_wave(partials + (long)item * P, nparts);
  // the stopping test is relative to (b, b) (ref, for a warm start) or to the
  // initial residual itself (a cold start, where r_0 = b)
  const double r0 = ref ? sum_partials_wave(ref + (long)item * P, nparts) : s;
  if (threadIdx.x == 0) {
    ItemScal& q = sc[item];
    q.rho = s;
    q.rho0 = (r0 > 0.0) ? r0 : s;
    q.halt = q.stopped = q.broke = 0;
    q.iters = 0;
    q.beta = 0.0;
    q.alpha = 0.0;
    q.fresh = 1;
    q.status = 0;
    const bool met = (s == 0.0) || sqrt(s / q.rho0) <= q.tol;
    q.conv = met ? 1 : 0;
    q.active = (!met && isfinite(s) && q.max_iter > 0) ? 1 : 0;
    if (!isfinite(s)) q.status = -5;
  }
}

__global__ __launch_bounds__(kThreads) void k_cg_finalize(ItemScal* sc, const double* partials,
                                                          int P, int nparts) {
  // one workgroup per item, after the iterations of a launch: books the last
  // update unless the item stopped before it, then retires a stopped item
  const int item = blockIdx.x;
  const ItemScal q0 = sc[item];
  if (!q0.active) return;
  const bool book = !q0.fresh && !q0.halt && !q0.broke;
  const double s = book ? sum_partials_wave(partials + (long)item * P, nparts) : 0.0;
  if (threadIdx.x == 0) {
    ItemScal& q = sc[item];
    if (book) {
      cg_book(q, s);
      q.fresh = 1;
    }
    if (q.halt || q.broke) {
      q.active = 0;
      q.stopped = 1;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_outer_check(ItemScal* sc, const double* partials,
                                                          int P, int nparts, int init,
                                                          const ItemScal* mask) {
  const int item = blockIdx.x;
  if (!sc[item].active || (mask && !mask[item].active)) return;
  const double s = sum_partials_wave(partials + (long)item * P, nparts);
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
                                                          int n0, ItemScal* outer, ItemScal* inner,
                                                          int max_iter, int keep_dir,
                                                          double* partials, int P,
                                                          const ItemScal* mask) {
  const int item = blockIdx.y;
  if (mask && !mask[item].active) return;
  if (!outer[item].active) {
    if (blockIdx.x == 0 && threadIdx.x == 0) inner[item].active = 0;
    return;
  }
  // one scale per solve, 1 / ||b||, so a kept direction stays consistent
  const double sc = 1.0 / sqrt(outer[item].rho0);
  const long base = (long)item * stride;
  double part = 0.0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (long)gridDim.x * blockDim.x) {
    const cpx<double> v = r64[base + e];
    const cpx<float> w = {(float)(v.x * sc), (float)(v.y * sc)};
    r32[base + e] = w;
    if (!keep_dir) p32[base + e] = w;
    x32[base + e] = cpx<float>{0.f, 0.f};
    const double wt = (((e / n0) % H) == 0) ? 1.0 : 2.0;
    part += wt * ((double)w.x * (double)w.x + (double)w.y * (double)w.y);
  }
  part = block_sum<kThreads>(part);
  if (threadIdx.x == 0) partials[(long)item * P + blockIdx.x] = part;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    inner[item].max_iter = max_iter;
    inner[item].active = 1;
    inner[item].halt = inner[item].stopped = inner[item].broke = 0;
    if (!keep_dir) {
      inner[item].iters = 0;
      inner[item].beta = 0.0;
      inner[item].rho = 0.0;
    }
    outer[item].iters += 1;   // FP64 residual evaluations that (re)started the recursion
  }
}

__global__ __launch_bounds__(kThreads) void k_inner_init(ItemScal* inner, const double* partials,
                                                         int P, int nparts, ItemScal* outer,
                                                         double eta, double theta,
                                                         const ItemScal* mask) {
  const int item = blockIdx.x;
  if ((mask && !mask[item].active) || !outer[item].active) return;
  const double s = sum_partials_wave(partials + (long)item * P, nparts);
  if (threadIdx.x == 0) {
    ItemScal& q = inner[item];
    // residual replacement: carry the direction on with beta rescaled to the
    // replaced residual, beta = (r_new, r_new) / (r_prev, r_prev); a fresh
    // start has rho = 0 and takes p = r
    const bool keep = q.rho > 0.0 && isfinite(q.beta) && q.status == 0 && s <= 4.0 * q.rho;
    q.beta = keep ? q.beta * (s / q.rho) : 0.0;
    q.rho = q.rho0 = s;
    // stop the recursion once its residual fell by eta, or earlier when it
    // predicts the outer tolerance (r32 carries the scale 1 / ||b||)
    const double rel = sqrt(s);
    q.tol = (rel > 0.0) ? fmax(eta, theta * outer[item].tol / rel) : eta;
    q.alpha = 0.0;
    q.fresh = 1;
    q.status = isfinite(s) ? 0 : -5;
    q.conv = (s == 0.0) ? 1 : 0;
    q.active = (s > 0.0 && isfinite(s) && q.iters < q.max_iter) ? 1 : 0;
    if (q.iters >= q.max_iter || !isfinite(s)) outer[item].active = 0;
  }
}

__global__ __launch_bounds__(kThreads) void k_inner_accumulate(cpx<double>* x64,
                                                               const cpx<float>* x32, long stride,
                                                               long count, const ItemScal* outer,
                                                               const ItemScal* mask) {
  const int item = blockIdx.y;
  if (!outer[item].active || (mask && !mask[item].active)) return;
  const double sc = sqrt(outer[item].rho0);
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

// Moulinec-Suquet step bookkeeping, one wave per item (every lane reads the
// scalars before lane 0 writes them; no other kernel runs meanwhile): s =
// (r, r) of the residual r = b - Op x the projection just wrote; the item
// stops when ||r|| <= tol ||b|| (or the budget is spent), else the step
// x += r / lambda follows and is counted
__global__ __launch_bounds__(64) void k_ms_book(ItemScal* sc, const double* partials, int P,
                                                int nparts) {
  const int item = blockIdx.x;
  if (!sc[item].active) return;
  const double s = sum_partials_wave(partials + (long)item * P, nparts);
  if (threadIdx.x == 0) {
    ItemScal& q = sc[item];
    q.rho = s;
    if (!isfinite(s)) {
      q.status = -5;
      q.active = 0;
    } else if (s == 0.0 || sqrt(s / q.rho0) <= q.tol) {
      q.conv = 1;
      q.active = 0;
    } else if (q.iters >= q.max_iter) {
      q.active = 0;
    } else {
      q.iters += 1;
    }
  }
}

// x += r / lambda for every item still iterating
__global__ __launch_bounds__(kThreads) void k_ms_axpy(cpx<double>* x, const cpx<double>* r,
                                                      long stride, long count,
                                                      const ItemScal* sc) {
  const int item = blockIdx.y;
  if (!sc[item].active) return;
  const double step = sc[item].step;
  const long base = (long)item * stride;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (long)gridDim.x * blockDim.x) {
    cpx<double> xv = x[base + e];
    const cpx<double> rv = r[base + e];
    xv.x += step * rv.x;
    xv.y += step * rv.y;
    x[base + e] = xv;
  }
}

__global__ void k_set_scal(ItemScal* sc, int items, double tol, int max_iter, int active,
                           double step) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < items) {
    ItemScal q{};
    q.step = step;
    q.tol = tol;
    q.max_iter = max_iter;
    q.active = active;
    sc[i] = q;
  }
}

// ---------------------------------------------------------------------------
// coefficient validation on the device: eigenvalue range and flags
// ---------------------------------------------------------------------------
constexpr int kRangeBlocks = 1024;

__global__ __launch_bounds__(kThreads) void k_a_range(const double* A, int d, int kind, long npts,
                                                      double* out) {
  const int nA = coef_values(kind, d);
  double lo = INFINITY, hi = 0.0;
  int flags = 0;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npts;
       p += (long)gridDim.x * blockDim.x) {
    double v[6], l = 0.0, h = 0.0;
    bool finite = true;
    for (int t = 0; t < nA; ++t) {
      v[t] = A[(long)t * npts + p];
      finite = finite && isfinite(v[t]);
    }
    if (!finite) {
      flags |= 1;
    } else if (!point_range(d, kind, v, &l, &h)) {
      flags |= 2;
    } else {
      lo = fmin(lo, l);
      hi = fmax(hi, h);
    }
  }
  __shared__ double slo[kThreads], shi[kThreads];
  __shared__ int sfl[kThreads];
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  sfl[threadIdx.x] = flags;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + o]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + o]);
      sfl[threadIdx.x] |= sfl[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[3 * blockIdx.x] = slo[0];
    out[3 * blockIdx.x + 1] = shi[0];
    out[3 * blockIdx.x + 2] = (double)sfl[0];
  }
}

hipError_t a_field_range(const double* A, int d, int kind, long npts, double* scratch,
                         double* host, hipStream_t s, double* lo, double* hi, int* flags) {
  const int blocks = (int)std::max(1L, std::min((long)kRangeBlocks, (npts + kThreads - 1) / kThreads));
  static_assert(3 * kRangeBlocks <= kQuadScratch, "range partials exceed the scratch buffer");
  hipLaunchKernelGGL(k_a_range, dim3(blocks), dim3(kThreads), 0, s, A, d, kind, npts, scratch);
  hipError_t e = hipGetLastError();
  double* h = host;
  if (e == hipSuccess)
    e = hipMemcpyAsync(h, scratch, sizeof(double) * 3 * blocks, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  *lo = INFINITY;
  *hi = 0.0;
  *flags = 0;
  for (int b = 0; b < blocks; ++b) {
    *lo = std::min(*lo, h[3 * b]);
    *hi = std::max(*hi, h[3 * b + 1]);
    *flags |= (int)h[3 * b + 2];
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// FP64 energy quadrature W_lm = <e_l . A e_m>, J_l = <A e_l>
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(kThreads) void k_quad(const double* e, long es, long ecs,
                                                   const double* A, long Acs, int kind,
                                                   long npts, int l0, int nl, int m0, int nm,
                                                   double* partials) {
  // D components and at most 3 x 3 load-case pairs: every loop has a
  // compile-time bound, so the accumulators stay in registers
  constexpr int NS = 9 + 3 * D;   // W slots l * 3 + m, then J slots 9 + m * D + q
  double acc[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) acc[t] = 0.0;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npts;
       p += (long)gridDim.x * blockDim.x) {
    double c[6];
    load_coef<double>(kind, D, A, Acs, p, c);
    double el[3][D];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int q = 0; q < D; ++q) el[l][q] = (l < nl) ? e[(l0 + l) * es + q * ecs + p] : 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if (m >= nm) break;
      double em[D], jm[D];
#pragma unroll
      for (int q = 0; q < D; ++q) em[q] = e[(m0 + m) * es + q * ecs + p];
      flux_coef<double>(kind, D, c, em, jm);
#pragma unroll
      for (int q = 0; q < D; ++q) acc[9 + m * D + q] += jm[q];
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) sum += el[l][q] * jm[q];
        acc[l * 3 + m] += sum;
      }
    }
  }
  // per wave, then across the waves in order (one barrier)
  __shared__ double red[kThreads / 64][NS];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    double v = acc[t];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) red[wid][t] = v;
  }
  __syncthreads();
  if (threadIdx.x < NS) {
    double v = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) v += red[w][threadIdx.x];
    partials[(long)blockIdx.x * kQuadSlots + threadIdx.x] = v;
  }
}

__global__ __launch_bounds__(kThreads) void k_quad_final(const double* partials, int blocks,
                                                         long npts, double* out) {
  // workgroup t: out[t], t < 9 a W slot (3x3), t >= 9 a J sum, divided by npts
  const int t = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < blocks; b += blockDim.x) v += partials[(long)b * kQuadSlots + t];
  v = block_sum<kThreads>(v);
  if (threadIdx.x == 0) out[t] = v / (double)npts;
}

__global__ void k_convert(const double* in, float* out, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

__global__ void k_zero(double* p, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void k_widen(const float* in, double* out, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// events armed for the next launches of this thread: the first dispatch
// records the start, the last one the stop, so the interval is the kernels'
// own, with no marker packet added
static thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;
static thread_local int t_ev_left = 0;
void arm_launch_events(hipEvent_t start, hipEvent_t stop, int launches) {
  t_ev_start = start;
  t_ev_stop = stop;
  t_ev_left = (start || stop) ? launches : 0;
}

template <class F, class... Args>
static void launch_k(F fn, dim3 grid, dim3 block, size_t lds, hipStream_t s, Args... args) {
  if (t_ev_left > 0) {
    hipEvent_t a = t_ev_start, z = (t_ev_left == 1) ? t_ev_stop : nullptr;
    t_ev_start = nullptr;
    if (--t_ev_left == 0) t_ev_stop = nullptr;
    hipExtLaunchKernelGGL(fn, grid, block, (std::uint32_t)lds, s, a, z, 0u, args...);
  } else {
    hipLaunchKernelGGL(fn, grid, block, lds, s, args...);
  }
}

template <class T>
hipError_t launch_col_expand(const ColExpandArgs<T>& a, int items, size_t lds, hipStream_t s,
                             const StaticKernel* sk) {
  dim3 grid(ceil_div(a.inner, a.W), items);
  if (sk) {
    auto fn = reinterpret_cast<void (*)(ColExpandArgs<T>)>(const_cast<void*>(sk->fn));
    launch_k(fn, grid, dim3(sk->NT), sk->lds, s, a);
    return hipGetLastError();
  }
  const long npos = (long)a.n_in * a.W;
  if (npos <= 8L * kThreads)
    launch_k((k_col_expand<T, ColGen, 8>), grid, dim3(kThreads), lds, s, a);
  else if (npos <= 16L * kThreads)
    launch_k((k_col_expand<T, ColGen, 16>), grid, dim3(kThreads), lds, s, a);
  else if (npos <= 32L * kThreads)
    launch_k((k_col_expand<T, ColGen, 32>), grid, dim3(kThreads), lds, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class T>
hipError_t launch_col_plain(const ColPlainArgs<T>& a, int items, int sign, size_t lds,
                            hipStream_t s, const StaticKernel* sk) {
  dim3 grid(ceil_div(a.inner, a.W), a.outer, items * a.d);
  if (sk) {
    auto fn = reinterpret_cast<void (*)(ColPlainArgs<T>)>(const_cast<void*>(sk->fn));
    launch_k(fn, grid, dim3(sk->NT), sk->lds, s, a);
    return hipGetLastError();
  }
  if (sign < 0)
    launch_k((k_col_plain<T, ColGen, -1>), grid, dim3(kThreads), lds, s, a);
  else
    launch_k((k_col_plain<T, ColGen, +1>), grid, dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_col_project(const ColProjectArgs<T>& a, int items, size_t lds, hipStream_t s,
                              const StaticKernel* sk) {
  dim3 grid(ceil_div(a.inner, a.W), items);
  if (sk) {
    auto fn = reinterpret_cast<void (*)(ColProjectArgs<T>)>(const_cast<void*>(sk->fn));
    launch_k(fn, grid, dim3(sk->NT), sk->lds, s, a);
    return hipGetLastError();
  }
  const long npos = (long)a.n_out * a.W;
  if (npos <= 8L * kThreads)
    launch_k((k_col_project<T, ColGen, 8>), grid, dim3(kThreads), lds, s, a);
  else if (npos <= 16L * kThreads)
    launch_k((k_col_project<T, ColGen, 16>), grid, dim3(kThreads), lds, s, a);
  else if (npos <= 32L * kThreads)
    launch_k((k_col_project<T, ColGen, 32>), grid, dim3(kThreads), lds, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class T>
hipError_t launch_row(const RowArgs<T>& a0, int items, int mode, size_t lds, hipStream_t s,
                      const StaticKernel* sk) {
  RowArgs<T> a = a0;
  a.items = items;
  const long pairs = (a.rows + 1) / 2;
  dim3 grid(ceil_div(pairs, a.RP), items);
  if (sk) {
    const int kind = (mode == ROW_APPLY) ? KK_ROW : (mode == ROW_CONST) ? KK_ROW_CONST
                   : (mode == ROW_SYNTH) ? KK_ROW_SYNTH : -1;
    if (sk->kind != kind) return hipErrorInvalidValue;
    if (sk->ilv) grid = dim3(ceil_div(pairs, a.RP) * items, 1);
    if (sk->ipw > 1) grid = dim3(ceil_div(pairs, a.RP), ceil_div(items, sk->ipw));
    auto fn = reinterpret_cast<void (*)(RowArgs<T>)>(const_cast<void*>(sk->fn));
    launch_k(fn, grid, dim3(sk->NT), sk->lds, s, a);
    return hipGetLastError();
  }
  switch (mode) {
    case ROW_APPLY: launch_k((k_row<T, RowGen, ROW_APPLY>), grid, dim3(kThreads), lds, s, a); break;
    case ROW_CONST: launch_k((k_row<T, RowGen, ROW_CONST>), grid, dim3(kThreads), lds, s, a); break;
    case ROW_SYNTH: launch_k((k_row<T, RowGen, ROW_SYNTH>), grid, dim3(kThreads), lds, s, a); break;
    case ROW_FWD: launch_k((k_row<T, RowGen, ROW_FWD>), grid, dim3(kThreads), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_cg_direction(const CgDirArgs<T>& a, int items, int blocks, hipStream_t s) {
  launch_k((k_cg_direction<T>), dim3(blocks, items), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_cg_update(const CgUpdateArgs<T>& a, int items, int blocks, hipStream_t s) {
  launch_k((k_cg_update<T>), dim3(blocks, items), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_cg_init(ItemScal* sc, const double* partials, int P, int nparts, int items,
                          hipStream_t s, const ItemScal* mask, const double* ref) {
  launch_k(k_cg_init, dim3(items), dim3(64), 0, s, sc, partials, P, nparts, mask, ref);
  return hipGetLastError();
}
hipError_t launch_cg_finalize(ItemScal* sc, const double* partials, int P, int nparts, int items,
                              hipStream_t s) {
  launch_k(k_cg_finalize, dim3(items), dim3(64), 0, s, sc, partials, P, nparts);
  return hipGetLastError();
}
hipError_t launch_outer_check(ItemScal* sc, const double* partials, int P, int nparts, int items,
                              int init, hipStream_t s, const ItemScal* mask) {
  launch_k(k_outer_check, dim3(items), dim3(64), 0, s, sc, partials, P, nparts,
                     init, mask);
  return hipGetLastError();
}
hipError_t launch_inner_start(const cpx<double>* r64, cpx<float>* r32, cpx<float>* p32,
                              cpx<float>* x32, long stride, long count, int H, int n0,
                              ItemScal* outer, ItemScal* inner, int max_iter, int keep_dir,
                              double* partials, int P, int blocks, int items, hipStream_t s,
                              const ItemScal* mask) {
  launch_k(k_inner_start, dim3(blocks, items), dim3(kThreads), 0, s, r64, r32, p32, x32,
                     stride, count, H, n0, outer, inner, max_iter, keep_dir, partials, P, mask);
  return hipGetLastError();
}
hipError_t launch_inner_init(ItemScal* inner, const double* partials, int P, int nparts, int items,
                             ItemScal* outer, double eta, double theta, hipStream_t s,
                             const ItemScal* mask) {
  launch_k(k_inner_init, dim3(items), dim3(64), 0, s, inner, partials, P, nparts,
                     outer, eta, theta, mask);
  return hipGetLastError();
}
hipError_t launch_inner_accumulate(cpx<double>* x64, const cpx<float>* x32, long stride, long count,
                                   const ItemScal* outer, int blocks, int items, hipStream_t s,
                                   const ItemScal* mask) {
  launch_k(k_inner_accumulate, dim3(blocks, items), dim3(kThreads), 0, s, x64, x32,
                     stride, count, outer, mask);
  return hipGetLastError();
}
hipError_t launch_ms_book(ItemScal* sc, const double* partials, int P, int nparts, int items,
                          hipStream_t s) {
  launch_k(k_ms_book, dim3(items), dim3(64), 0, s, sc, partials, P, nparts);
  return hipGetLastError();
}
hipError_t launch_ms_axpy(cpx<double>* x, const cpx<double>* r, long stride, long count,
                          const ItemScal* sc, int blocks, int items, hipStream_t s) {
  launch_k(k_ms_axpy, dim3(blocks, items), dim3(kThreads), 0, s, x, r, stride, count, sc);
  return hipGetLastError();
}
hipError_t launch_set_scal(ItemScal* sc, int items, double tol, int max_iter, int active,
                           hipStream_t s, double step) {
  launch_k(k_set_scal, dim3(ceil_div(items, 64)), dim3(64), 0, s, sc, items, tol,
                     max_iter, active, step);
  return hipGetLastError();
}
hipError_t launch_quad(const double* e, long e_stride, long e_cstride, const double* A,
                       long A_cstride, int kind, int d, long npts, int l0, int nl, int m0, int nm,
                       double* partials, int blocks, hipStream_t s) {
  if (nl < 1 || nl > 3 || nm < 1 || nm > 3) return hipErrorInvalidValue;
  switch (d) {
    case 1: launch_k(k_quad<1>, dim3(blocks), dim3(kThreads), 0, s, e, e_stride, e_cstride, A,
                     A_cstride, kind, npts, l0, nl, m0, nm, partials); break;
    case 2: launch_k(k_quad<2>, dim3(blocks), dim3(kThreads), 0, s, e, e_stride, e_cstride, A,
                     A_cstride, kind, npts, l0, nl, m0, nm, partials); break;
    case 3: launch_k(k_quad<3>, dim3(blocks), dim3(kThreads), 0, s, e, e_stride, e_cstride, A,
                     A_cstride, kind, npts, l0, nl, m0, nm, partials); break;
    case 6: launch_k(k_quad<6>, dim3(blocks), dim3(kThreads), 0, s, e, e_stride, e_cstride, A,
                     A_cstride, kind, npts, l0, nl, m0, nm, partials); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_quad_final(const double* partials, int blocks, int nl, int nm, int d, long npts,
                             double* out, hipStream_t s) {
  (void)nl;
  (void)nm;
  launch_k(k_quad_final, dim3(9 + 3 * d), dim3(kThreads), 0, s, partials, blocks, npts, out);
  return hipGetLastError();
}
hipError_t launch_convert(const double* in, float* out, long n, hipStream_t s) {
  int blocks = ceil_div(n, kThreads);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  launch_k(k_convert, dim3(blocks), dim3(kThreads), 0, s, in, out, n);
  return hipGetLastError();
}

template <class T>
hipError_t launch_sym_h0(const SymArgs<T>& a, int items, hipStream_t s) {
  int blocks = ceil_div((long)a.N0 * a.N1 * a.npot, kThreads);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  launch_k((k_sym_h0<T>), dim3(blocks, items), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_basis_expand(const BasisArgs<T>& a, int items, int blocks, hipStream_t s) {
  launch_k((k_basis_expand<T>), dim3(blocks, items), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_basis_project(const BasisArgs<T>& a, int items, int blocks, hipStream_t s) {
  if (blocks < 1 || blocks > a.P) return hipErrorInvalidValue;
  launch_k((k_basis_project<T>), dim3(blocks, items), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_norm_parts(const cpx<T>* v, long stride, long count, int n0, int H,
                             double* part, int P, int blocks, int items, const ItemScal* sc,
                             hipStream_t s) {
  if (blocks < 1 || blocks > P) return hipErrorInvalidValue;
  launch_k((k_norm_parts<T>), dim3(blocks, items), dim3(kThreads), 0, s, v, stride, count, n0, H,
           part, P, sc);
  return hipGetLastError();
}

hipError_t launch_zero(double* p, long n, hipStream_t s) {
  int blocks = ceil_div(n, kThreads);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  launch_k(k_zero, dim3(blocks), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_widen(const float* in, double* out, long n, hipStream_t s) {
  int blocks = ceil_div(n, kThreads);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  launch_k(k_widen, dim3(blocks), dim3(kThreads), 0, s, in, out, n);
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
  HOM_SET((k_col_expand<float, ColGen, 8>));
  HOM_SET((k_col_expand<float, ColGen, 16>));
  HOM_SET((k_col_expand<float, ColGen, 32>));
  HOM_SET((k_col_expand<double, ColGen, 8>));
  HOM_SET((k_col_expand<double, ColGen, 16>));
  HOM_SET((k_col_expand<double, ColGen, 32>));
  HOM_SET((k_col_project<float, ColGen, 8>));
  HOM_SET((k_col_project<float, ColGen, 16>));
  HOM_SET((k_col_project<float, ColGen, 32>));
  HOM_SET((k_col_project<double, ColGen, 8>));
  HOM_SET((k_col_project<double, ColGen, 16>));
  HOM_SET((k_col_project<double, ColGen, 32>));
  HOM_SET((k_col_plain<float, ColGen, -1>));
  HOM_SET((k_col_plain<float, ColGen, 1>));
  HOM_SET((k_col_plain<double, ColGen, -1>));
  HOM_SET((k_col_plain<double, ColGen, 1>));
  HOM_SET((k_row<float, RowGen, ROW_APPLY>));
  HOM_SET((k_row<float, RowGen, ROW_CONST>));
  HOM_SET((k_row<float, RowGen, ROW_SYNTH>));
  HOM_SET((k_row<float, RowGen, ROW_FWD>));
  HOM_SET((k_row<double, RowGen, ROW_APPLY>));
  HOM_SET((k_row<double, RowGen, ROW_CONST>));
  HOM_SET((k_row<double, RowGen, ROW_SYNTH>));
  HOM_SET((k_row<double, RowGen, ROW_FWD>));
#undef HOM_SET
  for (const StaticKernel& k : static_registry()) {
    if (k.lds > max_lds) continue;  // never selected on this device (see static_variants)
    hipError_t e2 = hipFuncSetAttribute(k.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)max_lds);
    if (e2 != hipSuccess) e = e2;
  }
  g_static_max_lds = max_lds;
  return e;
}

template hipError_t launch_col_expand<float>(const ColExpandArgs<float>&, int, size_t, hipStream_t, const StaticKernel*);
template hipError_t launch_col_expand<double>(const ColExpandArgs<double>&, int, size_t, hipStream_t, const StaticKernel*);
template hipError_t launch_col_plain<float>(const ColPlainArgs<float>&, int, int, size_t, hipStream_t, const StaticKernel*);
template hipError_t launch_col_plain<double>(const ColPlainArgs<double>&, int, int, size_t, hipStream_t, const StaticKernel*);
template hipError_t launch_col_project<float>(const ColProjectArgs<float>&, int, size_t, hipStream_t, const StaticKernel*);
template hipError_t launch_col_project<double>(const ColProjectArgs<double>&, int, size_t, hipStream_t, const StaticKernel*);
template hipError_t launch_row<float>(const RowArgs<float>&, int, int, size_t, hipStream_t, const StaticKernel*);
template hipError_t launch_row<double>(const RowArgs<double>&, int, int, size_t, hipStream_t, const StaticKernel*);
template hipError_t launch_cg_direction<float>(const CgDirArgs<float>&, int, int, hipStream_t);
template hipError_t launch_cg_direction<double>(const CgDirArgs<double>&, int, int, hipStream_t);
template hipError_t launch_basis_expand<float>(const BasisArgs<float>&, int, int, hipStream_t);
template hipError_t launch_basis_expand<double>(const BasisArgs<double>&, int, int, hipStream_t);
template hipError_t launch_basis_project<float>(const BasisArgs<float>&, int, int, hipStream_t);
template hipError_t launch_basis_project<double>(const BasisArgs<double>&, int, int, hipStream_t);
template hipError_t launch_sym_h0<float>(const SymArgs<float>&, int, hipStream_t);
template hipError_t launch_sym_h0<double>(const SymArgs<double>&, int, hipStream_t);
template hipError_t launch_norm_parts<float>(const cpx<float>*, long, long, int, int, double*, int,
                                             int, int, const ItemScal*, hipStream_t);
template hipError_t launch_norm_parts<double>(const cpx<double>*, long, long, int, int, double*,
                                              int, int, int, const ItemScal*, hipStream_t);
template hipError_t launch_cg_update<float>(const CgUpdateArgs<float>&, int, int, hipStream_t);
template hipError_t launch_cg_update<double>(const CgUpdateArgs<double>&, int, int, hipStream_t);

}  // namespace hom

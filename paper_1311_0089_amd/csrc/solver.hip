// solver.hip -- cell setup, operator pipelines, CG drivers (FP64 and mixed
// FP32/FP64 refinement), energy quadrature and the C ABI of hom.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <type_traits>
#include <vector>

#include "cell.hpp"


namespace hom {

// dynamic LDS budgets leave 1 KiB for the static LDS of the block reductions
static size_t g_lds_budget = 63 * 1024;   // preferred: two or more workgroups per CU
static size_t g_lds_max = 63 * 1024;      // device limit minus headroom (set once)
static bool g_configured = false;
static std::mutex g_cfg_mu;

static hipError_t ensure_configured() {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  if (g_configured) return hipSuccess;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return e;
  // a workgroup may take the whole LDS of a CU where the device allows it
  // (gfx950: 160 KiB); the tuner decides whether the large tiles pay
  size_t mx = std::max(prop.sharedMemPerBlock, prop.sharedMemPerBlockOptin);
  if (mx < 64 * 1024) mx = 64 * 1024;
  if (mx > 160 * 1024) mx = 160 * 1024;
  // 1 KiB stays free for the static LDS of the block reductions: a dynamic
  // size that would take a workgroup's whole LDS is refused for kernels
  // that also hold static LDS
  e = configure_kernels(mx - 1024);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    mx = 64 * 1024;
    e = configure_kernels(mx - 1024);
  }
  g_lds_max = mx - 1024;
  g_configured = (e == hipSuccess);
  return e;
}

template <class T>
Work<T>::~Work() {
  for (void* p : owned) (void)hipFree(p);
}

template <class T>
hipError_t Work<T>::alloc(int n, long S, long Xe, int d, int P) {
  for (void* p : owned) (void)hipFree(p);
  owned.clear();
  items = 0;
  auto get = [&](void** ptr, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(ptr, bytes > 0 ? bytes : 16);
    if (e == hipSuccess) owned.push_back(*ptr);
    return e;
  };
  const size_t sv = sizeof(cpx<T>) * (size_t)S * n;
  const size_t xv = sizeof(cpx<T>) * (size_t)Xe * d * n;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = get((void**)&x, sv);
  if (e == hipSuccess) e = get((void**)&r, sv);
  if (e == hipSuccess) e = get((void**)&p, sv);
  if (e == hipSuccess) e = get((void**)&q, sv);
  if (e == hipSuccess) e = get((void**)&b, sv);
  if (e == hipSuccess) e = get((void**)&X1, xv);
  if (e == hipSuccess) e = get((void**)&X2, xv);
  if (e == hipSuccess) e = get((void**)&part, sizeof(double) * (size_t)P * n);
  if (e == hipSuccess) e = get((void**)&part2, sizeof(double) * (size_t)P * n);
  if (e == hipSuccess) e = get((void**)&sc, sizeof(ItemScal) * (size_t)n);
  if (e == hipSuccess) e = get((void**)&mask, sizeof(ItemScal) * (size_t)n);
  if (e == hipSuccess) items = n;
  return e;
}
template struct Work<float>;
template struct Work<double>;

template <>
Work<double>& work_of<double>(CellImpl* c) { return c->w64; }
template <>
Work<float>& work_of<float>(CellImpl* c) { return c->w32; }

CellImpl::~CellImpl() {
  for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
  if (A64) (void)hipFree(A64);
  if (A32) (void)hipFree(A32);
  if (ebuf) (void)hipFree(ebuf);
  if (quad) (void)hipFree(quad);
  if (dE) (void)hipFree(dE);
  if (stream) (void)hipStreamDestroy(stream);
}

// Pinned host staging, one buffer per host thread (grown on demand, kept for
// the thread's life): cells are not re-entrant, so a thread's cells never
// use it concurrently, and thousands of cells cost no pinned memory each.
hipError_t pinned(CellImpl* c, size_t bytes, void** out) {
  (void)c;
  static thread_local void* buf = nullptr;
  static thread_local size_t cap = 0;
  if (cap < bytes) {
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    cap = 0;
    const size_t want = std::max<size_t>(bytes, 64 * 1024);
    hipError_t e = hipHostMalloc(&buf, want, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    cap = want;
  }
  *out = buf;
  return hipSuccess;
}

// device scratch of the coefficient check, one per device (creation only)
static std::mutex g_range_mu;
static hipError_t range_scratch(int device, double** out) {
  static std::map<int, double*> bufs;
  auto it = bufs.find(device);
  if (it != bufs.end()) {
    *out = it->second;
    return hipSuccess;
  }
  double* p = nullptr;
  hipError_t e = hipMalloc(&p, sizeof(double) * kQuadScratch);
  if (e != hipSuccess) return e;
  bufs[device] = p;
  *out = p;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// launch shapes
// ---------------------------------------------------------------------------
struct ColShape {
  int W = 0;
  size_t lds = 0;
};

static hipError_t col_shape(const FftPlan& p, int npos_rows, int inner, int esz, ColShape* s) {
  s->W = choose_col_W(p, npos_rows, inner, esz, g_lds_budget, &s->lds);
  if (!s->W) s->W = choose_col_W(p, npos_rows, inner, esz, g_lds_max, &s->lds);
  return s->W ? hipSuccess : hipErrorInvalidConfiguration;
}

static hipError_t row_shape(const FftPlan& p, int d, long rows, int esz, int* RP, size_t* lds) {
  *RP = choose_row_RP(p, d, rows, esz, g_lds_budget, lds);
  if (!*RP) *RP = choose_row_RP(p, d, rows, esz, g_lds_max, lds);
  return *RP ? hipSuccess : hipErrorInvalidConfiguration;
}

template <class T>
static const cpx<T>* tw_of(const DevPlan* p);
template <>
const cpx<double>* tw_of<double>(const DevPlan* p) { return p->tw64; }
template <>
const cpx<float>* tw_of<float>(const DevPlan* p) { return p->tw32; }

int update_blocks(long S) {
  long b = (S + kThreads - 1) / kThreads;
  if (b > 512) b = 512;
  if (b < 1) b = 1;
  return (int)b;
}

int partial_slots(const CellImpl* c) {
  // enough for every producer: column tiles (<= inner), last-axis tiles
  // (<= row pairs) and update blocks
  long inner = (c->dd == 3) ? (long)c->N[1] * c->H : c->H;
  long rows = (c->dd == 3) ? (long)c->Q[0] * c->Q[1] : c->Q[0];
  long P = std::max<long>(std::max<long>(inner, (rows + 1) / 2), 512);
  return (int)P;
}

hipError_t cell_setup(CellImpl* c) {
  hipError_t e = ensure_configured();
  if (e != hipSuccess) return e;
  const int dd = c->dd;
  c->H = (c->N[dd - 1] + 1) / 2;
  c->nN = 1;
  c->nQ = 1;
  for (int a = 0; a < dd; ++a) {
    c->nN *= c->N[a];
    c->nQ *= c->Q[a];
  }
  c->S = (long)c->H;
  c->Xe = (long)c->H;
  for (int a = 0; a < dd - 1; ++a) {
    c->S *= c->N[a];
    c->Xe *= c->Q[a];
  }
  // the 3-D dual problem has two potentials per frequency, stored one after
  // the other: every CG vector kernel sees them as one spectrum of 2S elements
  c->elastic = (c->kind == HOM_A_ELASTIC);
  c->npot = c->elastic ? dd : (c->dual && dd == 3) ? 2 : 1;
  c->nf = c->elastic ? dd * (dd + 1) / 2 : dd;
  c->S *= c->npot;
  // plans for every length used
  const DevPlan* p = nullptr;
  for (int a = 0; a < dd; ++a) {
    if ((e = get_dev_plan(c->Q[a], &p)) != hipSuccess) return e;
    if ((e = get_dev_plan(c->N[a], &p)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t ensure_work(CellImpl* c, int items, bool need32) {
  const int P = partial_slots(c);
  hipError_t e = hipSuccess;
  bool realloc = false;
  if (c->w64.items < items) {
    if ((e = c->w64.alloc(items, c->S, c->Xe, c->nf, P)) != hipSuccess) return e;
    realloc = true;
  }
  if (need32 && c->w32.items < items) {
    if ((e = c->w32.alloc(items, c->S, c->Xe, c->nf, P)) != hipSuccess) return e;
    realloc = true;
  }
  if (realloc) {
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
  }
  return e;
}

// ---------------------------------------------------------------------------
// pipeline stages on the quadrature grid
// ---------------------------------------------------------------------------
static NormalGeo normal_geo(const CellImpl* c) {
  NormalGeo g{};
  g.d = c->dd;
  g.N1 = (c->dd == 3) ? c->N[1] : 1;
  g.H = c->H;
  g.dual = c->dual;
  g.npot = c->npot;
  g.pot_stride = c->S / c->npot;
  g.nf = c->nf;
  g.elastic = c->elastic;
  for (int a = 0; a < 3; ++a) g.invY[a] = 1.0 / c->Y[a];
  return g;
}

// the compile-time expand / project kernels serve one potential per
// frequency; a cell with two (3-D dual) runs the generic ones
static const StaticKernel* col_static(const CellImpl* c, int kind, int esz, int n,
                                      const FftPlan& p) {
  if (c->npot > 1) return nullptr;
  return find_static(kind, esz, n, c->N[0], c->dd, p);
}

static long inner0(const CellImpl* c) { return (c->dd == 3) ? (long)c->N[1] * c->H : c->H; }

// the fused expansion kernel of a 3-D elastic cell's first axis, if any
template <class T>
static const StaticKernel* bexpand_kernel(const CellImpl* c) {
  if (!c->elastic || c->dd != 3) return nullptr;
  const DevPlan* p0;
  if (get_dev_plan(c->Q[0], &p0) != hipSuccess) return nullptr;
  return find_static(KK_BEXPAND, (int)sizeof(cpx<T>), c->Q[0], c->N[0], c->nf, p0->p);
}

// 3-D cells of one potential whose FP32 first- and middle-axis passes hand two
// spectra to each other instead of three (X_0 and Z = F_0^-1[c / |xi|] on the
// way in, X_0 and xi_1 X_1 + xi_2 X_2 on the way out; the middle-axis passes
// apply xi_1 and xi_2): when each of the four passes has such a kernel for
// the shape.  Every pass decides it the same way, so they agree.
template <class T>
static bool pair_mode(const CellImpl* c) {
  if (c->dd != 3 || c->npot != 1) return false;
  const DevPlan *p0, *p1;
  if (get_dev_plan(c->Q[0], &p0) != hipSuccess || get_dev_plan(c->Q[1], &p1) != hipSuccess)
    return false;
  const int esz = (int)sizeof(cpx<T>);
  return find_static(KK_EXPAND2, esz, c->Q[0], c->N[0], 3, p0->p) &&
         find_static(KK_PROJECT2, esz, c->Q[0], c->N[0], 3, p0->p) &&
         find_static(KK_MID2_INV, esz, c->Q[1], c->N[1], 0, p1->p) &&
         find_static(KK_MID2_FWD, esz, c->Q[1], c->N[1], 0, p1->p);
}

// the two-spectra form for passes over a G0 x G1 grid: the cell's form on the
// quadrature grid only (the trial-grid synthesis of a Ga cell runs the
// three-spectra kernels of its lengths)
template <class T>
static bool pair_on(const CellImpl* c, int G0, int G1) {
  return G0 == c->Q[0] && G1 == c->Q[1] && pair_mode<T>(c);
}

// Layout of the scalar spectra (c, r, p, q, b, x) of an item: 2-D cells keep
// them column-major (axis 0 contiguous), so the first-axis passes, whose
// tiles are few columns wide there, load and store whole cache lines; 3-D
// cells keep them row-major, where the tiles are wide enough already.
static bool scalar_colmajor(const CellImpl* c) { return c->dd == 2; }
static int scalar_si(const CellImpl* c) { return scalar_colmajor(c) ? 1 : (int)inner0(c); }
static int scalar_sc(const CellImpl* c) { return scalar_colmajor(c) ? c->N[0] : 1; }
// elements per column as the CG vector kernels see them (1: row-major)
int scalar_n0(const CellImpl* c) { return scalar_colmajor(c) ? c->N[0] : 1; }

// workgroups of the basis maps of a cell with several potentials per
// frequency (also the number of partial sums its projection writes)
static int basis_blocks(const CellImpl* c) {
  const long n = (long)c->N[0] * inner0(c);
  return (int)std::max(1L, std::min<long>(512, (n + 4L * kThreads - 1) / (4L * kThreads)));
}

// plain first-axis pass of the component spectra: inverse with padding
// N0 -> G0 (sign > 0) or forward with truncation G0 -> N0, the compile-time
// column kernels of the length where there are some
template <class T>
static hipError_t plain_axis0(CellImpl* c, int items, int sign, int G0, const cpx<T>* in,
                              cpx<T>* out, ItemScal* sc) {
  const DevPlan* p0;
  hipError_t e = get_dev_plan(G0, &p0);
  if (e != hipSuccess) return e;
  ColPlainArgs<T> a{};
  a.in = in;
  a.out = out;
  a.in_stride = a.out_stride = (long)c->nf * c->Xe;
  a.in_cstride = a.out_cstride = c->Xe;
  a.outer = 1;
  a.n_fft = G0;
  a.n_in = (sign > 0) ? c->N[0] : G0;
  a.n_out = (sign > 0) ? G0 : c->N[0];
  a.inner = (int)inner0(c);
  a.d = c->nf;
  a.scale = (sign > 0) ? T(1) : T(1.0 / (double)G0);
  a.plan = p0->p;
  a.tw = tw_of<T>(p0);
  a.sc = sc;
  const StaticKernel* sk = find_static(sign > 0 ? KK_PLAIN_INV : KK_PLAIN_FWD, sizeof(cpx<T>),
                                       G0, c->N[0], 0, p0->p);
  if (sk) {
    a.W = sk->W;
    return launch_col_plain<T>(a, items, sign, sk->lds, c->stream, sk);
  }
  ColShape sh;
  if ((e = col_shape(p0->p, std::max(a.n_in, a.n_out), a.inner, sizeof(cpx<T>), &sh)) !=
      hipSuccess)
    return e;
  a.W = sh.W;
  return launch_col_plain<T>(a, items, sign, sh.lds, c->stream);
}

template <class T>
static hipError_t stage_expand(CellImpl* c, Work<T>& w, int items, const cpx<T>* in, int G0,
                               ItemScal* sc, bool pair) {
  const DevPlan* p0;
  hipError_t e = get_dev_plan(G0, &p0);
  if (e != hipSuccess) return e;
  ColExpandArgs<T> a{};
  a.c = in;
  a.X = w.X1;
  a.c_stride = c->S;
  a.si = scalar_si(c);
  a.sc_ = scalar_sc(c);
  a.X_stride = (long)c->nf * c->Xe;
  a.X_cstride = c->Xe;
  a.n_in = c->N[0];
  a.n_fft = G0;
  a.inner = (int)inner0(c);
  a.g = normal_geo(c);
  a.plan = p0->p;
  a.tw = tw_of<T>(p0);
  a.sc = sc;
  if (c->npot > 1) {
    // 3-D elasticity with a fused kernel for the length: the six components
    // straight from the three potentials
    if (const StaticKernel* sk = bexpand_kernel<T>(c)) {
      a.W = sk->W;
      return launch_col_expand<T>(a, items, sk->lds, c->stream, sk);
    }
    // several potentials: basis map on the trial rows (into X2), then the
    // plain inverse pass with padding into X1
    BasisArgs<T> b{};
    b.c = in;
    b.Xo = w.X2;
    b.c_stride = c->S;
    b.X_stride = a.X_stride;
    b.X_cstride = c->Xe;
    b.N0 = c->N[0];
    b.inner = a.inner;
    b.si = a.si;
    b.sc_ = a.sc_;
    b.g = a.g;
    b.sc = sc;
    const long n = (long)c->N[0] * a.inner;
    const int blocks = (int)std::max(1L, std::min<long>(2048, (n + kThreads - 1) / kThreads));
    if ((e = launch_basis_expand<T>(b, items, blocks, c->stream)) != hipSuccess) return e;
    return plain_axis0<T>(c, items, +1, G0, w.X2, w.X1, sc);
  }
  const StaticKernel* sk = col_static(c, pair ? KK_EXPAND2 : KK_EXPAND, sizeof(cpx<T>), G0, p0->p);
  if (pair && !sk) return hipErrorInvalidValue;
  if (sk) {
    a.W = sk->W;
    return launch_col_expand<T>(a, items, sk->lds, c->stream, sk);
  }
  ColShape sh;
  if ((e = col_shape(p0->p, c->N[0], a.inner, sizeof(cpx<T>), &sh)) != hipSuccess) return e;
  a.W = sh.W;
  return launch_col_expand<T>(a, items, sh.lds, c->stream);
}

// axis-1 pass (3-D): inverse with padding N1 -> G1, or forward with truncation G1 -> N1
template <class T>
static hipError_t stage_axis1(CellImpl* c, Work<T>& w, int items, int sign, int G0, int G1,
                              const cpx<T>* in, cpx<T>* out, ItemScal* sc, bool pair) {
  const DevPlan* p1;
  hipError_t e = get_dev_plan(G1, &p1);
  if (e != hipSuccess) return e;
  (void)w;
  ColPlainArgs<T> a{};
  a.in = in;
  a.out = out;
  a.in_stride = a.out_stride = (long)c->nf * c->Xe;
  a.in_cstride = a.out_cstride = c->Xe;
  a.outer = G0;
  a.n_fft = G1;
  a.n_in = (sign > 0) ? c->N[1] : G1;
  a.n_out = (sign > 0) ? G1 : c->N[1];
  a.inner = c->H;
  a.d = c->nf;
  a.scale = (sign > 0) ? T(1) : T(1.0 / (double)G1);
  a.plan = p1->p;
  a.tw = tw_of<T>(p1);
  a.sc = sc;
  if (pair) {
    // two parts per item: X_0, and the xi_1 / xi_2 pair (k_col_mid2)
    const StaticKernel* sk = find_static(sign > 0 ? KK_MID2_INV : KK_MID2_FWD, sizeof(cpx<T>),
                                         G1, c->N[1], 0, p1->p);
    if (!sk) return hipErrorInvalidValue;
    const NormalGeo g = normal_geo(c);
    a.d = 2;
    a.xi1_step = g.invY[1];
    a.xi2_step = g.invY[2];
    a.W = sk->W;
    return launch_col_plain<T>(a, items, sign, sk->lds, c->stream, sk);
  }
  const StaticKernel* sk = find_static(sign > 0 ? KK_PLAIN_INV : KK_PLAIN_FWD, sizeof(cpx<T>),
                                       G1, c->N[1], 0, p1->p);
  if (sk) {
    a.W = sk->W;
    return launch_col_plain<T>(a, items, sign, sk->lds, c->stream, sk);
  }
  ColShape sh;
  if ((e = col_shape(p1->p, std::max(a.n_in, a.n_out), a.inner, sizeof(cpx<T>), &sh)) !=
      hipSuccess)
    return e;
  a.W = sh.W;
  return launch_col_plain<T>(a, items, sign, sh.lds, c->stream);
}

template <class T>
static hipError_t stage_row(CellImpl* c, int items, int mode, const cpx<T>* in, cpx<T>* out,
                            int G0, int G1, int Glast, const double* ureal, double* oreal,
                            const double* dE, ItemScal* sc, double* partials = nullptr) {
  const DevPlan* pl;
  hipError_t e = get_dev_plan(Glast, &pl);
  if (e != hipSuccess) return e;
  RowArgs<T> a{};
  a.in = in;
  a.out = out;
  a.in_stride = a.out_stride = (long)c->nf * c->Xe;
  a.in_cstride = a.out_cstride = c->Xe;
  const long rows = (c->dd == 3) ? (long)G0 * G1 : G0;
  a.ureal = ureal;
  a.oreal = oreal;
  a.real_cstride = rows * Glast;
  a.real_stride = (long)c->nf * a.real_cstride;
  a.A = (sizeof(T) == 8) ? (const T*)(const void*)c->A64 : (const T*)(const void*)c->A32;
  a.A_stride = c->A_block;
  a.A_group = c->A_group;
  a.A_cstride = c->nQ;
  a.kind = c->kind;
  a.E = dE;
  a.d = c->nf;
  a.rows = (int)rows;
  a.n = Glast;
  a.H = c->H;
  a.plan = pl->p;
  a.tw = tw_of<T>(pl);
  a.sc = sc;
  a.partials = (mode == ROW_APPLY) ? partials : nullptr;
  a.P = partial_slots(c);
  a.pscale = 1.0 / ((double)rows * Glast);
  const int Nlast = c->N[c->dd - 1];
  const int kind = (mode == ROW_APPLY) ? KK_ROW : (mode == ROW_CONST) ? KK_ROW_CONST
                 : (mode == ROW_SYNTH) ? KK_ROW_SYNTH : -1;
  const StaticKernel* sk =
      (kind >= 0) ? find_static(kind, sizeof(cpx<T>), Glast, Nlast, c->nf, pl->p) : nullptr;
  if (sk) {
    a.RP = sk->W;
    return launch_row<T>(a, items, mode, sk->lds, c->stream, sk);
  }
  // The generic FP64 last-axis kernel with a chirp-z (Bluestein) plan faulted
  // the GPU once in its flux / right-hand-side / synthesis modes (255 rows of
  // length 127, 4 row pairs per workgroup) and the cause is not known: those
  // modes are not run.  Lengths with a specialised FP64 kernel are served by
  // it; other such shapes are rejected when the cell is created.
  if (sizeof(T) == 8 && pl->p.blue && mode != ROW_FWD) return hipErrorNotSupported;
  size_t lds = 0;
  int RP = 0;
  if ((e = row_shape(pl->p, c->nf, rows, sizeof(cpx<T>), &RP, &lds)) != hipSuccess) return e;
  a.RP = RP;
  return launch_row<T>(a, items, mode, lds, c->stream);
}

template <class T>
static hipError_t stage_project(CellImpl* c, Work<T>& w, int items, const cpx<T>* X, int G0,
                                int epi, cpx<T>* out, const cpx<T>* pdot, cpx<T>* r, cpx<T>* pp,
                                cpx<T>* x, const cpx<T>* b, double* partials, ItemScal* sc,
                                int* tiles, bool pair, const CgFuse* cg = nullptr) {
  const DevPlan* p0;
  hipError_t e = get_dev_plan(G0, &p0);
  if (e != hipSuccess) return e;
  (void)w;
  ColProjectArgs<T> a{};
  a.X = X;
  a.X_stride = (long)c->nf * c->Xe;
  a.X_cstride = c->Xe;
  a.q = out;
  a.s_stride = c->S;
  a.si = scalar_si(c);
  a.sc_ = scalar_sc(c);
  a.p = pdot;
  a.r = r;
  a.pp = pp;
  a.x = x;
  a.b = b;
  a.partials = partials;
  a.P = partial_slots(c);
  a.n_fft = G0;
  a.n_out = c->N[0];
  a.inner = (int)inner0(c);
  a.epi = epi;
  a.d = c->nf;
  if (cg) {
    a.rr_part = cg->rr;
    a.rr_n = cg->rr_n;
    a.pq_part = cg->pq;
    a.pq_n = cg->pq_n;
  }
  a.scale = T(1.0 / (double)G0);
  a.g = normal_geo(c);
  a.plan = p0->p;
  a.tw = tw_of<T>(p0);
  a.sc = sc;
  if (c->npot > 1) {
    // several potentials: plain forward pass with truncation into the other
    // component buffer, then the basis map with the projection's epilogue
    cpx<T>* tmp = (X == w.X1) ? w.X2 : w.X1;
    if ((e = plain_axis0<T>(c, items, -1, G0, X, tmp, sc)) != hipSuccess) return e;
    BasisArgs<T> ba{};
    ba.Xi = tmp;
    ba.c_stride = c->S;
    ba.X_stride = a.X_stride;
    ba.X_cstride = c->Xe;
    ba.N0 = c->N[0];
    ba.inner = a.inner;
    ba.si = a.si;
    ba.sc_ = a.sc_;
    ba.q = out;
    ba.p = pdot;
    ba.r = r;
    ba.pp = pp;
    ba.x = x;
    ba.b = b;
    ba.partials = partials;
    ba.P = a.P;
    ba.epi = epi;
    ba.rr_part = a.rr_part;
    ba.rr_n = a.rr_n;
    ba.pq_part = a.pq_part;
    ba.pq_n = a.pq_n;
    ba.g = a.g;
    ba.sc = sc;
    const int blocks = basis_blocks(c);
    if (tiles) *tiles = blocks;
    return launch_basis_project<T>(ba, items, blocks, c->stream);
  }
  const StaticKernel* sk = col_static(c, pair ? KK_PROJECT2 : KK_PROJECT, sizeof(cpx<T>), G0,
                                      p0->p);
  if (pair && !sk) return hipErrorInvalidValue;
  if (sk) {
    a.W = sk->W;
    if (tiles) *tiles = (a.inner + sk->W - 1) / sk->W;
    return launch_col_project<T>(a, items, sk->lds, c->stream, sk);
  }
  ColShape sh;
  if ((e = col_shape(p0->p, c->N[0], a.inner, sizeof(cpx<T>), &sh)) != hipSuccess) return e;
  a.W = sh.W;
  if (tiles) *tiles = (a.inner + sh.W - 1) / sh.W;
  return launch_col_project<T>(a, items, sh.lds, c->stream);
}

template <class T>
int project_tiles(CellImpl* c) {
  const DevPlan* p0;
  if (get_dev_plan(c->Q[0], &p0) != hipSuccess) return 0;
  const int inner = (int)inner0(c);
  if (c->npot > 1) return basis_blocks(c);
  const StaticKernel* sk = col_static(c, pair_mode<T>(c) ? KK_PROJECT2 : KK_PROJECT,
                                      sizeof(cpx<T>), c->Q[0], p0->p);
  if (sk) return (inner + sk->W - 1) / sk->W;
  ColShape sh;
  if (col_shape(p0->p, c->N[0], inner, sizeof(cpx<T>), &sh) != hipSuccess) return 0;
  return (inner + sh.W - 1) / sh.W;
}

// workgroups per item of the last-axis flux pass (its partial sums)
template <class T>
int row_tiles(CellImpl* c) {
  const int Glast = c->Q[c->dd - 1];
  const DevPlan* pl;
  if (get_dev_plan(Glast, &pl) != hipSuccess) return 0;
  const long rows = (c->dd == 3) ? (long)c->Q[0] * c->Q[1] : c->Q[0];
  const long pairs = (rows + 1) / 2;
  const StaticKernel* sk =
      find_static(KK_ROW, sizeof(cpx<T>), Glast, c->N[c->dd - 1], c->nf, pl->p);
  int RP = sk ? sk->W : 0;
  size_t lds = 0;
  if (!sk && row_shape(pl->p, c->nf, rows, sizeof(cpx<T>), &RP, &lds) != hipSuccess) return 0;
  return (int)((pairs + RP - 1) / RP);
}

// q = Op(in) on the quadrature grid
template <class T>
hipError_t pipe_apply(CellImpl* c, Work<T>& w, int items, const cpx<T>* in, int epi,
                      cpx<T>* out, const cpx<T>* pdot, const cpx<T>* b, ItemScal* sc,
                      double* partials, const CgFuse* cg) {
  hipError_t e;
  const int Q0 = c->Q[0], Q1 = c->Q[1], Q2 = c->Q[2];
  // (in, q) with q = Op(in): the last-axis pass sums e . (A e) over the real
  // points (Parseval), so the projection reads no second spectrum for it
  const bool rowdot = (epi == EPI_STORE && pdot == in && partials != nullptr);
  double* rpart = rowdot ? partials : nullptr;
  const bool pair = pair_mode<T>(c);
  if ((e = stage_expand<T>(c, w, items, in, Q0, sc, pair)) != hipSuccess) return e;
  if (c->dd == 3) {
    if ((e = stage_axis1<T>(c, w, items, +1, Q0, Q1, w.X1, w.X2, sc, pair)) != hipSuccess)
      return e;
    if ((e = stage_row<T>(c, items, ROW_APPLY, w.X2, w.X2, Q0, Q1, Q2, nullptr, nullptr, nullptr,
                          sc, rpart)) != hipSuccess)
      return e;
    if ((e = stage_axis1<T>(c, w, items, -1, Q0, Q1, w.X2, w.X1, sc, pair)) != hipSuccess)
      return e;
  } else {
    if ((e = stage_row<T>(c, items, ROW_APPLY, w.X1, w.X1, Q0, 1, Q1, nullptr, nullptr, nullptr,
                          sc, rpart)) != hipSuccess)
      return e;
  }
  cpx<T>* rr = (epi == EPI_RESID) ? out : nullptr;
  return stage_project<T>(c, w, items, w.X1, Q0, epi, out, rowdot ? nullptr : pdot, rr, nullptr,
                          nullptr, b, rowdot ? nullptr : partials, sc, nullptr, pair, cg);
}

template <class T>
hipError_t pipe_rhs(CellImpl* c, Work<T>& w, int items, const double* dE, ItemScal* sc) {
  hipError_t e;
  const int Q0 = c->Q[0], Q1 = c->Q[1], Q2 = c->Q[2];
  if (c->dd == 3) {
    if ((e = stage_row<T>(c, items, ROW_CONST, nullptr, w.X2, Q0, Q1, Q2, nullptr, nullptr, dE,
                          sc)) != hipSuccess)
      return e;
    if ((e = stage_axis1<T>(c, w, items, -1, Q0, Q1, w.X2, w.X1, sc, pair_mode<T>(c))) !=
        hipSuccess)
      return e;
  } else {
    if ((e = stage_row<T>(c, items, ROW_CONST, nullptr, w.X1, Q0, 1, Q1, nullptr, nullptr, dE,
                          sc)) != hipSuccess)
      return e;
  }
  if ((e = stage_project<T>(c, w, items, w.X1, Q0, EPI_RHS, w.b, nullptr, w.r, w.p, w.x, nullptr,
                            w.part, sc, nullptr, pair_mode<T>(c))) != hipSuccess)
    return e;
  // b (and r = p = b) given the exact symmetry of the potential of a real
  // field on the h = 0 plane; (b, b) again, in the first project_tiles
  // partial slots, where the callers sum it
  SymArgs<T> sa{};
  sa.v[0] = w.b;
  sa.v[1] = w.r;
  sa.v[2] = w.p;
  sa.stride = c->S;
  sa.npot = c->npot;
  sa.even_pot = (c->dual && c->dd == 3) ? 1 : -1;   // t_2 of the 3-D dual
  sa.pot_stride = c->S / c->npot;
  sa.N0 = c->N[0];
  sa.N1 = (c->dd == 3) ? c->N[1] : 1;
  sa.s0 = scalar_si(c);
  sa.s1 = (c->dd == 3) ? c->H : 0;
  sa.sc = sc;
  if ((e = launch_sym_h0<T>(sa, items, c->stream)) != hipSuccess) return e;
  return launch_norm_parts<T>(w.b, c->S, c->S, scalar_n0(c), c->H, w.part, partial_slots(c),
                              project_tiles<T>(c), items, sc, c->stream);
}

hipError_t pipe_synth(CellImpl* c, Work<double>& w, int items, const cpx<double>* cin,
                      const double* dE, bool onQ, double* out) {
  hipError_t e;
  const int G0 = onQ ? c->Q[0] : c->N[0];
  const int G1 = onQ ? c->Q[1] : c->N[1];
  const int G2 = onQ ? c->Q[2] : c->N[2];
  const bool pair = c->dd == 3 && pair_on<double>(c, G0, G1);
  if ((e = stage_expand<double>(c, w, items, cin, G0, nullptr, pair)) != hipSuccess) return e;
  if (c->dd == 3) {
    if ((e = stage_axis1<double>(c, w, items, +1, G0, G1, w.X1, w.X2, nullptr, pair)) !=
        hipSuccess)
      return e;
    return stage_row<double>(c, items, ROW_SYNTH, w.X2, nullptr, G0, G1, G2, nullptr, out, dE,
                             nullptr);
  }
  return stage_row<double>(c, items, ROW_SYNTH, w.X1, nullptr, G0, 1, G1, nullptr, out, dE,
                           nullptr);
}

hipError_t pipe_project_real(CellImpl* c, Work<double>& w, int items, const double* u,
                             cpx<double>* cout) {
  hipError_t e;
  const int N0 = c->N[0], N1 = c->N[1], N2 = c->N[2];
  cpx<double>* X = w.X1;
  if (c->dd == 3) {
    if ((e = stage_row<double>(c, items, ROW_FWD, nullptr, w.X2, N0, N1, N2, u, nullptr, nullptr,
                               nullptr)) != hipSuccess)
      return e;
    // forward along axis 1 without truncation (N1 -> N1)
    const DevPlan* p1;
    if ((e = get_dev_plan(N1, &p1)) != hipSuccess) return e;
    ColPlainArgs<double> a{};
    a.in = w.X2;
    a.out = w.X1;
    a.in_stride = a.out_stride = (long)c->nf * c->Xe;
    a.in_cstride = a.out_cstride = c->Xe;
    a.outer = N0;
    a.n_in = a.n_fft = a.n_out = N1;
    a.inner = c->H;
    a.d = c->nf;
    a.scale = 1.0 / (double)N1;
    a.plan = p1->p;
    a.tw = p1->tw64;
    const StaticKernel* sk = find_static(KK_PLAIN_FWD, sizeof(cpx<double>), N1, N1, 0, p1->p);
    if (sk) {
      a.W = sk->W;
      e = launch_col_plain<double>(a, items, -1, sk->lds, c->stream, sk);
    } else {
      ColShape sh;
      if ((e = col_shape(p1->p, N1, a.inner, sizeof(cpx<double>), &sh)) != hipSuccess) return e;
      a.W = sh.W;
      e = launch_col_plain<double>(a, items, -1, sh.lds, c->stream);
    }
    if (e != hipSuccess) return e;
  } else {
    if ((e = stage_row<double>(c, items, ROW_FWD, nullptr, w.X1, N0, 1, N1, u, nullptr, nullptr,
                               nullptr)) != hipSuccess)
      return e;
  }
  // the axis-1 forward above leaves three spectra
  return stage_project<double>(c, w, items, X, N0, EPI_STORE, cout, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr, nullptr, nullptr, false);
}

template hipError_t pipe_apply<float>(CellImpl*, Work<float>&, int, const cpx<float>*, int,
                                      cpx<float>*, const cpx<float>*, const cpx<float>*, ItemScal*,
                                      double*, const CgFuse*);
template hipError_t pipe_apply<double>(CellImpl*, Work<double>&, int, const cpx<double>*, int,
                                       cpx<double>*, const cpx<double>*, const cpx<double>*,
                                       ItemScal*, double*, const CgFuse*);
template hipError_t pipe_rhs<float>(CellImpl*, Work<float>&, int, const double*, ItemScal*);
template int project_tiles<float>(CellImpl*);
template int project_tiles<double>(CellImpl*);
template hipError_t pipe_rhs<double>(CellImpl*, Work<double>&, int, const double*, ItemScal*);

// ---------------------------------------------------------------------------
// CG iterations, captured K at a time into a HIP graph
// ---------------------------------------------------------------------------
template <class T>
static CgUpdateArgs<T> update_args(CellImpl* c, Work<T>& w, int tiles, bool xupd,
                                   bool pq_sc = false) {
  CgUpdateArgs<T> u{};
  u.xupd = xupd ? 1 : 0;
  u.x = w.x;
  u.r = w.r;
  u.p = w.p;
  u.q = w.q;
  u.stride = c->S;
  u.count = c->S;
  u.H = c->H;
  u.n0 = scalar_n0(c);
  u.partials = w.part2;
  u.P = partial_slots(c);
  u.sc = w.sc;
  u.pq_part = w.part;
  u.pq_n = tiles;
  u.pq_sc = pq_sc ? 1 : 0;
  return u;
}

template <class T>
static CgDirArgs<T> direction_args(CellImpl* c, Work<T>& w, int ub, bool xdef) {
  CgDirArgs<T> a{};
  a.x = w.x;
  a.r = w.r;
  a.p = w.p;
  a.stride = c->S;
  a.count = c->S;
  a.sc = w.sc;
  a.rr_part = w.part2;
  a.rr_n = ub;
  a.P = partial_slots(c);
  a.xdef = xdef ? 1 : 0;
  return a;
}

template <class T>
static hipError_t cg_body(CellImpl* c, Work<T>& w, int items, int K, bool finalize = true) {
  // one iteration: direction step (beta and stopping test from the last
  // update's (r, r) partials, x += alpha p left by that update, p <- r + beta
  // p), the operator's passes on p (the last-axis pass leaves the (p, q)
  // partials), projection (q, bookkeeping of the last update), update (alpha
  // from the (p, q) partials,
  // r, (r, r) partials; x only in the last iteration, which leaves x current
  // at the end of the graph); after K iterations the last update is booked so
  // the host reads current scalars
  hipError_t e = hipSuccess;
  const int P = partial_slots(c);
  // the (p, q) partials come from the last-axis pass; the projection's first
  // workgroup sums them for the update
  const int rtiles = row_tiles<T>(c);
  const int ub = update_blocks(c->S);
  for (int k = 0; k < K && e == hipSuccess; ++k) {
    const CgFuse cg{w.part2, ub, k > 0 ? 1 : 0, w.part, rtiles};
    e = launch_cg_direction<T>(direction_args<T>(c, w, ub, k > 0), items, ub, c->stream);
    if (e == hipSuccess)
      e = pipe_apply<T>(c, w, items, w.p, EPI_STORE, w.q, w.p, nullptr, w.sc, w.part, &cg);
    if (e == hipSuccess)
      e = launch_cg_update<T>(update_args<T>(c, w, rtiles, k == K - 1, true), items, ub,
                              c->stream);
  }
  if (e == hipSuccess && finalize) e = launch_cg_finalize(w.sc, w.part2, P, ub, items, c->stream);
  return e;
}

// one Moulinec-Suquet iteration per step (FP64): r = b - Op x with the
// partials of (r, r), the booking (stop at ||r|| <= tol ||b||), x += r / lambda
static hipError_t ms_body(CellImpl* c, Work<double>& w, int items, int K) {
  hipError_t e = hipSuccess;
  const int P = partial_slots(c);
  const int tiles = project_tiles<double>(c);
  const int ub = update_blocks(c->S);
  for (int k = 0; k < K && e == hipSuccess; ++k) {
    e = pipe_apply<double>(c, w, items, w.x, EPI_RESID, w.r, nullptr, w.b, w.sc, w.part);
    if (e == hipSuccess) e = launch_ms_book(w.sc, w.part, P, tiles, items, c->stream);
    if (e == hipSuccess) e = launch_ms_axpy(w.x, w.r, c->S, c->S, w.sc, ub, items, c->stream);
  }
  return e;
}

template <class T>
hipError_t cg_graph(CellImpl* c, int items, int K, hipGraphExec_t* out, int solver) {
  GraphKey key{(int)sizeof(T), items, K, tune_version(), solver};
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) {
    *out = it->second;
    return hipSuccess;
  }
  // graphs captured with other kernel choices are never replayed again (the
  // stream is drained first: one of them may still be running)
  bool stale = false;
  for (const auto& g : c->graphs) stale = stale || g.first.version != key.version;
  if (stale) {
    hipError_t es = hipStreamSynchronize(c->stream);
    if (es != hipSuccess) return es;
  }
  for (auto g = c->graphs.begin(); g != c->graphs.end();) {
    if (g->first.version != key.version) {
      (void)hipGraphExecDestroy(g->second);
      g = c->graphs.erase(g);
    } else {
      ++g;
    }
  }
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t eb = (solver == 1) ? ms_body(c, c->w64, items, K)
                                 : cg_body<T>(c, work_of<T>(c), items, K);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->stream, &g);
  if (eb != hipSuccess) e = eb;
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return e;
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return e;
  c->graphs[key] = ex;
  *out = ex;
  return hipSuccess;
}

template hipError_t cg_graph<float>(CellImpl*, int, int, hipGraphExec_t*, int);
template hipError_t cg_graph<double>(CellImpl*, int, int, hipGraphExec_t*, int);

// Launch planner.  A captured graph runs K iterations; an item that stops
// inside it leaves the rest as launches that do nothing but still cost their
// dispatch, and every host check costs a round trip.  After each launch the
// host reads every item's residual ratio, estimates its convergence rate per
// iteration from the previous reading and launches the number of iterations
// (at most Kmax) predicted to bring the nearest item to its stopping test.
struct IterPlanner {
  int Kmax = 16;
  std::vector<double> prev_rho, rate;
  std::vector<int> prev_it;
  explicit IterPlanner(int items, int kmax) : Kmax(std::max(1, kmax)) {
    prev_rho.assign(items, -1.0);
    rate.assign(items, -1.0);
    prev_it.assign(items, 0);
  }
  // forget the reading of item i (its residual was replaced); its rate stays
  void reset(int i) { prev_rho[i] = -1.0; }
  int next(const std::vector<ItemScal>& hs, const std::vector<char>& live) {
    double need = 1e300;
    for (size_t i = 0; i < hs.size(); ++i) {
      if (!live[i] || !hs[i].active) continue;
      const ItemScal& q = hs[i];
      if (prev_rho[i] > 0.0 && q.iters > prev_it[i] && q.rho > 0.0 && q.rho < prev_rho[i])
        rate[i] = std::pow(q.rho / prev_rho[i], 1.0 / (q.iters - prev_it[i]));
      prev_rho[i] = q.rho;
      prev_it[i] = q.iters;
      if (!(rate[i] > 0.0 && rate[i] < 1.0) || !(q.rho > 0.0) || !(q.rho0 > 0.0)) {
        need = std::min(need, (double)Kmax);
        continue;
      }
      const double target = q.tol * q.tol * q.rho0;   // rho at which the item is done
      const double it = (q.rho <= target) ? 1.0 : std::log(target / q.rho) / std::log(rate[i]);
      need = std::min(need, std::max(1.0, std::ceil(it)));
    }
    return (need >= (double)Kmax) ? Kmax : (int)need;
  }
};

// K iterations as back-to-back launches of graphs of power-of-two lengths
template <class T>
static hipError_t cg_launch(CellImpl* c, int items, int K, int solver = 0) {
  hipError_t e = hipSuccess;
  for (int b = 1 << 30; b > 0 && e == hipSuccess; b >>= 1) {
    if (!(K & b)) continue;
    hipGraphExec_t g = nullptr;
    e = cg_graph<T>(c, items, b, &g, solver);
    if (e == hipSuccess) e = hipGraphLaunch(g, c->stream);
  }
  return e;
}

// scalar read-back through the cell's pinned staging (a DMA, no bounce)
static hipError_t read_scal(CellImpl* c, const ItemScal* d, int items, std::vector<ItemScal>& h) {
  h.resize(items);
  void* hp = nullptr;
  hipError_t e = pinned(c, sizeof(ItemScal) * items, &hp);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hp, d, sizeof(ItemScal) * items, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) std::memcpy(h.data(), hp, sizeof(ItemScal) * items);
  return e;
}

static hipError_t read_scal2(CellImpl* c, const ItemScal* d1, std::vector<ItemScal>& h1,
                             const ItemScal* d2, std::vector<ItemScal>& h2, int items) {
  h1.resize(items);
  h2.resize(items);
  const size_t b = sizeof(ItemScal) * items;
  void* hp = nullptr;
  hipError_t e = pinned(c, 2 * b, &hp);
  if (e == hipSuccess) e = hipMemcpyAsync(hp, d1, b, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync((char*)hp + b, d2, b, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) {
    std::memcpy(h1.data(), hp, b);
    std::memcpy(h2.data(), (char*)hp + b, b);
  }
  return e;
}

// host -> device through the pinned staging.  With wait == false the copy
// is only queued: the caller's next host access to the staging must follow a
// stream synchronisation (the read-backs synchronise before they touch it).
static hipError_t upload(CellImpl* c, void* dst, const void* src, size_t bytes, bool wait = true) {
  void* hp = nullptr;
  hipError_t e = pinned(c, bytes, &hp);
  if (e != hipSuccess) return e;
  std::memcpy(hp, src, bytes);
  e = hipMemcpyAsync(dst, hp, bytes, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && wait) e = hipStreamSynchronize(c->stream);
  return e;
}

// run CG (solver 0) or the Moulinec-Suquet iteration (solver 1) until every
// item is inactive
template <class T>
static hipError_t cg_run(CellImpl* c, int items, int max_iter, std::vector<ItemScal>& hs,
                         int solver = 0) {
  Work<T>& w = work_of<T>(c);
  IterPlanner plan(items, c->opt.check_every);
  std::vector<char> live(items, 1);
  hipError_t e = read_scal(c, w.sc, items, hs);
  if (e != hipSuccess) return e;
  int K = plan.next(hs, live);   // the first reading: no rate yet, Kmax
  long launched = 0;
  for (;;) {
    bool any = false;
    for (auto& s : hs) any = any || s.active;
    if (!any) break;
    if (launched > (long)max_iter + plan.Kmax) break;  // the device also stops at max_iter
    if ((e = cg_launch<T>(c, items, K, solver)) != hipSuccess) return e;
    launched += K;
    if ((e = read_scal(c, w.sc, items, hs)) != hipSuccess) return e;
    K = plan.next(hs, live);
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
// components of a load case, a strain field or a mean flux as the caller
// sees them: d, or the d(d+1)/2 Mandel components of an elastic cell
static int user_comps(const CellImpl* c) { return c->elastic ? c->nf : c->d; }

// the load cases on the device, in the cell's persistent buffer
static hipError_t upload_E(CellImpl* c, int L, const double* E, double** dE) {
  // [L][nf] with zero padding for d = 1 (E holds L x user_comps(c) values)
  const int nu = user_comps(c);
  std::vector<double> h((size_t)L * c->nf, 0.0);
  for (int l = 0; l < L; ++l)
    for (int a = 0; a < nu; ++a) h[(size_t)l * c->nf + a] = E[(size_t)l * nu + a];
  if (c->dE_items < L) {
    if (c->dE) (void)hipFree(c->dE);
    c->dE = nullptr;
    c->dE_items = 0;
    hipError_t e = hipMalloc(&c->dE, sizeof(double) * 6 * std::max(L, 8));
    if (e != hipSuccess) return e;
    c->dE_items = std::max(L, 8);
  }
  *dE = c->dE;
  return upload(c, c->dE, h.data(), sizeof(double) * h.size());
}

static hipError_t sum_partials_host(CellImpl* c, const double* dpart, int items, int nparts,
                                    std::vector<double>& out) {
  const int P = partial_slots(c);
  std::vector<double> h((size_t)items * P);
  void* hp = nullptr;
  hipError_t e = pinned(c, sizeof(double) * h.size(), &hp);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hp, dpart, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  std::memcpy(h.data(), hp, sizeof(double) * h.size());
  out.assign(items, 0.0);
  for (int i = 0; i < items; ++i)
    for (int t = 0; t < nparts; ++t) out[i] += h[(size_t)i * P + t];
  return hipSuccess;
}

static hipError_t ensure_ebuf(CellImpl* c, int items) {
  if (c->ebuf_items >= items) return hipSuccess;
  if (c->ebuf) (void)hipFree(c->ebuf);
  c->ebuf = nullptr;
  c->ebuf_items = 0;
  hipError_t e = hipMalloc(&c->ebuf, sizeof(double) * (size_t)items * c->nf * c->nQ);
  if (e == hipSuccess) c->ebuf_items = items;
  return e;
}

// W [L][L], J [L][d] from the FP64 potentials x of L items
static hipError_t homogenize(CellImpl* c, int L, const double* dE, double* strain_user,
                             double* W, double* J) {
  hipError_t e;
  const cpx<double>* x = c->w64.x;
  double* eQ = nullptr;
  const bool gani = (c->scheme == HOM_GANI);
  if (gani && strain_user && c->d == c->dd) {
    eQ = strain_user;
  } else {
    if ((e = ensure_ebuf(c, L)) != hipSuccess) return e;
    eQ = c->ebuf;
  }
  if ((e = pipe_synth(c, c->w64, L, x, dE, true, eQ)) != hipSuccess) return e;
  if (!c->quad) {
    if ((e = hipMalloc(&c->quad, sizeof(double) * kQuadScratch)) != hipSuccess) return e;
  }
  const int blocks = (int)std::min<long>(kQuadBlocks, (c->nQ + kThreads - 1) / kThreads);
  std::vector<double> hW((size_t)L * L, 0.0), hJ((size_t)L * c->nf, 0.0);
  for (int l0 = 0; l0 < L; l0 += 3) {
    const int nl = std::min(3, L - l0);
    for (int m0 = 0; m0 < L; m0 += 3) {
      const int nm = std::min(3, L - m0);
      if ((e = launch_quad(eQ, (long)c->nf * c->nQ, c->nQ, c->A64, c->nQ, c->kind, c->nf, c->nQ,
                           l0, nl, m0, nm, c->quad, blocks, c->stream)) != hipSuccess)
        return e;
      double* outp = c->quad + (size_t)kQuadBlocks * kQuadSlots;
      if ((e = launch_quad_final(c->quad, blocks, nl, nm, c->nf, c->nQ, outp, c->stream)) !=
          hipSuccess)
        return e;
      double h[kQuadSlots];
      void* hp = nullptr;
      if ((e = pinned(c, sizeof(h), &hp)) != hipSuccess) return e;
      if ((e = hipMemcpyAsync(hp, outp, sizeof(h), hipMemcpyDeviceToHost, c->stream)) !=
          hipSuccess)
        return e;
      if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
      std::memcpy(h, hp, sizeof(h));
      for (int l = 0; l < nl; ++l)
        for (int m = 0; m < nm; ++m) hW[(size_t)(l0 + l) * L + m0 + m] = h[l * 3 + m];
      if (l0 == 0)
        for (int m = 0; m < nm; ++m)
          for (int a = 0; a < c->nf; ++a) hJ[(size_t)(m0 + m) * c->nf + a] = h[9 + m * c->nf + a];
    }
  }
  if (W) std::memcpy(W, hW.data(), sizeof(double) * hW.size());
  if (J)
    for (int l = 0; l < L; ++l)
      for (int a = 0; a < user_comps(c); ++a)
        J[(size_t)l * user_comps(c) + a] = hJ[(size_t)l * c->nf + a];
  if (strain_user && eQ != strain_user) {
    if (gani && c->d == c->dd) {
      // unreachable: handled above
    } else if (c->d == c->dd) {
      if ((e = pipe_synth(c, c->w64, L, x, dE, false, strain_user)) != hipSuccess) return e;
    } else {
      // d = 1 run as 2-D with one point along axis 1: copy component 0 of each item
      if (!gani) {
        if ((e = pipe_synth(c, c->w64, L, x, dE, false, c->ebuf)) != hipSuccess) return e;
      }
      for (int l = 0; l < L; ++l) {
        const double* src = c->ebuf + (size_t)l * c->nf * (gani ? c->nQ : c->nN);
        if ((e = hipMemcpyAsync(strain_user + (size_t)l * c->nN, src, sizeof(double) * c->nN,
                                hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
          return e;
      }
    }
  }
  return hipSuccess;
}

static hipError_t warm_start(CellImpl* c, int L, const double* strain0, double* partials) {
  // x0 = n . F_N[strain0] (its E_N part); r = b - Op x0 with partials of
  // (r, r) in `partials`; p = r
  Work<double>& w = c->w64;
  hipError_t e = pipe_project_real(c, w, L, strain0, w.x);
  if (e != hipSuccess) return e;
  if ((e = pipe_apply<double>(c, w, L, w.x, EPI_RESID, w.r, nullptr, w.b, nullptr,
                              partials)) != hipSuccess)
    return e;
  return hipMemcpyAsync(w.p, w.r, sizeof(cpx<double>) * (size_t)c->S * L,
                        hipMemcpyDeviceToDevice, c->stream);
}


// ---------------------------------------------------------------------------
// engine pool: device buffers, stream and captured graphs of destroyed cells
// are kept (a few per process) and handed to new cells of the same shape, so
// that creating such a cell costs only the upload of its coefficient field
// ---------------------------------------------------------------------------
static std::mutex g_pool_mu;
static std::vector<CellImpl*> g_pool;
static const size_t kPoolMax = 4;

static bool same_shape(const CellImpl* a, const CellImpl& b) {
  if (a->dd != b.dd || a->scheme != b.scheme || a->kind != b.kind || a->nA != b.nA ||
      a->dual != b.dual)
    return false;
  for (int i = 0; i < 3; ++i)
    if (a->N[i] != b.N[i] || a->Q[i] != b.Q[i] || a->Y[i] != b.Y[i]) return false;
  return true;
}

CellImpl* pool_take(int device, const CellImpl& key) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (size_t i = g_pool.size(); i-- > 0;) {
    CellImpl* c = g_pool[i];
    if (c->device == device && same_shape(c, key)) {
      g_pool.erase(g_pool.begin() + (long)i);
      return c;
    }
  }
  return nullptr;
}

void pool_put(CellImpl* c) {
  CellImpl* evict = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pool.push_back(c);
    if (g_pool.size() > kPoolMax) {
      evict = g_pool.front();
      g_pool.erase(g_pool.begin());
    }
  }
  if (evict) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(evict->device);
    delete evict;
    (void)hipSetDevice(cur);
  }
}

}  // namespace hom

using namespace hom;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* hom_status_str(hom_status s) {
  switch (s) {
    case HOM_OK: return "ok";
    case HOM_EINVAL: return "invalid argument";
    case HOM_ENOTSPD: return "coefficient not symmetric positive definite";
    case HOM_ENOMEM: return "out of memory";
    case HOM_ENOTCONV: return "not converged";
    case HOM_EBREAKDOWN: return "CG breakdown";
    case HOM_EDEVICE: return "device error";
    case HOM_EBUSY: return "busy";
    case HOM_ESCRATCH: return "workspace exceeds the allocation-free scratch";
  }
  return "unknown status";
}

hom_status hom_options_default(hom_options* o) {
  if (!o) return HOM_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->scheme = HOM_GANI;
  o->prec = HOM_FP64;
  o->Y[0] = o->Y[1] = o->Y[2] = 0.5;
  o->max_iter = 10000;
  o->max_outer = 100;
  o->inner_tol = 1e-3;
  o->check_every = 16;
  o->stream = nullptr;
  o->a_trig = 0;
  o->dual = 0;
  return HOM_OK;
}

static hom_status dev_status(hipError_t e) {
  if (e == hipSuccess) return HOM_OK;
  if (e == hipErrorOutOfMemory) return HOM_ENOMEM;
  if (e == hipErrorNotSupported) return HOM_EINVAL;   // a shape no kernel serves
  return HOM_EDEVICE;
}

// eigenvalue range of the coefficient at one point; false if not SPD or not finite

// false if a last-axis pass of the cell would need the generic FP64 kernel
// with a chirp-z plan, which stage_row refuses: the flux, right-hand-side
// and synthesis passes on the quadrature grid, and (Ga) the synthesis of the
// strain on the trial grid
static bool fp64_rows_served(const CellImpl* c) {
  const int Nl = c->N[c->dd - 1];
  const int lens[2] = {c->Q[c->dd - 1], Nl};
  for (int i = 0; i < 2; ++i) {
    const DevPlan* pl = nullptr;
    if (get_dev_plan(lens[i], &pl) != hipSuccess) return false;
    if (!pl->p.blue) continue;
    for (int k : {KK_ROW, KK_ROW_CONST, KK_ROW_SYNTH}) {
      if (i == 1 && k != KK_ROW_SYNTH) continue;
      if (!find_static(k, (int)sizeof(cpx<double>), lens[i], Nl, c->nf, pl->p)) return false;
    }
  }
  return true;
}

// order the cell stream after work already queued on the caller's stream
static void wait_user_stream(CellImpl* c) {
  if (!c->opt.stream) return;
  hipEvent_t ev;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return;
  (void)hipEventRecord(ev, (hipStream_t)c->opt.stream);
  (void)hipStreamWaitEvent(c->stream, ev, 0);
  (void)hipEventDestroy(ev);
}

hom_status hom_create_cell(int d, const int32_t* N, hom_a_kind kind, const double* A,
                           int A_on_device, const hom_options* opt, hom_cell** out) {
  if (!out || !N || !A || d < 1 || d > 3) return HOM_EINVAL;
  if (kind < HOM_A_ISO || kind > HOM_A_ELASTIC) return HOM_EINVAL;
  *out = nullptr;
  hom_options o;
  if (opt)
    o = *opt;
  else
    hom_options_default(&o);
  if (o.scheme != HOM_GANI && o.scheme != HOM_GA) return HOM_EINVAL;
  if (o.prec != HOM_FP64 && o.prec != HOM_MIXED) return HOM_EINVAL;
  if (o.max_iter < 0 || o.check_every < 1 || o.max_outer < 1) return HOM_EINVAL;
  if (!(o.inner_tol > 0 && o.inner_tol < 1)) return HOM_EINVAL;
  if (o.a_trig != 0 && (o.a_trig != 1 || o.scheme != HOM_GA)) return HOM_EINVAL;
  if (o.dual != 0 && (o.dual != 1 || d < 2)) return HOM_EINVAL;
  // linear elasticity: d = 2 (plane strain) or 3, primal problem, sampled
  // Lame fields
  if (kind == HOM_A_ELASTIC && (d < 2 || o.dual || o.a_trig)) return HOM_EINVAL;
  for (int a = 0; a < d; ++a) {
    if (N[a] < 1 || (N[a] % 2) == 0 || N[a] > (1 << 20)) return HOM_EINVAL;
    if (!(o.Y[a] > 0) || !std::isfinite(o.Y[a])) return HOM_EINVAL;
  }
  // everything shape-related first; the device engine may come from the pool
  CellImpl key;
  key.d = d;
  key.dd = d < 2 ? 2 : d;
  key.scheme = o.scheme;
  key.dual = o.dual;
  const int nA_user = (kind == HOM_A_ISO) ? 1 : (kind == HOM_A_DIAG) ? d
                    : (kind == HOM_A_ELASTIC) ? 2 : d * (d + 1) / 2;
  // d = 1 runs as a 2-D cell with a single grid point along the second axis;
  // its one coefficient acts as an isotropic one (e_2 vanishes identically)
  key.kind = (d == 1) ? HOM_A_ISO : kind;
  key.nA = (d == 1) ? 1 : nA_user;
  for (int a = 0; a < key.dd; ++a) {
    key.N[a] = (a < d) ? N[a] : 1;
    key.Q[a] = (o.scheme == HOM_GA) ? 2 * key.N[a] - 1 : key.N[a];
    key.Y[a] = (a < d) ? o.Y[a] : 0.5;
  }
  long nQ = 1;
  for (int a = 0; a < key.dd; ++a) nQ *= key.Q[a];
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return dev_status(e);
  CellImpl* c = pool_take(device, key);
  if (!c) {
    c = new (std::nothrow) CellImpl();
    if (!c) return HOM_ENOMEM;
    c->device = device;
    c->d = key.d;
    c->dd = key.dd;
    c->scheme = key.scheme;
    c->dual = key.dual;
    c->kind = key.kind;
    c->nA = key.nA;
    for (int a = 0; a < 3; ++a) {
      c->N[a] = key.N[a];
      c->Q[a] = key.Q[a];
      c->Y[a] = key.Y[a];
    }
    const size_t nAd = (size_t)c->nA * nQ;
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&c->A64, sizeof(double) * nAd);
    if (e == hipSuccess) e = hipMalloc(&c->A32, sizeof(float) * nAd);
    if (e == hipSuccess) e = cell_setup(c);
    if (e != hipSuccess) {
      delete c;
      return dev_status(e);
    }
  }
  if (!fp64_rows_served(c)) {
    pool_put(c);
    return HOM_EINVAL;
  }
  c->d = d;
  c->opt = o;
  // A goes to the device as given (FP64), is validated there (A2: finite,
  // symmetric positive definite at every point; contrast from the eigenvalue
  // range) and converted to the FP32 copy of the mixed path
  const size_t nAd = (size_t)c->nA * nQ;
  wait_user_stream(c);
  e = hipMemcpyAsync(c->A64, A, sizeof(double) * nAd,
                     A_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream);
  double lo = 0.0, hi = 0.0;
  int flags = 0;
  void* hp = nullptr;
  if (e == hipSuccess) e = pinned(c, sizeof(double) * 3 * 1024, &hp);
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_range_mu);
    double* scratch = nullptr;
    e = range_scratch(device, &scratch);
    if (e == hipSuccess)
      e = a_field_range(c->A64, d == 1 ? 1 : d, d == 1 ? HOM_A_ISO : kind, nQ, scratch,
                        (double*)hp, c->stream, &lo, &hi, &flags);
  }
  // samples of a trigonometric polynomial (a_trig) need not be positive
  // definite point by point, only finite
  const int bad = o.a_trig ? (flags & 1) : flags;
  if (e == hipSuccess && bad == 0) e = launch_convert(c->A64, c->A32, (long)nAd, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    delete c;
    return dev_status(e);
  }
  if (bad != 0) {
    pool_put(c);
    return (flags & 1) ? HOM_EINVAL : HOM_ENOTSPD;
  }
  c->rhoA = (flags & 2) ? INFINITY : hi / lo;
  c->Alo = (flags & 2) ? 0.0 : lo;
  c->Ahi = hi;
  hom_cell* hc = new (std::nothrow) hom_cell();
  if (!hc) {
    pool_put(c);
    return HOM_ENOMEM;
  }
  hc->impl = c;
  *out = hc;
  return HOM_OK;
}

void hom_destroy_cell(hom_cell* hc) {
  if (!hc) return;
  CellImpl* c = hc->impl;
  (void)hipStreamSynchronize(c->stream);
  delete hc;
  pool_put(c);
}

hom_status hom_cell_dims(const hom_cell* c, int32_t* d, int32_t* N, int32_t* Q) {
  if (!c) return HOM_EINVAL;
  const CellImpl& i = *c->impl;
  if (d) *d = i.d;
  for (int a = 0; a < 3; ++a) {
    if (N) N[a] = (a < i.d) ? i.N[a] : 1;
    if (Q) Q[a] = (a < i.d) ? i.Q[a] : 1;
  }
  return HOM_OK;
}


hom_status hom_solve(hom_cell* hc, int L, const double* E, double tol, double* strain, double* W,
                     double* J, const double* strain0, hom_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  if (!hc || L < 1 || !E || !(tol > 0) || !std::isfinite(tol)) return HOM_EINVAL;
  for (int i = 0; i < L * user_comps(hc->impl); ++i)
    if (!std::isfinite(E[i])) return HOM_EINVAL;
  CellImpl* c = hc->impl;
  std::lock_guard<std::mutex> lk(c->mu);
  const bool mixed = (c->opt.prec == HOM_MIXED);
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = ensure_work(c, L, mixed);
  if (e != hipSuccess) return dev_status(e);
  wait_user_stream(c);
  double* dE = nullptr;
  if ((e = upload_E(c, L, E, &dE)) != hipSuccess) return dev_status(e);
  hom_status st = HOM_OK;
  int it_inner = 0, it_outer = 0;
  double relres = 0.0;
  std::vector<ItemScal> hs;
  Work<double>& w = c->w64;
  const int P = partial_slots(c);
  do {
    // right-hand side b = -n . F[A E], r = p = b, x = 0; partials of (b, b)
    if ((e = launch_set_scal(w.sc, L, tol, mixed ? c->opt.max_outer : c->opt.max_iter, 1,
                             c->stream)) != hipSuccess)
      break;
    if ((e = pipe_rhs<double>(c, w, L, dE, nullptr)) != hipSuccess) break;
    const int tiles64 = project_tiles<double>(c);
    // (b, b) per load case, for the true relative residual (the mixed path's
    // outer scalars keep it as rho0)
    std::vector<double> bb;
    if (!mixed && (e = sum_partials_host(c, w.part, L, tiles64, bb)) != hipSuccess) break;
    if (!mixed) {
      // rho = (r0, r0) of b, or of the warm residual (partials in part2); the
      // stopping test is relative to ||b|| either way, so a warm start that
      // already meets it does not iterate
      if (strain0) {
        if ((e = warm_start(c, L, strain0, w.part2)) != hipSuccess) break;
        if ((e = launch_cg_init(w.sc, w.part2, P, tiles64, L, c->stream, nullptr, w.part)) !=
            hipSuccess)
          break;
      } else if ((e = launch_cg_init(w.sc, w.part, P, tiles64, L, c->stream)) != hipSuccess) {
        break;
      }
      if ((e = cg_run<double>(c, L, c->opt.max_iter, hs)) != hipSuccess) break;
      for (auto& s : hs) {
        it_inner = std::max(it_inner, s.iters);
        if (s.status == -5) st = HOM_EBREAKDOWN;
        else if (!s.conv && st == HOM_OK) st = HOM_ENOTCONV;
      }
    } else {
      // FP32 CG recursion with FP64 residual replacement.  The outer scalars
      // hold (b, b) as rho0 and the true residual (r, r) as rho.  When an
      // item's recursive residual has fallen by its inner tolerance (inner_tol,
      // or less once it predicts tol), x64 += ||b|| x32 and the recursive
      // residual is replaced by the FP64 one, b - Op x64; the search direction
      // is kept, so the Krylov recursion goes on instead of restarting.
      Work<float>& w32 = c->w32;
      ItemScal* outer = w.sc;
      // the recursion's scalars start cleared: an item done before its first
      // recursion (b = 0, or a warm start that meets the test) reports 0
      // iterations
      if ((e = launch_set_scal(w32.sc, L, 0.0, c->opt.max_iter, 0, c->stream)) != hipSuccess) break;
      if ((e = launch_outer_check(outer, w.part, P, tiles64, L, 1, c->stream)) != hipSuccess) break;
      if (strain0) {
        if ((e = warm_start(c, L, strain0, w.part)) != hipSuccess) break;
        if ((e = launch_outer_check(outer, w.part, P, tiles64, L, 0, c->stream)) != hipSuccess)
          break;
      }
      const int ub = update_blocks(c->S);
      if ((e = launch_inner_start(w.r, w32.r, w32.p, w32.x, c->S, c->S, c->H, scalar_n0(c), outer,
                                  w32.sc,
                                  c->opt.max_iter, 0, w32.part, P, ub, L, c->stream)) != hipSuccess)
        break;
      if ((e = launch_inner_init(w32.sc, w32.part, P, ub, L, outer, c->opt.inner_tol, kTolSafety,
                                 c->stream)) != hipSuccess)
        break;
      IterPlanner plan(L, c->opt.check_every);
      std::vector<ItemScal> ho(L), hi(L), hm(L);
      std::vector<char> live(L, 1);
      if ((e = read_scal2(c, outer, ho, w32.sc, hi, L)) != hipSuccess) break;
      for (int i = 0; i < L; ++i) live[i] = ho[i].active;
      int K = plan.next(hi, live);   // the first reading: no rate yet, Kmax
      for (;;) {
        bool any_outer = false;
        for (int i = 0; i < L; ++i) any_outer = any_outer || ho[i].active;
        if (!any_outer) break;
        if ((e = cg_launch<float>(c, L, K)) != hipSuccess) break;
        if ((e = read_scal(c, w32.sc, L, hi)) != hipSuccess) break;
        // an item whose recursion stopped (its residual fell by its inner
        // tolerance, or budget or breakdown) gets the FP64 residual
        bool any_replace = false;
        for (int i = 0; i < L; ++i) {
          hm[i] = ItemScal{};
          live[i] = ho[i].active;
          if (!ho[i].active) continue;
          if (hi[i].status == -5) st = HOM_EBREAKDOWN;
          if (!hi[i].active) {
            hm[i].active = 1;
            any_replace = true;
          }
        }
        if (any_replace) {
          if ((e = upload(c, w.mask, hm.data(), sizeof(ItemScal) * L, false)) != hipSuccess) break;
          if ((e = launch_inner_accumulate(w.x, w32.x, c->S, c->S, outer, ub, L, c->stream,
                                           w.mask)) != hipSuccess)
            break;
          if ((e = pipe_apply<double>(c, w, L, w.x, EPI_RESID, w.r, nullptr, w.b, w.mask,
                                      w.part)) != hipSuccess)
            break;
          if ((e = launch_outer_check(outer, w.part, P, tiles64, L, 0, c->stream, w.mask)) !=
              hipSuccess)
            break;
          if ((e = launch_inner_start(w.r, w32.r, w32.p, w32.x, c->S, c->S, c->H, scalar_n0(c), outer,
                                  w32.sc,
                                      c->opt.max_iter, 1, w32.part, P, ub, L, c->stream,
                                      w.mask)) != hipSuccess)
            break;
          if ((e = launch_inner_init(w32.sc, w32.part, P, ub, L, outer, c->opt.inner_tol,
                                     kTolSafety, c->stream, w.mask)) != hipSuccess)
            break;
          if ((e = read_scal2(c, outer, ho, w32.sc, hi, L)) != hipSuccess) break;
          for (int i = 0; i < L; ++i) {
            if (hm[i].active) plan.reset(i);
            live[i] = ho[i].active;
          }
        }
        K = plan.next(hi, live);
      }
      if (e != hipSuccess) break;
      for (int i = 0; i < L; ++i) {
        it_inner = std::max(it_inner, hi[i].iters);
        it_outer = std::max(it_outer, ho[i].iters);
        if (ho[i].status == -5) st = HOM_EBREAKDOWN;
        else if (!ho[i].conv && st == HOM_OK) st = HOM_ENOTCONV;
      }
    }
    // true residual with the FP64 operator (the mixed path's last outer check
    // evaluated it for the final iterate already)
    std::vector<double> rr;
    if (mixed) {
      std::vector<ItemScal> ho;
      if ((e = read_scal(c, w.sc, L, ho)) != hipSuccess) break;
      for (int i = 0; i < L; ++i) {
        rr.push_back(ho[i].rho);
        bb.push_back(ho[i].rho0);
      }
    } else {
      if ((e = pipe_apply<double>(c, w, L, w.x, EPI_RESID, w.q, nullptr, w.b, nullptr,
                                  w.part2)) != hipSuccess)
        break;
      if ((e = sum_partials_host(c, w.part2, L, tiles64, rr)) != hipSuccess) break;
    }
    for (int i = 0; i < L; ++i) {
      const double v = (bb[i] > 0) ? std::sqrt(rr[i] / bb[i]) : std::sqrt(rr[i]);
      relres = std::max(relres, v);
    }
    if ((e = homogenize(c, L, dE, strain, W, J)) != hipSuccess) break;
    e = hipStreamSynchronize(c->stream);
  } while (false);
  if (e != hipSuccess) return dev_status(e);
  if (info) {
    info->iters_inner = it_inner;
    info->iters_outer = it_outer;
    info->rel_resid_true = relres;
    info->rho_A = c->rhoA;
    info->seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return st;
}

hom_status hom_solve_ms(hom_cell* hc, int L, const double* E, double tol, double* strain,
                        double* W, double* J, hom_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  if (!hc || L < 1 || !E || !(tol > 0) || !std::isfinite(tol)) return HOM_EINVAL;
  for (int i = 0; i < L * user_comps(hc->impl); ++i)
    if (!std::isfinite(E[i])) return HOM_EINVAL;
  CellImpl* c = hc->impl;
  // lambda = (c_A + C_A) / 2 needs a positive lower eigenvalue bound
  if (!(c->Alo > 0.0)) return HOM_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = ensure_work(c, L, false);
  if (e != hipSuccess) return dev_status(e);
  wait_user_stream(c);
  double* dE = nullptr;
  if ((e = upload_E(c, L, E, &dE)) != hipSuccess) return dev_status(e);
  Work<double>& w = c->w64;
  const int P = partial_slots(c);
  hom_status st = HOM_OK;
  int iters = 0;
  double relres = 0.0;
  std::vector<ItemScal> hs;
  do {
    // b = -n . F[A E], x = 0; rho0 = (b, b); the step 1 / lambda with
    // lambda = (c_A + C_A) / 2 goes to the device scalars (a captured graph
    // may serve later cells of this shape)
    if ((e = launch_set_scal(w.sc, L, tol, c->opt.max_iter, 1, c->stream,
                             2.0 / (c->Alo + c->Ahi))) != hipSuccess)
      break;
    if ((e = pipe_rhs<double>(c, w, L, dE, nullptr)) != hipSuccess) break;
    if ((e = launch_cg_init(w.sc, w.part, P, project_tiles<double>(c), L, c->stream)) !=
        hipSuccess)
      break;
    if ((e = cg_run<double>(c, L, c->opt.max_iter, hs, 1)) != hipSuccess) break;
    for (auto& q : hs) {
      iters = std::max(iters, q.iters);
      if (q.status == -5) st = HOM_EBREAKDOWN;
      else if (!q.conv && st == HOM_OK) st = HOM_ENOTCONV;
      // the last booking holds (r, r) of the returned iterate, r = b - Op x
      if (q.rho0 > 0) relres = std::max(relres, std::sqrt(q.rho / q.rho0));
    }
    if ((e = homogenize(c, L, dE, strain, W, J)) != hipSuccess) break;
    e = hipStreamSynchronize(c->stream);
  } while (false);
  if (e != hipSuccess) return dev_status(e);
  if (info) {
    info->iters_inner = iters;
    info->iters_outer = 0;
    info->rel_resid_true = relres;
    info->rho_A = c->rhoA;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return st;
}

hom_status hom_apply(hom_cell* hc, hom_prec prec, int L, const double* u, double* out) {
  if (!hc || L < 1 || !u || !out || (prec != HOM_FP64 && prec != HOM_MIXED)) return HOM_EINVAL;
  CellImpl* c = hc->impl;
  if (c->d != c->dd) return HOM_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = ensure_work(c, L, prec == HOM_MIXED);
  if (e != hipSuccess) return dev_status(e);
  wait_user_stream(c);
  Work<double>& w = c->w64;
  double* dE = nullptr;
  std::vector<double> zero((size_t)L * user_comps(c), 0.0);
  do {
    if ((e = upload_E(c, L, zero.data(), &dE)) != hipSuccess) break;
    if ((e = pipe_project_real(c, w, L, u, w.x)) != hipSuccess) break;
    if (prec == HOM_FP64) {
      if ((e = pipe_apply<double>(c, w, L, w.x, EPI_STORE, w.q, nullptr, nullptr, nullptr,
                                  nullptr)) != hipSuccess)
        break;
    } else {
      Work<float>& w32 = c->w32;
      const long n = 2 * c->S * L;
      if ((e = launch_convert((const double*)w.x, (float*)w32.x, n, c->stream)) != hipSuccess) break;
      if ((e = pipe_apply<float>(c, w32, L, w32.x, EPI_STORE, w32.q, nullptr, nullptr, nullptr,
                                 nullptr)) != hipSuccess)
        break;
      if ((e = launch_widen((const float*)w32.q, (double*)w.q, n, c->stream)) != hipSuccess) break;
    }
    if ((e = pipe_synth(c, c->w64, L, w.q, dE, false, out)) != hipSuccess) break;
    e = hipStreamSynchronize(c->stream);
  } while (false);
  return dev_status(e);
}

hom_status hom_project(hom_cell* hc, int L, const double* u, double* out) {
  if (!hc || L < 1 || !u || !out) return HOM_EINVAL;
  CellImpl* c = hc->impl;
  if (c->d != c->dd) return HOM_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = ensure_work(c, L, false);
  if (e != hipSuccess) return dev_status(e);
  wait_user_stream(c);
  double* dE = nullptr;
  std::vector<double> zero((size_t)L * user_comps(c), 0.0);
  do {
    if ((e = upload_E(c, L, zero.data(), &dE)) != hipSuccess) break;
    if ((e = pipe_project_real(c, c->w64, L, u, c->w64.x)) != hipSuccess) break;
    if ((e = pipe_synth(c, c->w64, L, c->w64.x, dE, false, out)) != hipSuccess) break;
    e = hipStreamSynchronize(c->stream);
  } while (false);
  return dev_status(e);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// allocation-free operator apply: the workspace lives in a fixed array of
// device memory inside the library (one copy per GPU, kept until the process
// ends) instead of the cell's own buffers
// ---------------------------------------------------------------------------
namespace hom {

static __device__ __align__(256) unsigned char scratch[HOM_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, unsigned char*> g_scratch_ptr;

// device address of this GPU's copy of the array, taken once per device with
// that device current (the array's name is only a host-side stand-in)
static hipError_t scratch_base(int device, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<unsigned char*>(ptr);
  *out = static_cast<unsigned char*>(ptr);
  return hipSuccess;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// scratch bytes of an apply on L items: FP64 potential, output and two
// component-spectrum buffers (the FP32 pass reuses the latter), FP32 potential
// and output (HOM_MIXED), zero load cases for the synthesis
static size_t noalloc_bytes(const CellImpl* c, int L, bool mixed) {
  const size_t sv = sizeof(cpx<double>) * (size_t)c->S * L;
  const size_t xv = sizeof(cpx<double>) * (size_t)c->Xe * c->nf * L;
  size_t b = 2 * align256(sv) + 2 * align256(xv) + align256(sizeof(double) * 6 * (size_t)L);
  if (mixed) b += 2 * align256(sizeof(cpx<float>) * (size_t)c->S * L);
  return b;
}

}  // namespace hom

extern "C" hom_status hom_apply_noalloc(hom_cell* hc, hom_prec prec, int L, const double* u,
                                        double* out) {
  if (!hc || L < 1 || !u || !out || (prec != HOM_FP64 && prec != HOM_MIXED)) return HOM_EINVAL;
  CellImpl* c = hc->impl;
  if (c->d != c->dd) return HOM_EINVAL;
  const bool mixed = (prec == HOM_MIXED);
  if (noalloc_bytes(c, L, mixed) > (size_t)HOM_NOALLOC_SCRATCH_BYTES) return HOM_ESCRATCH;
  std::lock_guard<std::mutex> lk(c->mu);
  hipError_t e = hipSetDevice(c->device);
  unsigned char* base = nullptr;
  if (e == hipSuccess) e = scratch_base(c->device, &base);
  if (e != hipSuccess) return dev_status(e);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* q = base + off;
    off += align256(bytes);
    return q;
  };
  const size_t sv = sizeof(cpx<double>) * (size_t)c->S * L;
  const size_t xv = sizeof(cpx<double>) * (size_t)c->Xe * c->nf * L;
  Work<double> w;
  w.items = L;
  w.x = reinterpret_cast<cpx<double>*>(take(sv));
  w.q = reinterpret_cast<cpx<double>*>(take(sv));
  w.X1 = reinterpret_cast<cpx<double>*>(take(xv));
  w.X2 = reinterpret_cast<cpx<double>*>(take(xv));
  w.r = w.p = w.b = w.x;   // not read by these passes (no CG epilogue)
  double* dE = reinterpret_cast<double*>(take(sizeof(double) * 6 * (size_t)L));
  Work<float> w32;
  if (mixed) {
    w32.items = L;
    w32.x = reinterpret_cast<cpx<float>*>(take(sizeof(cpx<float>) * (size_t)c->S * L));
    w32.q = reinterpret_cast<cpx<float>*>(take(sizeof(cpx<float>) * (size_t)c->S * L));
    // the FP32 component spectra fit in the first half of the FP64 ones,
    // which are not live while the FP32 passes run
    w32.X1 = reinterpret_cast<cpx<float>*>(w.X1);
    w32.X2 = reinterpret_cast<cpx<float>*>(w.X2);
    w32.r = w32.p = w32.b = w32.x;
  }
  // work is queued on the caller's stream (the cell's own when it gave none)
  // and not waited for; the cell's stream is restored before returning
  const hipStream_t own = c->stream;
  if (c->opt.stream) c->stream = (hipStream_t)c->opt.stream;
  do {
    // the synthesis adds the load case, which is zero here; the array keeps
    // the last call's contents, so it is cleared on every call
    if ((e = launch_zero(dE, 6 * (long)L, c->stream)) != hipSuccess) break;
    if ((e = pipe_project_real(c, w, L, u, w.x)) != hipSuccess) break;
    if (!mixed) {
      if ((e = pipe_apply<double>(c, w, L, w.x, EPI_STORE, w.q, nullptr, nullptr, nullptr,
                                  nullptr)) != hipSuccess)
        break;
    } else {
      const long n = 2 * c->S * L;
      if ((e = launch_convert((const double*)w.x, (float*)w32.x, n, c->stream)) != hipSuccess) break;
      if ((e = pipe_apply<float>(c, w32, L, w32.x, EPI_STORE, w32.q, nullptr, nullptr, nullptr,
                                 nullptr)) != hipSuccess)
        break;
      if ((e = launch_widen((const float*)w32.q, (double*)w.q, n, c->stream)) != hipSuccess) break;
    }
    e = pipe_synth(c, w, L, w.q, dE, false, out);
  } while (false);
  c->stream = own;
  return dev_status(e);
}

// ---------------------------------------------------------------------------
// per-kernel timing of one CG iteration
// ---------------------------------------------------------------------------
namespace hom {

template <class T>
static hipError_t profile_impl(CellImpl* c, int L, int reps, double* ms, double* bytes) {
  const bool pair = pair_mode<T>(c);
  Work<T>& w = work_of<T>(c);
  hipError_t e;
  std::vector<double> hE((size_t)L * c->nf, 0.0);
  for (int l = 0; l < L; ++l) hE[(size_t)l * c->nf + (l % c->nf)] = 1.0;
  double* dE = nullptr;
  if ((e = hipMalloc(&dE, sizeof(double) * hE.size())) != hipSuccess) return e;
  if ((e = hipMemcpy(dE, hE.data(), sizeof(double) * hE.size(), hipMemcpyHostToDevice)) !=
      hipSuccess) {
    (void)hipFree(dE);
    return e;
  }
  const int P = partial_slots(c);
  const int Q0 = c->Q[0], Q1 = c->Q[1], Q2 = c->Q[2];
  const int tiles = project_tiles<T>(c), rtiles = row_tiles<T>(c);
  const int ub = update_blocks(c->S);
  auto reset = [&]() -> hipError_t {
    hipError_t e2 = launch_set_scal(w.sc, L, 0.0, 1 << 30, 1, c->stream);
    if (e2 == hipSuccess) e2 = pipe_rhs<T>(c, w, L, dE, nullptr);
    if (e2 == hipSuccess) e2 = launch_cg_init(w.sc, w.part, P, tiles, L, c->stream);
    return e2;
  };
  for (int i = 0; i < 9; ++i) ms[i] = bytes[i] = 0.0;
  const double esz = sizeof(cpx<T>), Ts = sizeof(T);
  const long inner = inner0(c);
  const long rows = (c->dd == 3) ? (long)Q0 * Q1 : Q0;
  const double S = (double)c->S;
  cpx<T>* Xrow = (c->dd == 3) ? w.X2 : w.X1;
  // every kernel of `reps` consecutive CG iterations carries its own event
  // pair, recorded by the dispatch itself (no marker packets in between), so
  // each kernel is timed in the context it runs in during a solve: caches
  // as left by its predecessor, no gaps added
  // slots: 0 expand, 1 axis-1 inverse, 2 row, 3 axis-1 forward, 4 project,
  // 5 update (alpha and beta are derived inside these kernels), 6 the
  // end-of-launch bookkeeping (once per launch of up to 16 iterations, shown
  // per iteration as 1/16 of its duration), 7 the direction step; ms[7] and
  // bytes[7] are then moved to slot 8 and slot 7 holds the whole iteration
  const int NK = 8;
  std::vector<hipEvent_t> ev((size_t)reps * NK * 2, nullptr);
  for (auto& x : ev) (void)hipEventCreate(&x);
  std::vector<int> launched((size_t)reps * NK, 0);
  e = reset();
  for (int it = 0; it < reps && e == hipSuccess; ++it) {
    // as inside a launched graph: x is left to the next expansion except in
    // the last iteration
    const CgFuse cg{w.part2, ub, it > 0 ? 1 : 0, w.part, rtiles};
    hipEvent_t* E = ev.data() + (size_t)it * NK * 2;
    int* Ln = launched.data() + (size_t)it * NK;
    // the first-axis stages of a cell with several potentials are two kernels
    auto arm = [&](int k) {
      const bool two = c->npot > 1 && ((k == 0 && !bexpand_kernel<T>(c)) || k == 4);
      arm_launch_events(E[2 * k], E[2 * k + 1], two ? 2 : 1);
      Ln[k] = 1;
    };
    arm(7);
    e = launch_cg_direction<T>(direction_args<T>(c, w, ub, it > 0), L, ub, c->stream);
    if (e == hipSuccess) {
      arm(0);
      e = stage_expand<T>(c, w, L, w.p, Q0, w.sc, pair);
    }
    if (e == hipSuccess && c->dd == 3) {
      arm(1);
      e = stage_axis1<T>(c, w, L, +1, Q0, Q1, w.X1, w.X2, w.sc, pair);
    }
    if (e == hipSuccess) {
      arm(2);
      e = stage_row<T>(c, L, ROW_APPLY, Xrow, Xrow, Q0, c->dd == 3 ? Q1 : 1, c->dd == 3 ? Q2 : Q1,
                       nullptr, nullptr, nullptr, w.sc, w.part);
    }
    if (e == hipSuccess && c->dd == 3) {
      arm(3);
      e = stage_axis1<T>(c, w, L, -1, Q0, Q1, w.X2, w.X1, w.sc, pair);
    }
    if (e == hipSuccess) {
      arm(4);
      e = stage_project<T>(c, w, L, w.X1, Q0, EPI_STORE, w.q, nullptr, nullptr, nullptr, nullptr,
                           nullptr, nullptr, w.sc, nullptr, pair, &cg);
    }
    if (e == hipSuccess) {
      arm(5);
      e = launch_cg_update<T>(update_args<T>(c, w, rtiles, it == reps - 1, true), L, ub,
                              c->stream);
    }
    if (e == hipSuccess && it == reps - 1) {
      arm(6);
      e = launch_cg_finalize(w.sc, w.part2, P, ub, L, c->stream);
    }
  }
  arm_launch_events(nullptr, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  for (int it = 0; it < reps && e == hipSuccess; ++it) {
    hipEvent_t* E = ev.data() + (size_t)it * NK * 2;
    const int* Ln = launched.data() + (size_t)it * NK;
    for (int k = 0; k < NK; ++k) {
      float t = 0.f;
      if (!Ln[k] || hipEventElapsedTime(&t, E[2 * k], E[2 * k + 1]) != hipSuccess) continue;
      ms[k] += (k == 6) ? t / 16.0 : t / reps;
    }
  }
  ms[8] = ms[7];
  ms[7] = 0.0;
  if (c->dd != 3) ms[1] = ms[3] = 0.0;
  for (int k = 0; k < 7; ++k) ms[7] += ms[k];
  ms[7] += ms[8];
  // algorithmic bytes of the steady state inside a graph: the direction step
  // reads r, p, x and writes p, x; the expansion reads p and writes the d
  // fields; the update reads r, q, writes r
  // (cells that hand two spectra between the first- and middle-axis passes:
  // two fields there instead of d)
  const double nx = pair ? 2.0 : (double)c->nf;
  bytes[8] = L * 5.0 * S * esz;
  bytes[0] = L * (S * esz + nx * Q0 * inner * esz);
  if (c->dd == 3) {
    bytes[1] = L * (double)Q0 * c->H * esz * (nx * c->N[1] + (double)c->nf * Q1);
    bytes[3] = bytes[1];
  }
  bytes[2] = L * 2.0 * c->nf * rows * c->H * esz + (double)c->nA * c->nQ * Ts;
  bytes[4] = L * (nx * Q0 * inner * esz + S * esz);
  bytes[5] = L * 3.0 * S * esz;
  for (int i = 0; i < 6; ++i) bytes[7] += bytes[i];
  bytes[7] += bytes[8];
  for (auto& x : ev) (void)hipEventDestroy(x);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(dE);
  return e;
}

}  // namespace hom

extern "C" hom_status hom_profile_iteration(hom_cell* hc, hom_prec prec, int L, int reps,
                                            double* ms, double* bytes) {
  if (!hc || L < 1 || reps < 1 || !ms || !bytes) return HOM_EINVAL;
  if (prec != HOM_FP64 && prec != HOM_MIXED) return HOM_EINVAL;
  CellImpl* c = hc->impl;
  std::lock_guard<std::mutex> lk(c->mu);
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = ensure_work(c, L, prec == HOM_MIXED);
  if (e != hipSuccess) return dev_status(e);
  if (prec == HOM_FP64) e = profile_impl<double>(c, L, reps, ms, bytes);
  else e = profile_impl<float>(c, L, reps, ms, bytes);
  return dev_status(e);
}

extern "C" hom_status hom_set_specialized(int enable) {
  hom::set_static_enabled(enable != 0);
  return HOM_OK;
}

// ---------------------------------------------------------------------------
// autotuner: time every variant of each pass of a cell's CG iteration
// ---------------------------------------------------------------------------
namespace hom {

// the passes of one CG iteration of c with their tuning keys and FFT lengths,
// in the order expand, axis-1 inverse, row, axis-1 forward, project (the
// axis-1 passes only in 3-D)
struct PassKey {
  int slot;
  TuneKey key;
  int fft_len;
};
template <class T>
static std::vector<PassKey> pass_keys(const CellImpl* c) {
  const int dd = c->dd, esz = (int)sizeof(cpx<T>);
  const int Q0 = c->Q[0], Q1 = c->Q[1], Q2 = c->Q[2];
  const int Glast = (dd == 3) ? Q2 : Q1;
  std::vector<PassKey> v;
  // elastic cells run the generic kernels of every pass but the axis-1 ones
  // (shared with the scalar cells of the shape): nothing of theirs to tune
  if (c->elastic) return v;
  // a cell with two potentials per frequency runs the generic expand and
  // project kernels: their variants are not its to time or force
  const bool col = (c->npot == 1);
  // cells whose first- and middle-axis passes hand over two spectra tune
  // the kernels of that form
  const bool pair = pair_mode<T>(c);
  if (col) v.push_back({0, TuneKey{pair ? KK_EXPAND2 : KK_EXPAND, esz, Q0, c->N[0], dd}, Q0});
  if (dd == 3)
    v.push_back({1, TuneKey{pair ? KK_MID2_INV : KK_PLAIN_INV, esz, Q1, c->N[1], 0}, Q1});
  v.push_back({2, TuneKey{KK_ROW, esz, Glast, c->N[dd - 1], dd}, Glast});
  if (dd == 3)
    v.push_back({3, TuneKey{pair ? KK_MID2_FWD : KK_PLAIN_FWD, esz, Q1, c->N[1], 0}, Q1});
  if (col) v.push_back({4, TuneKey{pair ? KK_PROJECT2 : KK_PROJECT, esz, Q0, c->N[0], dd}, Q0});
  return v;
}

static int pass_variant_count(const PassKey& pk) {
  const DevPlan* pl = nullptr;
  if (get_dev_plan(pk.fft_len, &pl) != hipSuccess) return 0;
  return (int)static_variants(pk.key.kind, pk.key.esz, pk.key.n, pk.key.ntrial, pk.key.d, pl->p)
      .size();
}

// Each variant of each pass is timed inside whole CG iterations (the other
// passes at their current choice), so it sees the caches its predecessor
// leaves, as in a solve; passes are tuned one after the other.
template <class T>
static hipError_t autotune_impl(CellImpl* c, int L, int reps, double* best_us) {
  Work<T>& w = work_of<T>(c);
  hipError_t e;
  std::vector<double> hE((size_t)L * c->nf, 0.0);
  for (int l = 0; l < L; ++l) hE[(size_t)l * c->nf + (l % c->nf)] = 1.0;
  double* dE = nullptr;
  if ((e = hipMalloc(&dE, sizeof(double) * hE.size())) != hipSuccess) return e;
  e = hipMemcpy(dE, hE.data(), sizeof(double) * hE.size(), hipMemcpyHostToDevice);
  const int P = partial_slots(c);
  // a fresh right-hand side before every measurement; tol 0 keeps every item
  // iterating through the few iterations timed
  auto reset = [&]() -> hipError_t {
    hipError_t e2 = launch_set_scal(w.sc, L, 0.0, 1 << 30, 1, c->stream);
    if (e2 == hipSuccess) e2 = pipe_rhs<T>(c, w, L, dE, nullptr);
    if (e2 == hipSuccess) e2 = launch_cg_init(w.sc, w.part, P, project_tiles<T>(c), L, c->stream);
    return e2;
  };
  hipEvent_t ev0, ev1;
  (void)hipEventCreate(&ev0);
  (void)hipEventCreate(&ev1);
  const int R = std::max(1, reps);
  for (const PassKey& pk : pass_keys<T>(c)) {
    if (e != hipSuccess) break;
    const int nvar = pass_variant_count(pk);
    double best = 1e30;
    int best_v = nvar > 0 ? 0 : -1;
    for (int v = -1; v < nvar; ++v) {
      set_choice(pk.key, v);
      hipError_t e2 = reset();
      if (e2 == hipSuccess) e2 = cg_body<T>(c, w, L, 2);  // warm-up; fails when no generic shape fits
      if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
      if (e2 != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
      (void)hipEventRecord(ev0, c->stream);
      e2 = cg_body<T>(c, w, L, R);
      (void)hipEventRecord(ev1, c->stream);
      if (e2 == hipSuccess) e2 = hipEventSynchronize(ev1);
      float ms = 0.f;
      if (e2 == hipSuccess) e2 = hipEventElapsedTime(&ms, ev0, ev1);
      if (e2 != hipSuccess) {
        e = e2;
        break;
      }
      const double us = 1e3 * ms / R;
      if (us < best) {
        best = us;
        best_v = v;
      }
    }
    set_choice(pk.key, best_v);
    if (best_us) best_us[pk.slot] = best;
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(dE);
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  return e;
}

static std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string a = prop.gcnArchName;
  return a.substr(0, a.find(':'));
}

}  // namespace hom

extern "C" hom_status hom_autotune(hom_cell* hc, hom_prec prec, int L, int reps, double* best_us) {
  if (!hc || L < 1 || reps < 1 || (prec != HOM_FP64 && prec != HOM_MIXED)) return HOM_EINVAL;
  CellImpl* c = hc->impl;
  std::lock_guard<std::mutex> lk(c->mu);
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = ensure_work(c, L, prec == HOM_MIXED);
  if (e != hipSuccess) return dev_status(e);
  if (best_us)
    for (int i = 0; i < 5; ++i) best_us[i] = 0.0;
  e = (prec == HOM_FP64) ? autotune_impl<double>(c, L, reps, best_us)
                         : autotune_impl<float>(c, L, reps, best_us);
  return dev_status(e);
}

extern "C" hom_status hom_pass_variants(hom_cell* hc, hom_prec prec, int32_t* counts) {
  if (!hc || !counts || (prec != HOM_FP64 && prec != HOM_MIXED)) return HOM_EINVAL;
  hom::CellImpl* c = hc->impl;
  std::lock_guard<std::mutex> lk(c->mu);
  if (hipSetDevice(c->device) != hipSuccess) return HOM_EDEVICE;
  for (int i = 0; i < 5; ++i) counts[i] = 0;
  const auto keys = (prec == HOM_FP64) ? hom::pass_keys<double>(c) : hom::pass_keys<float>(c);
  for (const auto& pk : keys) counts[pk.slot] = hom::pass_variant_count(pk);
  return HOM_OK;
}

extern "C" hom_status hom_force_variant(hom_cell* hc, hom_prec prec, int pass, int variant) {
  if (!hc || (prec != HOM_FP64 && prec != HOM_MIXED) || pass < 0 || pass > 4) return HOM_EINVAL;
  hom::CellImpl* c = hc->impl;
  std::lock_guard<std::mutex> lk(c->mu);
  if (hipSetDevice(c->device) != hipSuccess) return HOM_EDEVICE;
  const auto keys = (prec == HOM_FP64) ? hom::pass_keys<double>(c) : hom::pass_keys<float>(c);
  for (const auto& pk : keys) {
    if (pk.slot != pass) continue;
    if (variant < -1 || variant >= hom::pass_variant_count(pk)) return HOM_EINVAL;
    hom::set_choice(pk.key, variant);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    return HOM_OK;
  }
  return HOM_EINVAL;   // the pass does not exist for this cell (axis 1 of a 2-D cell)
}

extern "C" hom_status hom_current_variant(hom_cell* hc, hom_prec prec, int pass,
                                          int32_t* variant) {
  if (!hc || !variant || (prec != HOM_FP64 && prec != HOM_MIXED) || pass < 0 || pass > 4)
    return HOM_EINVAL;
  hom::CellImpl* c = hc->impl;
  std::lock_guard<std::mutex> lk(c->mu);
  if (hipSetDevice(c->device) != hipSuccess) return HOM_EDEVICE;
  const auto keys = (prec == HOM_FP64) ? hom::pass_keys<double>(c) : hom::pass_keys<float>(c);
  for (const auto& pk : keys) {
    if (pk.slot != pass) continue;
    const hom::DevPlan* pl = nullptr;
    if (hom::get_dev_plan(pk.fft_len, &pl) != hipSuccess) return HOM_EDEVICE;
    const hom::StaticKernel* sk =
        hom::find_static(pk.key.kind, pk.key.esz, pk.key.n, pk.key.ntrial, pk.key.d, pl->p);
    *variant = -1;
    if (sk) {
      const auto v = hom::static_variants(pk.key.kind, pk.key.esz, pk.key.n, pk.key.ntrial,
                                          pk.key.d, pl->p);
      for (size_t i = 0; i < v.size(); ++i)
        if (v[i] == sk) *variant = (int32_t)i;
    }
    return HOM_OK;
  }
  return HOM_EINVAL;
}

extern "C" hom_status hom_tune_save(const char* path) {
  if (!path) return HOM_EINVAL;
  FILE* f = std::fopen(path, "w");
  if (!f) return HOM_EINVAL;
  std::fprintf(f, "{\"arch\": \"%s\", \"choices\": [", hom::arch_name().c_str());
  bool first = true;
  for (const auto& kv : hom::all_choices()) {
    const hom::TuneKey& k = kv.first;
    std::fprintf(f, "%s\n  [%d, %d, %d, %d, %d, %d]", first ? "" : ",", k.kind, k.esz, k.n,
                 k.ntrial, k.d, kv.second);
    first = false;
  }
  std::fprintf(f, "\n]}\n");
  std::fclose(f);
  return HOM_OK;
}

extern "C" hom_status hom_tune_load(const char* path) {
  if (!path) return HOM_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return HOM_EINVAL;
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, n);
  std::fclose(f);
  const size_t a = s.find("\"arch\"");
  const size_t q1 = (a == std::string::npos) ? a : s.find('"', s.find(':', a) + 1);
  const size_t q2 = (q1 == std::string::npos) ? q1 : s.find('"', q1 + 1);
  if (q2 == std::string::npos) return HOM_EINVAL;
  if (s.substr(q1 + 1, q2 - q1 - 1) != hom::arch_name()) return HOM_EINVAL;  // tuned elsewhere
  size_t p = s.find("\"choices\"");
  if (p == std::string::npos) return HOM_EINVAL;
  std::vector<long> v;
  for (p = s.find('[', p); p < s.size(); ++p) {
    if ((s[p] >= '0' && s[p] <= '9') || s[p] == '-') {
      char* end = nullptr;
      v.push_back(std::strtol(s.c_str() + p, &end, 10));
      p = (size_t)(end - s.c_str()) - 1;
    }
  }
  if (v.size() % 6) return HOM_EINVAL;
  for (size_t i = 0; i < v.size(); i += 6)
    hom::set_choice(hom::TuneKey{(int)v[i], (int)v[i + 1], (int)v[i + 2], (int)v[i + 3], (int)v[i + 4]},
                    (int)v[i + 5]);
  return HOM_OK;
}

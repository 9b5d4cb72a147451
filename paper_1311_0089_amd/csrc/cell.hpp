// cell.hpp -- internal cell, workspace and pipeline declarations.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "hom.h"
#include "kernels.hpp"
#include "plan.hpp"

namespace hom {

// device buffers of one precision for `items` solver items
template <class T>
struct Work {
  int items = 0;
  cpx<T>* x = nullptr;   // iterate (scalar potential)      [items][S]
  cpx<T>* r = nullptr;   // residual                        [items][S]
  cpx<T>* p = nullptr;   // search direction                [items][S]
  cpx<T>* q = nullptr;   // operator output                 [items][S]
  cpx<T>* b = nullptr;   // right-hand side                 [items][S]
  cpx<T>* X1 = nullptr;  // component spectra, ping         [items][d][Xe]
  cpx<T>* X2 = nullptr;  // component spectra, pong         [items][d][Xe]
  double* part = nullptr;   // partial sums                 [items][P]
  double* part2 = nullptr;  // second partial buffer        [items][P]
  ItemScal* sc = nullptr;   // solver scalars               [items]
  ItemScal* mask = nullptr; // per-item selection of masked launches [items]
  std::vector<void*> owned;
  ~Work();
  hipError_t alloc(int items, long S, long Xe, int d, int P);
};

// a captured CG graph: precision, items, iterations, and the version of the
// kernel choices it was captured with (tune_version)
struct GraphKey {
  int prec, items, K;
  unsigned version;
  int solver;   // 0 conjugate gradients, 1 Moulinec-Suquet
  bool operator<(const GraphKey& o) const {
    if (solver != o.solver) return solver < o.solver;
    if (prec != o.prec) return prec < o.prec;
    if (items != o.items) return items < o.items;
    if (K != o.K) return K < o.K;
    return version < o.version;
  }
};

struct CellImpl {
  int d = 0, dd = 0;          // user dimension, dimension run on the device (>= 2)
  int N[3] = {1, 1, 1};       // trial grid (device dims)
  int Q[3] = {1, 1, 1};       // quadrature grid
  int scheme = HOM_GANI, kind = HOM_A_ISO, nA = 1;
  int dual = 0;               // dual (flux) problem on J_N
  int npot = 1;               // potentials per frequency (2: 3-D dual; d: elasticity)
  int nf = 2;                 // field components: dd, or dd(dd+1)/2 (elasticity)
  int elastic = 0;            // linear elasticity (kind HOM_A_ELASTIC)
  double Y[3] = {0.5, 0.5, 0.5};
  hom_options opt{};
  double rhoA = 1.0;
  double Alo = 1.0, Ahi = 1.0;  // eigenvalue range c_A, C_A of the coefficient (A2)
  long S = 0;                 // scalar spectrum elements per item
  long Xe = 0;                // component-spectrum elements per component per item
  long nN = 0, nQ = 0;        // grid points
  int H = 0;                  // half-spectrum bins of the last axis
  double* A64 = nullptr;      // [nA][Q]
  float* A32 = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
  Work<double> w64;
  Work<float> w32;
  double* ebuf = nullptr;     // FP64 real strain scratch [items][d][Q]
  long ebuf_items = 0;
  double* quad = nullptr;     // quadrature partials / outputs
  double* dE = nullptr;       // device copy of the load cases [items][dd]
  int dE_items = 0;
  int A_group = 1 << 30;      // items sharing one coefficient block (batched cells: d)
  long A_block = 0;           // elements per coefficient block (0: one shared block)
  std::map<GraphKey, hipGraphExec_t> graphs;
  std::mutex mu;
  ~CellImpl();
};

// non-owning view of items [i0, items) of a workspace
template <class T>
Work<T> work_view(const Work<T>& w, int i0, long S, long Xe, int d, int P) {
  Work<T> v;
  v.items = w.items - i0;
  v.x = w.x + (long)i0 * S;
  v.r = w.r + (long)i0 * S;
  v.p = w.p + (long)i0 * S;
  v.q = w.q + (long)i0 * S;
  v.b = w.b + (long)i0 * S;
  v.X1 = w.X1 + (long)i0 * d * Xe;
  v.X2 = w.X2 + (long)i0 * d * Xe;
  v.part = w.part + (long)i0 * P;
  v.part2 = w.part2 + (long)i0 * P;
  v.sc = w.sc + i0;
  return v;
}

// engine pool (solver.hip): reuse the device state of destroyed cells
CellImpl* pool_take(int device, const CellImpl& key);
void pool_put(CellImpl* c);

// pipeline entry points (solver.hip)
hipError_t cell_setup(CellImpl* c);
hipError_t ensure_work(CellImpl* c, int items, bool need32);
template <class T>
Work<T>& work_of(CellImpl* c);

// RHS b = -n . F[A E] (with r = p = b, x = 0) and rho0 = (b, b)
template <class T>
hipError_t pipe_rhs(CellImpl* c, Work<T>& w, int items, const double* dE, ItemScal* sc);
// q = Op(in) with epilogue epi
template <class T>
hipError_t pipe_apply(CellImpl* c, Work<T>& w, int items, const cpx<T>* in, int epi,
                      cpx<T>* out, const cpx<T>* pdot, const cpx<T>* b, ItemScal* sc,
                      double* partials, const CgFuse* cg = nullptr);
// real strain on grid G (G = N or Q) from the potential: e = E + F_G^-1 Pad(n c)
hipError_t pipe_synth(CellImpl* c, Work<double>& w, int items, const cpx<double>* cin,
                      const double* dE, bool onQ, double* out);
// launch helpers shared with the serving runtime
int update_blocks(long S);
// pinned host staging of at least `bytes` bytes (the calling thread's)
hipError_t pinned(CellImpl* c, size_t bytes, void** out);
int scalar_n0(const CellImpl* c);
int partial_slots(const CellImpl* c);
template <class T>
int project_tiles(CellImpl* c);
// K captured iterations of conjugate gradients (solver 0) or of the
// Moulinec-Suquet scheme (solver 1, FP64 only)
template <class T>
hipError_t cg_graph(CellImpl* c, int items, int K, hipGraphExec_t* out, int solver = 0);
// scalar potential of a real field u on the N grid: c = n . F_N[u]
hipError_t pipe_project_real(CellImpl* c, Work<double>& w, int items, const double* u,
                             cpx<double>* cout);

}  // namespace hom

struct hom_cell {
  hom::CellImpl* impl;
};

// server.cpp -- continuous batching of cell solves (hom_server_* of hom.h).
//
// Requests are grouped into size classes (device dims, grid, quadrature,
// coefficient layout, cell lengths).  A class owns one batched engine with
// `slots` slots of d solver items each: coefficient blocks per slot, FP64
// and FP32 workspaces for every item, and one captured HIP graph of K inner
// (FP32) CG iterations over all items.  Per-item flags in device memory mask
// every kernel, so a slot can be admitted, refined or retired while the
// others keep iterating:
//   admit   copy the request's coefficients into a free slot, FP64 RHS and
//           outer check, start the inner FP32 solve       (mask: new items)
//   tick    replay the class graph (K iterations, all live items), read the
//           flags back
//   refine  items whose FP32 recursion stopped: x64 += x32, FP64 residual
//           with the FP64 operator, outer check, the FP64 residual replaces
//           the recursive one (search direction kept)  (mask: those items)
//   retire  slots whose items all stopped: FP64 strain synthesis and energy
//           quadrature, results, free the slot
// Classes run on their own streams, so their work overlaps on the device.
// Admission is by device footprint against the server's budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "cell.hpp"

namespace hom {

struct Req {
  uint64_t ticket = 0;
  CellImpl* cell = nullptr;
  int L = 0;
  std::vector<double> E;
  double tol = 0;
  double t_submit = 0, t_admit = -1, t_done = -1;
  int status = HOM_EBUSY;
  std::vector<double> W, J;
  hom_info info{};
  int slot = -1;
  bool done = false;
  std::vector<int> inner_sum;
};

struct SizeClass {
  CellImpl* eng = nullptr;   // batched engine of this shape
  int slots = 0, dd = 0, items = 0;
  std::vector<Req*> slot_req;
  double* dE = nullptr;       // [items][dd]
  ItemScal* mask = nullptr;   // [items]
  double* ebuf = nullptr;     // one slot's strain on the quadrature grid [dd][dd][nQ]
  size_t bytes = 0;
  std::vector<ItemScal> h_outer, h_inner, h_mask;
  int live() const {
    int n = 0;
    for (Req* r : slot_req) n += (r != nullptr);
    return n;
  }
  ~SizeClass() {
    if (dE) (void)hipFree(dE);
    if (mask) (void)hipFree(mask);
    if (ebuf) (void)hipFree(ebuf);
    delete eng;
  }
};

static double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

static bool same_class(const CellImpl* e, const CellImpl* c) {
  if (e->dd != c->dd || e->scheme != c->scheme || e->kind != c->kind || e->nA != c->nA) return false;
  for (int a = 0; a < 3; ++a)
    if (e->N[a] != c->N[a] || e->Q[a] != c->Q[a] || e->Y[a] != c->Y[a]) return false;
  return e->device == c->device;
}

// device bytes of one slot (d items) and of a class's fixed part
static void footprint(const CellImpl* c, size_t* per_slot, size_t* fixed) {
  const int P = partial_slots(c);
  const size_t w64 = 5 * sizeof(cpx<double>) * c->S + 2 * sizeof(cpx<double>) * c->dd * c->Xe +
                     2 * sizeof(double) * P + sizeof(ItemScal);
  const size_t w32 = 5 * sizeof(cpx<float>) * c->S + 2 * sizeof(cpx<float>) * c->dd * c->Xe +
                     2 * sizeof(double) * P + sizeof(ItemScal);
  *per_slot = (size_t)c->nA * c->nQ * (sizeof(double) + sizeof(float)) +
              (size_t)c->dd * (w64 + w32 + sizeof(ItemScal) + 3 * sizeof(double));
  *fixed = sizeof(double) * (size_t)c->dd * c->dd * c->nQ + sizeof(double) * kQuadScratch;
}

}  // namespace hom

using namespace hom;

struct hom_server {
  size_t budget = 0, used = 0;
  hom_options opt{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  std::deque<Req*> queue;
  std::map<uint64_t, Req*> reqs;
  uint64_t next = 1;
  std::vector<SizeClass*> classes;
  std::thread worker;
  std::chrono::steady_clock::time_point t0;
  hipError_t error = hipSuccess;

  void run();
  hipError_t admit_pending();
  SizeClass* make_class(const CellImpl* like, size_t free_bytes);
  hipError_t admit(SizeClass* k, std::vector<std::pair<int, Req*>>& adm);
  hipError_t tick(std::vector<SizeClass*>& busy);
  hipError_t refine_and_retire(SizeClass* k);
  hipError_t retire(SizeClass* k, int s);
  void finish(Req* r, int status);
};

SizeClass* hom_server::make_class(const CellImpl* like, size_t free_bytes) {
  size_t per_slot = 0, fixed = 0;
  footprint(like, &per_slot, &fixed);
  if (per_slot + fixed > free_bytes) return nullptr;
  const int max_slots = 16;
  int slots = (int)std::min<size_t>(max_slots, (free_bytes - fixed) / per_slot);
  if (slots < 1) return nullptr;
  SizeClass* k = new SizeClass();
  CellImpl* e = new CellImpl();
  e->device = like->device;
  e->d = like->dd;
  e->dd = like->dd;
  e->scheme = like->scheme;
  e->kind = like->kind;
  e->nA = like->nA;
  for (int a = 0; a < 3; ++a) {
    e->N[a] = like->N[a];
    e->Q[a] = like->Q[a];
    e->Y[a] = like->Y[a];
  }
  e->opt = opt;
  k->eng = e;
  k->slots = slots;
  k->dd = e->dd;
  k->items = slots * e->dd;
  k->slot_req.assign(slots, nullptr);
  hipError_t err = hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking);
  if (err == hipSuccess) err = cell_setup(e);
  const size_t nAd = (size_t)e->nA * e->nQ;
  e->A_group = e->dd;
  e->A_block = (long)nAd;
  if (err == hipSuccess) err = hipMalloc(&e->A64, sizeof(double) * nAd * slots);
  if (err == hipSuccess) err = hipMalloc(&e->A32, sizeof(float) * nAd * slots);
  if (err == hipSuccess) err = ensure_work(e, k->items, true);
  if (err == hipSuccess) err = hipMalloc(&k->dE, sizeof(double) * k->items * k->dd);
  if (err == hipSuccess) err = hipMalloc(&k->mask, sizeof(ItemScal) * k->items);
  if (err == hipSuccess) err = hipMalloc(&k->ebuf, sizeof(double) * (size_t)k->dd * k->dd * e->nQ);
  if (err == hipSuccess && !e->quad) err = hipMalloc(&e->quad, sizeof(double) * kQuadScratch);
  // every item starts inactive
  if (err == hipSuccess) err = launch_set_scal(e->w64.sc, k->items, 1.0, 0, 0, e->stream);
  if (err == hipSuccess) err = launch_set_scal(e->w32.sc, k->items, 1.0, 0, 0, e->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
  if (err != hipSuccess) {
    delete k;
    error = err;
    return nullptr;
  }
  k->bytes = per_slot * slots + fixed;
  k->h_outer.resize(k->items);
  k->h_inner.resize(k->items);
  k->h_mask.resize(k->items);
  return k;
}

void hom_server::finish(Req* r, int status) {
  std::lock_guard<std::mutex> lk(mu);
  r->status = status;
  r->t_done = now_s(t0);
  r->info.seconds = r->t_done - r->t_admit;
  r->done = true;
}

hipError_t hom_server::admit(SizeClass* k, std::vector<std::pair<int, Req*>>& adm) {
  CellImpl* e = k->eng;
  hipError_t err = hipSuccess;
  const int P = partial_slots(e);
  const int ub = update_blocks(e->S);
  const int dd = k->dd;
  std::vector<ItemScal>& m = k->h_mask;
  for (auto& q : m) q = ItemScal{};
  std::vector<double> hE(dd * dd);
  for (auto& sr : adm) {
    const int s = sr.first;
    Req* r = sr.second;
    const size_t nAd = (size_t)e->nA * e->nQ;
    // coefficient block of the slot (the request's cell holds FP64 and FP32 copies)
    err = hipMemcpyAsync(e->A64 + nAd * s, r->cell->A64, sizeof(double) * nAd,
                         hipMemcpyDeviceToDevice, e->stream);
    if (err == hipSuccess)
      err = hipMemcpyAsync(e->A32 + nAd * s, r->cell->A32, sizeof(float) * nAd,
                           hipMemcpyDeviceToDevice, e->stream);
    std::fill(hE.begin(), hE.end(), 0.0);
    for (int l = 0; l < r->L; ++l)
      for (int a = 0; a < r->cell->d; ++a) hE[l * dd + a] = r->E[(size_t)l * r->cell->d + a];
    if (err == hipSuccess)
      err = hipMemcpyAsync(k->dE + (size_t)s * dd * dd, hE.data(), sizeof(double) * dd * dd,
                           hipMemcpyHostToDevice, e->stream);
    std::vector<ItemScal> outer(dd);
    for (int l = 0; l < dd; ++l) {
      outer[l] = ItemScal{};
      outer[l].tol = r->tol;
      outer[l].max_iter = opt.max_outer;
      outer[l].active = (l < r->L) ? 1 : 0;
      outer[l].conv = (l < r->L) ? 0 : 1;
      m[(size_t)s * dd + l].active = (l < r->L) ? 1 : 0;
    }
    if (err == hipSuccess)
      err = hipMemcpyAsync(e->w64.sc + (size_t)s * dd, outer.data(), sizeof(ItemScal) * dd,
                           hipMemcpyHostToDevice, e->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(e->stream);  // host buffers are locals
    if (err != hipSuccess) return err;
    k->slot_req[s] = r;
    r->slot = s;
    r->inner_sum.assign(r->L, 0);
    {
      std::lock_guard<std::mutex> lk(mu);
      r->t_admit = now_s(t0);
    }
  }
  err = hipMemcpyAsync(k->mask, m.data(), sizeof(ItemScal) * k->items, hipMemcpyHostToDevice,
                       e->stream);
  // FP64 right-hand side, outer initialisation and the first inner start of the new items
  Work<double>& w = e->w64;
  Work<float>& w32 = e->w32;
  if (err == hipSuccess) err = pipe_rhs<double>(e, w, k->items, k->dE, k->mask);
  if (err == hipSuccess)
    err = launch_outer_check(w.sc, w.part, P, project_tiles<double>(e), k->items, 1, e->stream,
                             k->mask);
  if (err == hipSuccess)
    err = launch_inner_start(w.r, w32.r, w32.p, w32.x, e->S, e->S, e->H, scalar_n0(e), w.sc, w32.sc,
                             opt.max_iter, 0, w32.part, P, ub, k->items, e->stream, k->mask);
  if (err == hipSuccess)
    err = launch_inner_init(w32.sc, w32.part, P, ub, k->items, w.sc, opt.inner_tol, kTolSafety,
                            e->stream, k->mask);
  if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
  return err;
}

hipError_t hom_server::admit_pending() {
  std::vector<Req*> pending;
  {
    std::lock_guard<std::mutex> lk(mu);
    pending.assign(queue.begin(), queue.end());
  }
  std::map<SizeClass*, std::vector<std::pair<int, Req*>>> adm;
  std::vector<Req*> admitted;
  for (Req* r : pending) {
    SizeClass* k = nullptr;
    for (SizeClass* c : classes)
      if (same_class(c->eng, r->cell)) k = c;
    if (!k) {
      // free idle classes of other shapes if memory is short
      size_t per_slot = 0, fixed = 0;
      footprint(r->cell, &per_slot, &fixed);
      if (used + per_slot + fixed > budget) {
        for (size_t i = 0; i < classes.size();) {
          if (classes[i]->live() == 0 && adm.find(classes[i]) == adm.end()) {
            used -= classes[i]->bytes;
            (void)hipStreamSynchronize(classes[i]->eng->stream);
            delete classes[i];
            classes.erase(classes.begin() + (long)i);
          } else {
            ++i;
          }
        }
      }
      if (used + per_slot + fixed > budget) continue;  // waits for memory
      k = make_class(r->cell, budget - used);
      if (!k) {
        if (error != hipSuccess) return error;
        continue;
      }
      classes.push_back(k);
      used += k->bytes;
    }
    int s = -1;
    std::vector<std::pair<int, Req*>>& a = adm[k];
    for (int i = 0; i < k->slots && s < 0; ++i) {
      bool taken = (k->slot_req[i] != nullptr);
      for (auto& p : a) taken = taken || (p.first == i);
      if (!taken) s = i;
    }
    if (s < 0) continue;  // class full: stays queued
    a.push_back({s, r});
    admitted.push_back(r);
  }
  if (!admitted.empty()) {
    std::lock_guard<std::mutex> lk(mu);
    for (Req* r : admitted) queue.erase(std::find(queue.begin(), queue.end(), r));
  }
  for (auto& kv : adm) {
    if (kv.second.empty()) continue;
    hipError_t e = admit(kv.first, kv.second);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t hom_server::retire(SizeClass* k, int s) {
  CellImpl* e = k->eng;
  Req* r = k->slot_req[s];
  const int dd = k->dd, L = r->L;
  const int P = partial_slots(e);
  hipError_t err;
  Work<double> v = work_view(e->w64, s * dd, e->S, e->Xe, dd, P);
  // FP64 strain of the slot's load cases on the quadrature grid, then W and J
  err = pipe_synth(e, v, L, v.x, k->dE + (size_t)s * dd * dd, true, k->ebuf);
  const double* A = e->A64 + (size_t)e->A_block * s;
  const int blocks = (int)std::min<long>(kQuadBlocks, (e->nQ + kThreads - 1) / kThreads);
  std::vector<double> hW((size_t)L * L, 0.0), hJ((size_t)L * dd, 0.0);
  for (int l0 = 0; l0 < L && err == hipSuccess; l0 += 3) {
    const int nl = std::min(3, L - l0);
    for (int m0 = 0; m0 < L && err == hipSuccess; m0 += 3) {
      const int nm = std::min(3, L - m0);
      err = launch_quad(k->ebuf, (long)dd * e->nQ, e->nQ, A, e->nQ, e->kind, dd, e->nQ, l0, nl,
                        m0, nm, e->quad, blocks, e->stream);
      double* outp = e->quad + (size_t)kQuadBlocks * kQuadSlots;
      if (err == hipSuccess)
        err = launch_quad_final(e->quad, blocks, nl, nm, dd, e->nQ, outp, e->stream);
      double h[kQuadSlots];
      if (err == hipSuccess)
        err = hipMemcpyAsync(h, outp, sizeof(h), hipMemcpyDeviceToHost, e->stream);
      if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
      if (err != hipSuccess) break;
      for (int l = 0; l < nl; ++l)
        for (int m = 0; m < nm; ++m) hW[(size_t)(l0 + l) * L + m0 + m] = h[l * 3 + m];
      if (l0 == 0)
        for (int m = 0; m < nm; ++m)
          for (int a = 0; a < dd; ++a) hJ[(size_t)(m0 + m) * dd + a] = h[9 + m * dd + a];
    }
  }
  if (err != hipSuccess) return err;
  int status = HOM_OK, it_in = 0, it_out = 0;
  double relres = 0.0;
  for (int l = 0; l < L; ++l) {
    const ItemScal& o = k->h_outer[(size_t)s * dd + l];
    it_out = std::max(it_out, o.iters);
    it_in = std::max(it_in, r->inner_sum[l]);
    relres = std::max(relres, o.rho0 > 0 ? std::sqrt(o.rho / o.rho0) : 0.0);
    if (o.status == -5) status = HOM_EBREAKDOWN;
    else if (!o.conv && status == HOM_OK) status = HOM_ENOTCONV;
  }
  const int d = r->cell->d;
  r->W = hW;
  r->J.assign((size_t)L * d, 0.0);
  for (int l = 0; l < L; ++l)
    for (int a = 0; a < d; ++a) r->J[(size_t)l * d + a] = hJ[(size_t)l * dd + a];
  r->info.iters_inner = it_in;
  r->info.iters_outer = it_out;
  r->info.rel_resid_true = relres;
  r->info.rho_A = r->cell->rhoA;
  k->slot_req[s] = nullptr;
  finish(r, status);
  return hipSuccess;
}

hipError_t hom_server::refine_and_retire(SizeClass* k) {
  CellImpl* e = k->eng;
  // the flags come back through the engine's pinned staging: [outer][inner][mask]
  const size_t b = sizeof(ItemScal) * k->items;
  void* hp = nullptr;
  hipError_t err = pinned(e, 3 * b, &hp);
  if (err == hipSuccess) err = hipMemcpyAsync(hp, e->w64.sc, b, hipMemcpyDeviceToHost, e->stream);
  if (err == hipSuccess)
    err = hipMemcpyAsync((char*)hp + b, e->w32.sc, b, hipMemcpyDeviceToHost, e->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
  if (err != hipSuccess) return err;
  std::memcpy(k->h_outer.data(), hp, b);
  std::memcpy(k->h_inner.data(), (char*)hp + b, b);
  const int dd = k->dd;
  // retire slots whose load cases all stopped
  for (int s = 0; s < k->slots; ++s) {
    Req* r = k->slot_req[s];
    if (!r) continue;
    bool all_done = true;
    for (int l = 0; l < r->L; ++l) all_done = all_done && !k->h_outer[(size_t)s * dd + l].active;
    if (all_done && (err = retire(k, s)) != hipSuccess) return err;
  }
  // residual replacement for items whose recursion stopped (its residual
  // fell by the inner tolerance, or budget or breakdown)
  bool any = false;
  for (int i = 0; i < k->items; ++i) {
    ItemScal& m = k->h_mask[i];
    m = ItemScal{};
    const Req* r = k->slot_req[i / dd];
    if (!r || (i % dd) >= r->L) continue;
    if (k->h_outer[i].active && !k->h_inner[i].active) {
      m.active = 1;
      any = true;
      k->slot_req[i / dd]->inner_sum[i % dd] = k->h_inner[i].iters;
      if (k->h_inner[i].status == -5) k->h_outer[i].status = -5;
    }
  }
  if (!any) return hipSuccess;
  const int P = partial_slots(e);
  const int ub = update_blocks(e->S);
  Work<double>& w = e->w64;
  Work<float>& w32 = e->w32;
  // the mask region of the staging is not written again before this copy has
  // run: the next write follows the next read-back, which synchronises
  if ((err = pinned(e, 3 * b, &hp)) != hipSuccess) return err;   // retiring may not move it; cheap
  std::memcpy((char*)hp + 2 * b, k->h_mask.data(), b);
  err = hipMemcpyAsync(k->mask, (char*)hp + 2 * b, b, hipMemcpyHostToDevice, e->stream);
  if (err == hipSuccess)
    err = launch_inner_accumulate(w.x, w32.x, e->S, e->S, w.sc, ub, k->items, e->stream, k->mask);
  if (err == hipSuccess)
    err = pipe_apply<double>(e, w, k->items, w.x, EPI_RESID, w.r, nullptr, w.b, k->mask,
                             w.part);
  if (err == hipSuccess)
    err = launch_outer_check(w.sc, w.part, P, project_tiles<double>(e), k->items, 0, e->stream,
                             k->mask);
  if (err == hipSuccess)
    err = launch_inner_start(w.r, w32.r, w32.p, w32.x, e->S, e->S, e->H, scalar_n0(e), w.sc, w32.sc,
                             opt.max_iter, 1, w32.part, P, ub, k->items, e->stream, k->mask);
  if (err == hipSuccess)
    err = launch_inner_init(w32.sc, w32.part, P, ub, k->items, w.sc, opt.inner_tol, kTolSafety,
                            e->stream, k->mask);
  if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
  return err;
}

hipError_t hom_server::tick(std::vector<SizeClass*>& busy) {
  // replay every busy class's graph on its own stream first, then collect
  for (SizeClass* k : busy) {
    hipGraphExec_t g = nullptr;
    hipError_t err = cg_graph<float>(k->eng, k->items, std::max(1, opt.check_every), &g);
    if (err == hipSuccess) err = hipGraphLaunch(g, k->eng->stream);
    if (err != hipSuccess) return err;
  }
  for (SizeClass* k : busy) {
    hipError_t err = refine_and_retire(k);
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

void hom_server::run() {
  (void)hipSetDevice(device);
  for (;;) {
    hipError_t err = admit_pending();
    std::vector<SizeClass*> busy;
    for (SizeClass* k : classes)
      if (k->live() > 0) busy.push_back(k);
    if (err == hipSuccess && !busy.empty()) err = tick(busy);
    if (err != hipSuccess) {
      // a device error ends the service: fail every request still open
      std::lock_guard<std::mutex> lk(mu);
      error = err;
      for (auto& kv : reqs)
        if (!kv.second->done) {
          kv.second->status = HOM_EDEVICE;
          kv.second->done = true;
          kv.second->t_done = now_s(t0);
        }
      queue.clear();
      stop = true;
      cv.notify_all();
      return;
    }
    if (busy.empty()) {
      std::unique_lock<std::mutex> lk(mu);
      if (stop && queue.empty()) return;
      cv.wait_for(lk, std::chrono::milliseconds(1), [&] { return stop || !queue.empty(); });
      if (stop && queue.empty()) {
        bool live = false;
        for (SizeClass* k : classes) live = live || k->live() > 0;
        if (!live) return;
      }
    }
  }
}

extern "C" {

hom_status hom_server_create(size_t hbm_budget_bytes, const hom_options* opt, hom_server** out) {
  if (!out || hbm_budget_bytes == 0) return HOM_EINVAL;
  *out = nullptr;
  hom_options o;
  if (opt)
    o = *opt;
  else
    hom_options_default(&o);
  if (o.prec != HOM_MIXED) return HOM_EINVAL;  // the served form is FP32-inner / FP64-refined
  if (o.max_iter < 1 || o.check_every < 1 || o.max_outer < 1) return HOM_EINVAL;
  if (!(o.inner_tol > 0 && o.inner_tol < 1)) return HOM_EINVAL;
  hom_server* s = new (std::nothrow) hom_server();
  if (!s) return HOM_ENOMEM;
  s->budget = hbm_budget_bytes;
  s->opt = o;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return HOM_EDEVICE;
  }
  s->t0 = std::chrono::steady_clock::now();
  s->worker = std::thread([s]() { s->run(); });
  *out = s;
  return HOM_OK;
}

hom_status hom_server_submit(hom_server* s, hom_cell* c, int L, const double* E, double tol,
                             uint64_t* ticket) {
  if (!s || !c || !E || !ticket || L < 1 || !(tol > 0) || !std::isfinite(tol)) return HOM_EINVAL;
  CellImpl* cell = c->impl;
  if (L > cell->dd) return HOM_EINVAL;  // a slot holds at most d load cases
  // size classes batch primal scalar cells only
  if (cell->dual || cell->elastic) return HOM_EINVAL;
  for (int i = 0; i < L * cell->d; ++i)
    if (!std::isfinite(E[i])) return HOM_EINVAL;
  if (cell->device != s->device) return HOM_EINVAL;
  size_t per_slot = 0, fixed = 0;
  footprint(cell, &per_slot, &fixed);
  if (per_slot + fixed > s->budget) return HOM_ENOMEM;
  Req* r = new (std::nothrow) Req();
  if (!r) return HOM_ENOMEM;
  r->cell = cell;
  r->L = L;
  r->E.assign(E, E + (size_t)L * cell->d);
  r->tol = tol;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete r;
      return s->error != hipSuccess ? HOM_EDEVICE : HOM_EINVAL;
    }
    r->ticket = s->next++;
    r->t_submit = now_s(s->t0);
    s->reqs[r->ticket] = r;
    s->queue.push_back(r);
  }
  s->cv.notify_all();
  *ticket = r->ticket;
  return HOM_OK;
}

hom_status hom_server_times(hom_server* s, uint64_t ticket, double* t) {
  if (!s || !t) return HOM_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return HOM_EINVAL;
  if (!it->second->done) return HOM_EBUSY;
  t[0] = it->second->t_submit;
  t[1] = it->second->t_admit;
  t[2] = it->second->t_done;
  return HOM_OK;
}

hom_status hom_server_poll(hom_server* s, uint64_t ticket, double* W, double* J, hom_info* info) {
  if (!s) return HOM_EINVAL;
  Req* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return HOM_EINVAL;
    if (!it->second->done) return HOM_EBUSY;
    r = it->second;
    s->reqs.erase(it);
  }
  if (W && !r->W.empty()) std::memcpy(W, r->W.data(), sizeof(double) * r->W.size());
  if (J && !r->J.empty()) std::memcpy(J, r->J.data(), sizeof(double) * r->J.size());
  if (info) *info = r->info;
  const int st = r->status;
  delete r;
  return (hom_status)st;
}

hom_status hom_server_destroy(hom_server* s) {
  if (!s) return HOM_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  const bool failed = (s->error != hipSuccess);
  for (SizeClass* k : s->classes) {
    (void)hipStreamSynchronize(k->eng->stream);
    delete k;
  }
  for (auto& kv : s->reqs) delete kv.second;
  delete s;
  return failed ? HOM_EDEVICE : HOM_OK;
}

}  // extern "C"

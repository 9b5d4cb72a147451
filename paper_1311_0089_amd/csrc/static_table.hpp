// static_table.hpp -- the transform lengths that get compile-time
// specialised pass kernels, with their launch shapes.
//
// Each entry: FFT length n, trial length (n for GaNi, (n+1)/2 for the doubled
// Ga grid), radix plan (must equal the host planner's factorisation: odd
// radices largest first, then 8, 4, 2; Bluestein grids for primes above 31),
// column tile width W and workgroup size for FP32 and for FP64, and row pairs
// per workgroup for 2 and 3 components.  Shapes keep dynamic LDS <= 66 KiB
// (two or more workgroups per CU; the all-components column tiles may take
// up to a CU's LDS) and each Stockham stage within the per-thread register
// budget (checked at compile time below).
#pragma once
#include "kernel_bodies.hpp"

namespace hom {

template <class T, class SP, int NTRIAL, int W, int NT, bool MF = false, int WPE = 1>
struct RegCol {
  static constexpr int PMAX = (NTRIAL * W + NT - 1) / NT;
  // the column-major expand / project tiles use the padded row length
  static constexpr size_t lds = (size_t)SP::len * odd_rowlen(W) * sizeof(cpx<T>);
  static constexpr size_t lds_rm = (size_t)SP::len * W * sizeof(cpx<T>);
  static_assert(lds <= 150 * 1024, "column tile exceeds the LDS of a CU");
  static_assert(PMAX <= 32, "too many positions per thread");
  RegCol() {
    // expand / project per scalar layout: column-major for 2-D cells,
    // row-major for 3-D cells; the plain passes do not touch scalars
    using P2 = ColStat<SP, NTRIAL, W, NT, 1, MF, WPE>;
    using P3 = ColStat<SP, NTRIAL, W, NT, 2, MF, WPE>;
    add(KK_EXPAND, (const void*)&k_col_expand<T, P2, PMAX>, 2, lds);
    add(KK_PROJECT, (const void*)&k_col_project<T, P2, PMAX>, 2, lds);
    add(KK_EXPAND, (const void*)&k_col_expand<T, P3, PMAX>, 3, lds_rm);
    add(KK_PROJECT, (const void*)&k_col_project<T, P3, PMAX>, 3, lds_rm);
    using P = ColStat<SP, NTRIAL, W, NT, 0, MF, WPE>;
    add(KK_PLAIN_INV, (const void*)&k_col_plain<T, P, +1>, 0, lds_rm);
    add(KK_PLAIN_FWD, (const void*)&k_col_plain<T, P, -1>, 0, lds_rm);
  }
  template <int... Rs>
  static void fill(StaticKernel& k, Rad<Rs...>) {
    const int r[] = {Rs...};
    k.nst = (int)sizeof...(Rs);
    for (int i = 0; i < k.nst; ++i) k.rad[i] = r[i];
  }
  static void add(int kind, const void* fn, int d, size_t lds_bytes) {
    StaticKernel k{};
    k.kind = kind;
    k.esz = (int)sizeof(cpx<T>);
    k.n = SP::n;
    k.ntrial = NTRIAL;
    k.d = d;
    k.fn = fn;
    k.W = W;
    k.NT = NT;
    k.lds = lds_bytes;
    k.len = SP::len;
    k.blue = SP::blue;
    fill(k, typename SP::radices{});
    register_static(k);
  }
};

// axis-0 projection of 3-D cells with every component's tile loaded before
// the first transform (row-major scalars)
template <class T, class SP, int NTRIAL, int W, int NT>
struct RegProjPre {
  static constexpr int PMAX = (NTRIAL * W + NT - 1) / NT;
  static constexpr size_t lds = (size_t)SP::len * W * sizeof(cpx<T>);
  RegProjPre() {
    using P = ColStat<SP, NTRIAL, W, NT, 2, false, 1, true>;
    RegCol<T, SP, NTRIAL, W, NT>::add(KK_PROJECT, (const void*)&k_col_project<T, P, PMAX>, 3, lds);
  }
};

// axis-0 expand and project with all D components of a W-column tile in one
// LDS tile and one transform call (matches cells with D device components)
template <class T, class SP, int NTRIAL, int W, int D, int NT, bool MF = false>
struct RegColCP {
  static constexpr int PMAX = (NTRIAL * W + NT - 1) / NT;
  static constexpr size_t lds =
      (size_t)SP::len * (D == 2 ? odd_rowlen(W * D) : W * D) * sizeof(cpx<T>);
  static_assert(lds <= 150 * 1024, "column tile exceeds the LDS of a CU");
  static_assert(PMAX <= 32, "too many positions per thread");
  RegColCP() {
    using P = ColStatCP<SP, NTRIAL, W, D, NT, MF>;
    add(KK_EXPAND, (const void*)&k_col_expand<T, P, PMAX>);
    add(KK_PROJECT, (const void*)&k_col_project<T, P, PMAX>);
  }
  static void add(int kind, const void* fn) {
    StaticKernel k{};
    k.kind = kind;
    k.esz = (int)sizeof(cpx<T>);
    k.n = SP::n;
    k.ntrial = NTRIAL;
    k.d = D;
    k.fn = fn;
    k.W = W;
    k.NT = NT;
    k.lds = lds;
    k.len = SP::len;
    k.blue = SP::blue;
    RegCol<T, SP, NTRIAL, 1, 256>::fill(k, typename SP::radices{});
    register_static(k);
  }
};

template <class T, class SP, int NTRIAL, int D, int RP, int NT, bool MF = false, bool ILV = false>
struct RegRow {
  static constexpr size_t lds = (size_t)D * RP * SP::len * sizeof(cpx<T>);
  static_assert(lds <= 66 * 1024 + 512, "row tile exceeds the LDS budget");
  RegRow() {
    using P = RowStat<SP, NTRIAL, D, RP, NT, MF, ILV>;
    add(KK_ROW, (const void*)&k_row<T, P, ROW_APPLY>);
    // the FP64 right-hand side and strain synthesis passes of the same shape
    if constexpr (sizeof(T) == 8 && !ILV) {
      add(KK_ROW_CONST, (const void*)&k_row<T, P, ROW_CONST>);
      add(KK_ROW_SYNTH, (const void*)&k_row<T, P, ROW_SYNTH>);
    }
  }
  static void add(int kind, const void* fn) {
    StaticKernel k{};
    k.kind = kind;
    k.esz = (int)sizeof(cpx<T>);
    k.n = SP::n;
    k.ntrial = NTRIAL;
    k.d = D;
    k.fn = fn;
    k.W = RP;
    k.NT = NT;
    k.lds = lds;
    k.len = SP::len;
    k.blue = SP::blue;
    k.ilv = ILV ? 1 : 0;
    RegCol<T, SP, NTRIAL, 1, 256>::fill(k, typename SP::radices{});
    register_static(k);
  }
};

// plain column passes of a two-stage plan with the register pipeline
// (k_col_reg2): one LDS exchange per tile
template <class T, class SP, int NTRIAL, int W, int NT>
struct RegColReg2 {
  static constexpr size_t lds = (size_t)SP::n * W * sizeof(cpx<T>);
  static_assert(lds <= 66 * 1024, "column tile exceeds the LDS budget");
  RegColReg2() {
    add(KK_PLAIN_INV, (const void*)&k_col_reg2<T, SP, NTRIAL, W, NT, +1>);
    add(KK_PLAIN_FWD, (const void*)&k_col_reg2<T, SP, NTRIAL, W, NT, -1>);
  }
  static void add(int kind, const void* fn) { add_kind(kind, 0, lds, fn); }
  static void add_kind(int kind, int d, size_t lds_bytes, const void* fn) {
    StaticKernel k{};
    k.kind = kind;
    k.esz = (int)sizeof(cpx<T>);
    k.n = SP::n;
    k.ntrial = NTRIAL;
    k.d = d;
    k.fn = fn;
    k.W = W;
    k.NT = NT;
    k.lds = lds_bytes;
    k.len = SP::len;
    k.blue = SP::blue;
    RegCol<T, SP, NTRIAL, 1, 256>::fill(k, typename SP::radices{});
    register_static(k);
  }
};

// first-axis expansion and projection of 3-D cells with the register
// pipeline (k_col_expand_r2 / k_col_project_r2), two-stage plans
template <class T, class SP, int NTRIAL, int W, int NT>
struct RegColR2 {
  static constexpr size_t lds = (size_t)SP::n * W * sizeof(cpx<T>);
  static_assert(lds <= 66 * 1024, "column tile exceeds the LDS budget");
  RegColR2() {
    using R = RegColReg2<T, SP, NTRIAL, W, NT>;
    R::add_kind(KK_EXPAND, 3, lds, (const void*)&k_col_expand_r2<T, SP, NTRIAL, W, NT>);
    R::add_kind(KK_PROJECT, 3, lds, (const void*)&k_col_project_r2<T, SP, NTRIAL, W, NT>);
    // the same with two spectra towards the middle-axis passes (k_col_mid2)
    R::add_kind(KK_EXPAND2, 3, lds, (const void*)&k_col_expand_r2<T, SP, NTRIAL, W, NT, true>);
    R::add_kind(KK_PROJECT2, 3, lds, (const void*)&k_col_project_r2<T, SP, NTRIAL, W, NT, true>);
  }
};

// middle-axis passes between the two-spectra first-axis passes
template <class T, class SP, int NTRIAL, int W, int NT>
struct RegMid2 {
  static constexpr size_t lds = (size_t)SP::n * W * sizeof(cpx<T>);
  static_assert(lds <= 66 * 1024, "column tile exceeds the LDS budget");
  RegMid2() {
    using R = RegColReg2<T, SP, NTRIAL, W, NT>;
    R::add_kind(KK_MID2_INV, 0, lds, (const void*)&k_col_mid2<T, SP, NTRIAL, W, NT, +1>);
    R::add_kind(KK_MID2_FWD, 0, lds, (const void*)&k_col_mid2<T, SP, NTRIAL, W, NT, -1>);
  }
};

// 3-D elasticity: expansion of the six Mandel components from the three
// displacement potentials in one register-pipeline pass
template <class T, class SP, int NTRIAL, int W, int NT>
struct RegBExpand {
  static constexpr size_t lds = (size_t)SP::n * W * sizeof(cpx<T>);
  RegBExpand() {
    RegColReg2<T, SP, NTRIAL, W, NT>::add_kind(
        KK_BEXPAND, 6, lds, (const void*)&k_col_bexpand_r2<T, SP, NTRIAL, W, NT>);
  }
};

// last-axis flux pass with IT load cases per workgroup (k_row_multi)
template <class T, class SP, int NTRIAL, int D, int RP, int NT, int IT>
struct RegRowMulti {
  static constexpr size_t lds = (size_t)IT * D * RP * SP::len * sizeof(cpx<T>);
  static_assert(lds <= 66 * 1024 + 512, "row tile exceeds the LDS budget");
  RegRowMulti() {
    StaticKernel k{};
    k.kind = KK_ROW;
    k.esz = (int)sizeof(cpx<T>);
    k.n = SP::n;
    k.ntrial = NTRIAL;
    k.d = D;
    k.fn = (const void*)&k_row_multi<T, RowMulti<SP, NTRIAL, D, RP, NT, IT>>;
    k.W = RP;
    k.NT = NT;
    k.lds = lds;
    k.len = SP::len;
    k.blue = SP::blue;
    k.ipw = IT;
    RegCol<T, SP, NTRIAL, 1, 256>::fill(k, typename SP::radices{});
    register_static(k);
  }
};

// plans
using P1023 = SPlan<1023, 1023, 0, Rad<31, 11, 3>>;
using P255 = SPlan<255, 255, 0, Rad<17, 15>>;
using P127 = SPlan<127, 256, 1, Rad<8, 8, 4>>;
using P63 = SPlan<63, 63, 0, Rad<9, 7>>;
using P31 = SPlan<31, 31, 0, Rad<31>>;
using P15 = SPlan<15, 15, 0, Rad<15>>;
using P253 = SPlan<253, 253, 0, Rad<23, 11>>;
using P125 = SPlan<125, 125, 0, Rad<5, 5, 5>>;
using P61 = SPlan<61, 128, 1, Rad<8, 8, 2>>;
using P29 = SPlan<29, 29, 0, Rad<29>>;
using P509 = SPlan<509, 1024, 1, Rad<8, 8, 8, 2>>;
// Rader plans of the primes above 31 whose n - 1 factors into the radices:
// lines of n + 1 rows, the radices of the (n-1)-point transform
using P127R = SPlan<127, 128, 2, Rad<9, 7, 2>>;
using P61R = SPlan<61, 62, 2, Rad<15, 4>>;

}  // namespace hom

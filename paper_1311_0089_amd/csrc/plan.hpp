// plan.hpp -- host-side FFT planning: factorisation into the radices the
// device code implements, twiddle and Bluestein tables (computed in long
// double, rounded once), launch shapes that respect the LDS and register
// budgets of the device kernels, and a per-device cache of uploaded tables.
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <vector>

#include "fft_device.hpp"

namespace hom {

struct HostPlan {
  FftPlan p;
  std::vector<std::complex<long double>> table;  // all tables, forward convention
};

// radices supported by the device Stockham stages
bool radix_supported(int r);
// Stockham factorisation of n (largest radices first); empty if a prime
// factor above 31 remains.
std::vector<int> factorize(int n);
HostPlan build_plan(int n);

// device copy of a plan's tables in both precisions
struct DevPlan {
  FftPlan p;
  cpx<double>* tw64 = nullptr;
  cpx<float>* tw32 = nullptr;
};
// cached per (device, n); thread safe; tables live until process exit
hipError_t get_dev_plan(int n, const DevPlan** out);

// rounds each thread needs per stage for W lines: must not exceed the
// register budget of the device code (MaxRounds)
bool rounds_fit(const FftPlan& p, int lines, int esize);

// column-tile width W for a pass over len-point lines whose per-thread
// position count is npos_rows * W / 256 (<= 32); 0 if nothing fits
int choose_col_W(const FftPlan& p, int npos_rows, int inner, int esize, size_t lds_budget,
                 size_t* lds_out);
// row pairs per workgroup for the last-axis pass; 0 if nothing fits
int choose_row_RP(const FftPlan& p, int d, long rows, int esize, size_t lds_budget,
                  size_t* lds_out);

}  // namespace hom

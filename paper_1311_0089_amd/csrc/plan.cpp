// plan.cpp -- see plan.hpp.
#include "plan.hpp"

#include <cmath>
#include <map>
#include <mutex>

namespace hom {

static const int kRadices[] = {31, 29, 23, 19, 17, 15, 13, 11, 9, 7, 5, 3, 8, 4, 2};

bool radix_supported(int r) {
  for (int x : kRadices)
    if (x == r) return true;
  return false;
}

std::vector<int> factorize(int n) {
  std::vector<int> f;
  int m = n;
  // odd radices, largest first; 15 (a register 3 x 5 prime-factor butterfly)
  // before 5 and 3, so 255 -> 17 15; 9 before 3 so 27 -> 9 3, 81 -> 9 9
  for (int r : {31, 29, 23, 19, 17, 15, 13, 11, 9, 7, 5, 3}) {
    while (m % r == 0) {
      f.push_back(r);
      m /= r;
    }
  }
  for (int r : {8, 4, 2}) {
    while (m % r == 0) {
      f.push_back(r);
      m /= r;
    }
  }
  if (m != 1) f.clear();
  return f;
}

static std::complex<long double> root(long t, long n) {
  // exp(-2 pi i t / n), t reduced mod n
  t %= n;
  if (t < 0) t += n;
  const long double pi = 3.141592653589793238462643383279502884L;
  const long double a = 2.0L * pi * (long double)t / (long double)n;
  return {std::cos(a), -std::sin(a)};
}

static void stockham_tables(int len, const std::vector<int>& rad, FftPlan& p,
                            std::vector<std::complex<long double>>& tab) {
  p.nst = (int)rad.size();
  long Ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = rad[s];
    p.rad[s] = R;
    p.twoff[s] = (int)tab.size();
    if (Ns > 1)
      for (long k = 0; k < Ns; ++k)
        for (int r = 1; r < R; ++r) tab.push_back(root(r * k, Ns * R));
    Ns *= R;
  }
  (void)len;
}

static bool is_prime(int n) {
  if (n < 2) return false;
  for (int q = 2; (long)q * q <= n; ++q)
    if (n % q == 0) return false;
  return true;
}

// smallest generator of the multiplicative group mod a prime n
static int primitive_root(int n) {
  std::vector<int> f;
  int m = n - 1;
  for (int q = 2; q * q <= m; ++q)
    if (m % q == 0) {
      f.push_back(q);
      while (m % q == 0) m /= q;
    }
  if (m > 1) f.push_back(m);
  for (int g = 2; g < n; ++g) {
    bool ok = true;
    for (int q : f) {
      long r = 1, b = g;
      for (int e = (n - 1) / q; e > 0; e >>= 1, b = b * b % n)
        if (e & 1) r = r * b % n;
      if (r == 1) ok = false;
    }
    if (ok) return g;
  }
  return 0;
}

// Rader (1968): for prime n and a generator g, X_{g^q} = x_0 + sum_p
// x_{g^-p} w^{g^(q-p)}, a cyclic convolution of length L = n - 1 of
// a_p = x_{g^-p} with b_m = w^{g^m}, evaluated as IFFT_L(FFT_L(a) B) with
// B = FFT_L(b) / L; X_0 = x_0 + FFT_L(a)_0.
static void add_rader(int n, HostPlan& h) {
  if (!is_prime(n) || n < 5) return;
  const int L = n - 1;
  const std::vector<int> f = factorize(L);
  if (f.empty() || (int)f.size() > kMaxStages) return;
  const int g = primitive_root(n);
  if (!g) return;
  FftPlan t{};
  h.p.r_off = (int)h.table.size();
  stockham_tables(L, f, t, h.table);
  h.p.r_nst = t.nst;
  for (int s = 0; s < t.nst; ++s) h.p.r_rad[s] = t.rad[s];
  std::vector<long> gp(L);
  gp[0] = 1;
  for (int m = 1; m < L; ++m) gp[m] = gp[m - 1] * g % n;
  for (int sgn = 0; sgn < 2; ++sgn) {
    // sgn 0: forward transform, w = exp(-2 pi i / n); 1: inverse, w = exp(+2 pi i / n)
    (sgn == 0 ? h.p.r_bf : h.p.r_bi) = (int)h.table.size();
    for (long k = 0; k < L; ++k) {
      std::complex<long double> s = {0.0L, 0.0L};
      for (long m = 0; m < L; ++m) s += root(sgn == 0 ? gp[m] : -gp[m], n) * root(m * k, L);
      h.table.push_back(s / (long double)L);
    }
  }
  h.p.r_gidx = (int)h.table.size();
  for (long p = 0; p < L; ++p) h.table.push_back({(long double)gp[(L - p) % L], 0.0L});
  h.p.r_sidx = (int)h.table.size();
  for (long q = 0; q < L; ++q) h.table.push_back({(long double)gp[q], 0.0L});
  h.p.rader = 1;
}

HostPlan build_plan(int n) {
  HostPlan h{};
  h.p.n = n;
  std::vector<int> f = factorize(n);
  if (n == 1 || !f.empty()) {
    h.p.len = n;
    h.p.blue = 0;
    stockham_tables(n, f, h.p, h.table);
    return h;
  }
  // Bluestein: X_k = c_k sum_j (x_j c_j) conj(c)_{k-j}, c_j = exp(-i pi j^2 / n),
  // evaluated as a cyclic convolution of length m >= 2n - 1 (power of two)
  int m = 1;
  while (m < 2 * n - 1) m *= 2;
  h.p.len = m;
  h.p.blue = 1;
  stockham_tables(m, factorize(m), h.p, h.table);
  std::vector<std::complex<long double>> c(n);
  for (long j = 0; j < n; ++j) c[j] = root((j * j) % (2L * n), 2L * n);
  h.p.chirp_off = (int)h.table.size();
  for (long j = 0; j < n; ++j) h.table.push_back(c[j]);
  std::vector<std::complex<long double>> w(m);
  for (long t = 0; t < m; ++t) w[t] = root(t, m);
  for (int sgn = 0; sgn < 2; ++sgn) {
    // sgn 0: forward, b = conj(c); sgn 1: inverse, b = c
    std::vector<std::complex<long double>> b(m, {0.0L, 0.0L});
    for (long j = 0; j < n; ++j) {
      const auto v = sgn == 0 ? std::conj(c[j]) : c[j];
      b[j] = v;
      if (j > 0) b[m - j] = v;
    }
    (sgn == 0 ? h.p.dfwd_off : h.p.dinv_off) = (int)h.table.size();
    for (long k = 0; k < m; ++k) {
      std::complex<long double> s = {0.0L, 0.0L};
      for (long j = 0; j < m; ++j)
        if (b[j] != std::complex<long double>(0.0L, 0.0L)) s += b[j] * w[(k * j) % m];
      h.table.push_back(s / (long double)m);
    }
  }
  add_rader(n, h);
  return h;
}

namespace {
std::mutex g_mu;
std::map<std::pair<int, int>, DevPlan*> g_cache;
}  // namespace

hipError_t get_dev_plan(int n, const DevPlan** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cache.find({dev, n});
  if (it != g_cache.end()) {
    *out = it->second;
    return hipSuccess;
  }
  HostPlan h = build_plan(n);
  DevPlan* d = new DevPlan();
  d->p = h.p;
  const size_t cnt = h.table.size() > 0 ? h.table.size() : 1;
  std::vector<cpx<double>> t64(cnt, cpx<double>{0, 0});
  std::vector<cpx<float>> t32(cnt, cpx<float>{0, 0});
  for (size_t i = 0; i < h.table.size(); ++i) {
    t64[i] = {(double)h.table[i].real(), (double)h.table[i].imag()};
    t32[i] = {(float)h.table[i].real(), (float)h.table[i].imag()};
  }
  e = hipMalloc(&d->tw64, cnt * sizeof(cpx<double>));
  if (e == hipSuccess) e = hipMalloc(&d->tw32, cnt * sizeof(cpx<float>));
  if (e == hipSuccess)
    e = hipMemcpy(d->tw64, t64.data(), cnt * sizeof(cpx<double>), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(d->tw32, t32.data(), cnt * sizeof(cpx<float>), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (d->tw64) (void)hipFree(d->tw64);
    if (d->tw32) (void)hipFree(d->tw32);
    delete d;
    return e;
  }
  g_cache[{dev, n}] = d;
  *out = d;
  return hipSuccess;
}

static int max_rounds(int R, int esize) {
  const int budget = (esize == 8) ? 32 : 24;  // complex elements per thread (float / double)
  const int v = budget / R;
  return v > 0 ? v : 1;
}

bool rounds_fit(const FftPlan& p, int lines, int esize) {
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.rad[s];
    const long total = (long)(p.len / R) * lines;
    const long rounds = (total + 255) / 256;
    if (rounds > max_rounds(R, esize)) return false;
  }
  return true;
}

int choose_col_W(const FftPlan& p, int npos_rows, int inner, int esize, size_t lds_budget,
                 size_t* lds_out) {
  for (int W : {16, 8, 4, 2, 1}) {
    if (W > 1 && W / 2 >= inner) continue;  // do not tile far wider than the data
    const size_t lds = (size_t)p.len * W * esize;
    if (lds > lds_budget) continue;
    if ((long)npos_rows * W > 32L * 256) continue;
    if (!rounds_fit(p, W, esize)) continue;
    *lds_out = lds;
    return W;
  }
  return 0;
}

int choose_row_RP(const FftPlan& p, int d, long rows, int esize, size_t lds_budget,
                  size_t* lds_out) {
  const long pairs = (rows + 1) / 2;
  for (int RP : {8, 4, 2, 1}) {
    if (RP > 1 && RP / 2 >= pairs) continue;
    const size_t lds = (size_t)d * RP * p.len * esize;
    if (lds > lds_budget) continue;
    if (!rounds_fit(p, d * RP, esize)) continue;
    *lds_out = lds;
    return RP;
  }
  return 0;
}

}  // namespace hom

// fft_device.hpp -- workgroup-level FFT of many lines held in LDS (gfx950).
//
// Mixed-radix Stockham autosort (Govindaraju et al., "High performance
// discrete Fourier transforms on graphics processors", SC 2008): a stage of
// radix R and span Ns reads x[j + r n/R], multiplies by exp(s 2 pi i r k /
// (Ns R)) with k = j mod Ns, applies the R-point DFT and writes
// y[(j / Ns) Ns R + k + r Ns]; input and output are in natural order.
// Each stage is done in place: every thread first loads all of its
// butterflies' inputs into registers, the workgroup synchronises, then every
// thread computes and stores.  Odd radices use the symmetric-pair form of the
// R-point DFT, which halves its multiplications.  Lengths with a prime factor
// above 31 go through Bluestein's chirp-z convolution on a power-of-two grid.
//
// The DFT convention is the paper's (Sec. 4.1): s = -1 forward, s = +1
// inverse, no normalisation here (callers scale by 1/n on forward passes).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hom {

template <class T>
struct cpx {
  T x, y;
};

template <class T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.x, -a.y}; }
template <class T>
__device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by S*i
template <int S, class T>
__device__ __forceinline__ cpx<T> mul_si(cpx<T> a) {
  return (S > 0) ? cpx<T>{-a.y, a.x} : cpx<T>{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// compile-time cos / sin of 2 pi t / n with exact quadrant reduction in
// integers and Taylor series on [0, pi/4]
// ---------------------------------------------------------------------------
constexpr double kPiD = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k <= 13; ++k) {
    term = -term * x2 / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k <= 13; ++k) {
    term = -term * x2 / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
constexpr double cos2pi(long t, long n) {
  t %= n;
  if (t < 0) t += n;
  long q = (4 * t) / n, m = 4 * t - q * n;
  double c = 0, s = 0;
  if (2 * m <= n) {
    double a = (kPiD / 2) * double(m) / double(n);
    c = taylor_cos(a);
    s = taylor_sin(a);
  } else {
    double a = (kPiD / 2) * double(n - m) / double(n);
    c = taylor_sin(a);
    s = taylor_cos(a);
  }
  return q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}
constexpr double sin2pi(long t, long n) {
  t %= n;
  if (t < 0) t += n;
  long q = (4 * t) / n, m = 4 * t - q * n;
  double c = 0, s = 0;
  if (2 * m <= n) {
    double a = (kPiD / 2) * double(m) / double(n);
    c = taylor_cos(a);
    s = taylor_sin(a);
  } else {
    double a = (kPiD / 2) * double(n - m) / double(n);
    c = taylor_sin(a);
    s = taylor_cos(a);
  }
  return q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
}

template <int R>
struct RootTable {
  double c[R], s[R];
  constexpr RootTable() : c(), s() {
    for (int t = 0; t < R; ++t) {
      c[t] = cos2pi(t, R);
      s[t] = sin2pi(t, R);
    }
  }
};

// ---------------------------------------------------------------------------
// R-point DFTs in registers, y_k = sum_j v_j exp(S 2 pi i j k / R)
// ---------------------------------------------------------------------------
template <class T, int R, int S>
struct Dft;

template <class T, int S>
struct Dft<T, 2, S> {
  __device__ __forceinline__ static void run(cpx<T>* v) {
    cpx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <class T, int S>
struct Dft<T, 4, S> {
  __device__ __forceinline__ static void run(cpx<T>* v) {
    cpx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    cpx<T> t2 = cadd(v[1], v[3]), t3 = mul_si<S>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[1] = cadd(t1, t3);
    v[2] = csub(t0, t2);
    v[3] = csub(t1, t3);
  }
};

template <class T, int S>
struct Dft<T, 8, S> {
  __device__ __forceinline__ static void run(cpx<T>* v) {
    // decimation in frequency: a_j = v_j + v_{j+4}, b_j = (v_j - v_{j+4}) w8^{S j}
    const T h = T(0.70710678118654752440084436210484903928);
    cpx<T> a[4], b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[j] = cadd(v[j], v[j + 4]);
      b[j] = csub(v[j], v[j + 4]);
    }
    // w8^{S}   = h (1 + S i);  w8^{2S} = S i;  w8^{3S} = h (-1 + S i)
    b[1] = cscale(cadd(b[1], mul_si<S>(b[1])), h);
    b[2] = mul_si<S>(b[2]);
    b[3] = cscale(csub(mul_si<S>(b[3]), b[3]), h);
    Dft<T, 4, S>::run(a);
    Dft<T, 4, S>::run(b);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = a[k];
      v[2 * k + 1] = b[k];
    }
  }
};

// R = 15 by the prime-factor (Good-Thomas) mapping 15 = 3 x 5, which needs
// no twiddles between the two factors: with n = (5 n1 + 3 n2) mod 15 and
// k = (10 k1 + 6 k2) mod 15, y_k = sum_n1 w3^(S n1 k1) sum_n2 w5^(S n2 k2)
// v_n (the indices of the Chinese remainder theorem for the coprime 3, 5)
template <class T, int S>
struct Dft<T, 15, S> {
  __device__ __forceinline__ static void run(cpx<T>* v) {
    cpx<T> y[3][5];
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) {
#pragma unroll
      for (int n2 = 0; n2 < 5; ++n2) y[n1][n2] = v[(5 * n1 + 3 * n2) % 15];
      Dft<T, 5, S>::run(y[n1]);
    }
#pragma unroll
    for (int k2 = 0; k2 < 5; ++k2) {
      cpx<T> z[3] = {y[0][k2], y[1][k2], y[2][k2]};
      Dft<T, 3, S>::run(z);
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) v[(10 * k1 + 6 * k2) % 15] = z[k1];
    }
  }
};

// Odd R: pair j with R - j.  y_0 = v_0 + sum s_j; for k = 1..(R-1)/2,
// a_k = v_0 + sum_j s_j cos(2 pi j k / R), b_k = sum_j d_j sin(2 pi j k / R),
// y_k = a_k + S i b_k, y_{R-k} = a_k - S i b_k, with s_j = v_j + v_{R-j},
// d_j = v_j - v_{R-j}.
template <class T, int R, int S>
struct Dft {
  static_assert(R % 2 == 1 && R >= 3, "odd radix");
  __device__ __forceinline__ static void run(cpx<T>* v) {
    constexpr int H = (R - 1) / 2;
    constexpr RootTable<R> tb{};
    cpx<T> s[H], d[H];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      s[j - 1] = cadd(v[j], v[R - j]);
      d[j - 1] = csub(v[j], v[R - j]);
    }
    cpx<T> y0 = v[0];
#pragma unroll
    for (int j = 0; j < H; ++j) y0 = cadd(y0, s[j]);
    cpx<T> out[R];
    out[0] = y0;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      cpx<T> a = v[0], b = {T(0), T(0)};
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        const T c = T(tb.c[(j * k) % R]);
        const T sn = T(tb.s[(j * k) % R]);
        a.x += s[j - 1].x * c;
        a.y += s[j - 1].y * c;
        b.x += d[j - 1].x * sn;
        b.y += d[j - 1].y * sn;
      }
      cpx<T> ib = mul_si<S>(b);
      out[k] = cadd(a, ib);
      out[R - k] = csub(a, ib);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = out[k];
  }
};

// ---------------------------------------------------------------------------
// plans (host-built, passed by value in kernel arguments)
// ---------------------------------------------------------------------------
constexpr int kMaxStages = 8;

struct FftPlan {
  int n;                    // logical transform length
  int len;                  // length held in LDS per line (n, or the Bluestein grid m)
  int nst;                  // stages of the len-point Stockham transform
  int rad[kMaxStages];      // radices
  int twoff[kMaxStages];    // offsets of the per-stage twiddle tables
  int blue;                 // 1 if Bluestein is used
  int chirp_off;            // offset of the n chirp values exp(-i pi j^2 / n)
  int dfwd_off;             // offset of D_- = FFT_m(conj chirp) / m   (forward)
  int dinv_off;             // offset of D_+ = FFT_m(chirp) / m        (inverse)
  // Rader's algorithm for a prime n whose n - 1 factors into the Stockham
  // radices (used by the compile-time kernels that choose it; the generic
  // kernels keep Bluestein): tables after the Bluestein ones
  int rader;                // 1 if present
  int r_nst;                // stages of the (n-1)-point Stockham transform
  int r_rad[kMaxStages];    // its radices
  int r_off;                // its twiddles
  int r_bf, r_bi;           // B_-/+ = FFT_{n-1}(b) / (n-1), b_m = exp(-/+ 2 pi i g^m / n)
  int r_gidx, r_sidx;       // g^-p mod n and g^q mod n (as the real parts)
};

// Maximum complex values a thread holds during one stage.
template <class T>
struct RegBudget {
  static constexpr int kElems = (sizeof(T) == 4) ? 32 : 24;
};
template <class T, int R>
struct MaxRounds {
  static constexpr int v = (RegBudget<T>::kElems / R) > 0 ? (RegBudget<T>::kElems / R) : 1;
};

// Layout of W lines in LDS: element (w, i) lives at buf[w * ls + i * es].
// wfast: consecutive threads take consecutive lines (column tiles, es = W,
// ls = 1); otherwise consecutive butterflies of a line (rows, es = 1).
struct LdsLines {
  int W, ls, es;
  bool wfast;
};

template <class T, int R, int S>
__device__ __forceinline__ void stockham_stage(cpx<T>* buf, int len, const LdsLines& L, int Ns,
                                               const cpx<T>* __restrict__ tw) {
  constexpr int MB = MaxRounds<T, R>::v;
  const int nb = len / R;
  const int total = nb * L.W;
  const int T_ = blockDim.x;
  cpx<T> v[MB][R];
  int obase[MB];
#pragma unroll
  for (int it = 0; it < MB; ++it) {
    const int f = threadIdx.x + it * T_;
    obase[it] = -1;
    if (f < total) {
      int w, j;
      if (L.wfast) {
        w = f % L.W;
        j = f / L.W;
      } else {
        j = f % nb;
        w = f / nb;
      }
      const cpx<T>* line = buf + w * L.ls;
      const int k = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = line[(j + r * nb) * L.es];
      if (Ns > 1) {
        const cpx<T>* t = tw + k * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w_ = t[r - 1];
          if (S > 0) w_.y = -w_.y;
          v[it][r] = cmul(v[it][r], w_);
        }
      }
      obase[it] = w * L.ls + ((j / Ns) * Ns * R + k) * L.es;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MB; ++it) {
    if (obase[it] >= 0) {
      Dft<T, R, S>::run(v[it]);
      cpx<T>* o = buf + obase[it];
#pragma unroll
      for (int r = 0; r < R; ++r) o[r * Ns * L.es] = v[it][r];
    }
  }
  __syncthreads();
}

// Stockham transform of length len on all lines (no Bluestein), sign S.
// tw: twiddles of the forward transform, tw[off + k (R-1) + r - 1] =
// exp(-2 pi i r k / (Ns R)); the inverse uses their conjugates.
template <class T, int S>
__device__ void stockham(cpx<T>* buf, const FftPlan& P, const LdsLines& L,
                         const cpx<T>* __restrict__ tw) {
  int Ns = 1;
  for (int s = 0; s < P.nst; ++s) {
    const int R = P.rad[s];
    const cpx<T>* t = tw + P.twoff[s];
    switch (R) {
      case 2: stockham_stage<T, 2, S>(buf, P.len, L, Ns, t); break;
      case 3: stockham_stage<T, 3, S>(buf, P.len, L, Ns, t); break;
      case 4: stockham_stage<T, 4, S>(buf, P.len, L, Ns, t); break;
      case 5: stockham_stage<T, 5, S>(buf, P.len, L, Ns, t); break;
      case 7: stockham_stage<T, 7, S>(buf, P.len, L, Ns, t); break;
      case 8: stockham_stage<T, 8, S>(buf, P.len, L, Ns, t); break;
      case 9: stockham_stage<T, 9, S>(buf, P.len, L, Ns, t); break;
      case 11: stockham_stage<T, 11, S>(buf, P.len, L, Ns, t); break;
      case 13: stockham_stage<T, 13, S>(buf, P.len, L, Ns, t); break;
      case 15: stockham_stage<T, 15, S>(buf, P.len, L, Ns, t); break;
      case 17: stockham_stage<T, 17, S>(buf, P.len, L, Ns, t); break;
      case 19: stockham_stage<T, 19, S>(buf, P.len, L, Ns, t); break;
      case 23: stockham_stage<T, 23, S>(buf, P.len, L, Ns, t); break;
      case 29: stockham_stage<T, 29, S>(buf, P.len, L, Ns, t); break;
      case 31: stockham_stage<T, 31, S>(buf, P.len, L, Ns, t); break;
      default: break;  // the host planner only emits the radices above
    }
    Ns *= R;
  }
}

// Full n-point DFT of sign S on every line.  For Bluestein plans the lines
// must have room for len = m entries; entries n..m-1 are overwritten.
template <class T, int S>
__device__ void line_fft(cpx<T>* buf, const FftPlan& P, const LdsLines& L,
                         const cpx<T>* __restrict__ tw) {
  if (!P.blue) {
    stockham<T, S>(buf, P, L, tw);
    return;
  }
  const int n = P.n, m = P.len;
  const cpx<T>* chirp = tw + P.chirp_off;
  const cpx<T>* D = tw + (S < 0 ? P.dfwd_off : P.dinv_off);
  const int total = m * L.W;
  // a_j = x_j c_j (c = chirp of sign S), zero for j >= n
  for (int f = threadIdx.x; f < total; f += blockDim.x) {
    int w, j;
    if (L.wfast) { w = f % L.W; j = f / L.W; } else { j = f % m; w = f / m; }
    cpx<T>* e = buf + w * L.ls + j * L.es;
    if (j < n) {
      cpx<T> c = chirp[j];
      if (S > 0) c.y = -c.y;
      *e = cmul(*e, c);
    } else {
      *e = cpx<T>{T(0), T(0)};
    }
  }
  __syncthreads();
  stockham<T, -1>(buf, P, L, tw);
  for (int f = threadIdx.x; f < total; f += blockDim.x) {
    int w, j;
    if (L.wfast) { w = f % L.W; j = f / L.W; } else { j = f % m; w = f / m; }
    cpx<T>* e = buf + w * L.ls + j * L.es;
    *e = cmul(*e, D[j]);
  }
  __syncthreads();
  stockham<T, +1>(buf, P, L, tw);
  for (int f = threadIdx.x; f < n * L.W; f += blockDim.x) {
    int w, j;
    if (L.wfast) { w = f % L.W; j = f / L.W; } else { j = f % n; w = f / n; }
    cpx<T>* e = buf + w * L.ls + j * L.es;
    cpx<T> c = chirp[j];
    if (S > 0) c.y = -c.y;
    *e = cmul(*e, c);
  }
  __syncthreads();
}

}  // namespace hom

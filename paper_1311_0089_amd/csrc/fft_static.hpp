// fft_static.hpp -- compile-time specialised LDS FFT (same algorithm as
// fft_device.hpp: mixed-radix Stockham autosort, Bluestein above radix 31)
// with the radix sequence, spans, line count, layout and workgroup size all
// known to the compiler, so index arithmetic folds to constants and each
// stage holds exactly the registers it needs.
#pragma once
#include "fft_device.hpp"

namespace hom {

template <int... Rs>
struct Rad {};

// N_: transform length; LEN_: LDS line length (N_, or the Bluestein grid);
// BLUE_: Bluestein; R_: radices of the LEN_-point Stockham transform.
template <int N_, int LEN_, int BLUE_, class R_>
struct SPlan {
  static constexpr int n = N_, len = LEN_, blue = BLUE_;
  using radices = R_;
};

// twiddle-table size of a radix list (same layout as the host planner)
template <int Ns, int... Rs>
struct TwSize;
template <int Ns>
struct TwSize<Ns> {
  static constexpr int v = 0;
};
template <int Ns, int R, int... Rest>
struct TwSize<Ns, R, Rest...> {
  static constexpr int v = (Ns > 1 ? Ns * (R - 1) : 0) + TwSize<Ns * R, Rest...>::v;
};
template <class R_>
struct TwSizeOf;
template <int... Rs>
struct TwSizeOf<Rad<Rs...>> {
  static constexpr int v = TwSize<1, Rs...>::v;
};

// max over stages of (rounds per thread) x radix: complex values a thread holds
template <int LEN, int W, int NT, int... Rs>
struct StageRegs;
template <int LEN, int W, int NT>
struct StageRegs<LEN, W, NT> {
  static constexpr int v = 0;
};
template <int LEN, int W, int NT, int R, int... Rest>
struct StageRegs<LEN, W, NT, R, Rest...> {
  static constexpr int here = (((LEN / R) * W + NT - 1) / NT) * R;
  static constexpr int rest = StageRegs<LEN, W, NT, Rest...>::v;
  static constexpr int v = here > rest ? here : rest;
};

template <class T, int R, int S, int LEN, int W, bool WF, int LS, int ES, int Ns, int NT>
__device__ __forceinline__ void sstage(cpx<T>* buf, const cpx<T>* __restrict__ tw) {
  constexpr int nb = LEN / R;
  constexpr int total = nb * W;
  constexpr int MB = (total + NT - 1) / NT;
  constexpr int NTW = (Ns > 1) ? R - 1 : 1;
  // butterfly f of this thread's round it: line w, index j in the line.  Every
  // read is unconditional (a thread past the last butterfly repeats its reads
  // and writes nothing), so the twiddle loads of all rounds go out together
  // instead of each being waited for under its own branch.
  auto at = [](int it, int& w, int& j) __attribute__((always_inline)) {
    const int f0 = threadIdx.x + it * NT;
    const int f = ((total % NT) == 0) ? f0 : min(f0, total - 1);
    if (WF) {
      w = f % W;
      j = f / W;
    } else {
      j = f % nb;
      w = f / nb;
    }
    return ((total % NT) == 0) || f0 < total;
  };
  cpx<T> v[MB][R];
  cpx<T> t[MB][NTW];
  int ob[MB];
  if (Ns > 1) {
#pragma unroll
    for (int it = 0; it < MB; ++it) {
      int w, j;
      at(it, w, j);
      const cpx<T>* tk = tw + (j % Ns) * (R - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) t[it][r - 1] = tk[r - 1];
    }
  }
#pragma unroll
  for (int it = 0; it < MB; ++it) {
    int w, j;
    const bool live = at(it, w, j);
    const cpx<T>* line = buf + w * LS;
#pragma unroll
    for (int r = 0; r < R; ++r) v[it][r] = line[(j + r * nb) * ES];
    const int k = j % Ns;
    ob[it] = live ? w * LS + ((j / Ns) * Ns * R + k) * ES : -1;
  }
  if (Ns > 1) {
#pragma unroll
    for (int it = 0; it < MB; ++it) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cpx<T> w_ = t[it][r - 1];
        if (S > 0) w_.y = -w_.y;
        v[it][r] = cmul(v[it][r], w_);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MB; ++it) {
    if (ob[it] >= 0) {
      Dft<T, R, S>::run(v[it]);
      cpx<T>* o = buf + ob[it];
#pragma unroll
      for (int r = 0; r < R; ++r) o[r * Ns * ES] = v[it][r];
    }
  }
  __syncthreads();
}

// cos / sin (2 pi t / R) rounded once to FP32 (the values the register DFT of
// the same radix uses), as a device table for per-lane lookups
template <int R>
struct MfmaRoots {
  float c[R], s[R];
  constexpr MfmaRoots() : c(), s() {
    for (int t = 0; t < R; ++t) {
      c[t] = float(cos2pi(t, R));
      s[t] = float(sin2pi(t, R));
    }
  }
};
template <int R>
__device__ constexpr MfmaRoots<R> kMfmaRoots{};

typedef float f32x4 __attribute__((ext_vector_type(4)));

// First Stockham stage (Ns = 1, no twiddles) of an odd radix R <= 31 on the
// matrix cores.  With s_0 = v_0, s_j = v_j + v_{R-j}, d_j = v_j - v_{R-j}
// (j = 1..H, H = (R-1)/2, zero past H), the butterfly outputs are
// y_0 = P_0, y_k = P_k + S i Q_k and y_{R-k} = P_k - S i Q_k (k = 1..H), where
// P = C s and Q = Sn d with C_kj = cos(2 pi jk/R), Sn_kj = sin(2 pi jk/R),
// k, j = 0..15 -- the symmetric-pair form of the register DFT, as products of
// 16x16 constant matrices with 16 butterflies at a time (the columns).  Each
// 16-butterfly column block takes KC steps of v_mfma_f32_16x16x4_f32 per real
// part (P re, P im, Q re, Q im); lane l supplies row (l mod 16) of the
// constant and column (l mod 16) of the data at K index l / 16, and holds
// rows 4 (l / 16) .. 4 (l / 16) + 3 of column l mod 16 of the result.
template <int R, int S, int LEN, int W, bool WF, int LS, int ES, int NT>
__device__ __forceinline__ void mstage(cpx<float>* buf) {
  constexpr int H = (R - 1) / 2;
  constexpr int KC = (H + 1 + 3) / 4;
  constexpr int nb = LEN / R, total = nb * W;
  constexpr int NCB = (total + 15) / 16;
  constexpr int NW = NT / 64;
  constexpr int CPW = (NCB + NW - 1) / NW;
  static_assert(NT % 64 == 0 && H + 1 <= 16, "matrix-core stage shape");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 15, g = lane >> 4;
  float ca[KC], sa[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const int j = 4 * c + g, t = (n * j) % R;
    ca[c] = (j <= H) ? kMfmaRoots<R>.c[t] : 0.f;
    sa[c] = (j <= H) ? kMfmaRoots<R>.s[t] : 0.f;
  }
  auto at = [](int f, int& w, int& b) __attribute__((always_inline)) {
    if (WF) {
      w = f % W;
      b = f / W;
    } else {
      b = f % nb;
      w = f / nb;
    }
  };
  f32x4 pr[CPW], pi[CPW], qr[CPW], qi[CPW];
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    pr[q] = pi[q] = qr[q] = qi[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int cb = wave + q * NW;
    if (cb < NCB) {   // the same for every lane of the wave
      int w, b;
      at(min(cb * 16 + n, total - 1), w, b);
      const cpx<float>* line = buf + w * LS;
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        const int j = 4 * c + g;
        float sr = 0.f, si = 0.f, dr = 0.f, di = 0.f;
        if (j == 0) {
          const cpx<float> v0 = line[b * ES];
          sr = v0.x;
          si = v0.y;
        } else if (j <= H) {
          const cpx<float> x = line[(b + j * nb) * ES], y = line[(b + (R - j) * nb) * ES];
          sr = x.x + y.x;
          si = x.y + y.y;
          dr = x.x - y.x;
          di = x.y - y.y;
        }
        pr[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[c], sr, pr[q], 0, 0, 0);
        pi[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[c], si, pi[q], 0, 0, 0);
        qr[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(sa[c], dr, qr[q], 0, 0, 0);
        qi[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(sa[c], di, qi[q], 0, 0, 0);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int cb = wave + q * NW, f = cb * 16 + n;
    if (cb < NCB && f < total) {
      int w, b;
      at(f, w, b);
      cpx<float>* o = buf + w * LS + b * R * ES;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = 4 * g + r;
        const float Pr = pr[q][r], Pi = pi[q][r], Qr = qr[q][r], Qi = qi[q][r];
        if (k == 0) {
          o[0] = cpx<float>{Pr, Pi};
        } else if (k <= H) {
          o[k * ES] = cpx<float>{Pr - float(S) * Qi, Pi + float(S) * Qr};
          o[(R - k) * ES] = cpx<float>{Pr + float(S) * Qi, Pi - float(S) * Qr};
        }
      }
    }
  }
  __syncthreads();
}

// the matrix-core form serves the first stage of FP32 transforms with an odd
// radix of 17 or more (where the register DFT's quadratic cost dominates)
template <class T, int R, int Ns, bool MF>
constexpr bool use_mstage() {
  return MF && Ns == 1 && R % 2 == 1 && R >= 17 && R <= 31 && sizeof(T) == 4;
}

template <class T, int S, int LEN, int W, bool WF, int LS, int ES, int NT, bool MF, int Ns, int OFF,
          int... Rs>
struct SStages;
template <class T, int S, int LEN, int W, bool WF, int LS, int ES, int NT, bool MF, int Ns, int OFF>
struct SStages<T, S, LEN, W, WF, LS, ES, NT, MF, Ns, OFF> {
  __device__ __forceinline__ static void run(cpx<T>*, const cpx<T>*) {}
};
template <class T, int S, int LEN, int W, bool WF, int LS, int ES, int NT, bool MF, int Ns, int OFF,
          int R, int... Rest>
struct SStages<T, S, LEN, W, WF, LS, ES, NT, MF, Ns, OFF, R, Rest...> {
  __device__ __forceinline__ static void run(cpx<T>* buf, const cpx<T>* tw) {
    if constexpr (use_mstage<T, R, Ns, MF>())
      mstage<R, S, LEN, W, WF, LS, ES, NT>(buf);
    else
      sstage<T, R, S, LEN, W, WF, LS, ES, Ns, NT>(buf, tw + OFF);
    SStages<T, S, LEN, W, WF, LS, ES, NT, MF, Ns * R, OFF + (Ns > 1 ? Ns * (R - 1) : 0),
            Rest...>::run(buf, tw);
  }
};

template <class T, int S, int LEN, int W, bool WF, int LS, int ES, int NT, bool MF, class R_>
struct SStockham;
template <class T, int S, int LEN, int W, bool WF, int LS, int ES, int NT, bool MF, int... Rs>
struct SStockham<T, S, LEN, W, WF, LS, ES, NT, MF, Rad<Rs...>> {
  __device__ __forceinline__ static void run(cpx<T>* buf, const cpx<T>* tw) {
    SStages<T, S, LEN, W, WF, LS, ES, NT, MF, 1, 0, Rs...>::run(buf, tw);
  }
};

// Rader's algorithm for a prime n on W lines of n + 1 rows (the plan's tables
// after the Bluestein ones, see FftPlan): a_p = x_{g^-p} in rows 0..n-2 and x_0
// in row n; the (n-1)-point forward transform; X_0 = x_0 + A_0 into row n-1;
// A times B of sign S; the inverse transform gives the cyclic convolution c,
// and X_{g^q} = x_0 + c_q, X_0 go back to the rows of their indices.
template <class T, int S, class SP, int W, bool WF, int LS, int ES, int NT>
__device__ __forceinline__ void rader_fft(cpx<T>* buf, const cpx<T>* __restrict__ tw,
                                          const FftPlan& P) {
  using R_ = typename SP::radices;
  constexpr int n = SP::n, L = n - 1;
  constexpr int NG = (L * W + NT - 1) / NT;
  const cpx<T>* gi = tw + P.r_gidx;
  const cpx<T>* si = tw + P.r_sidx;
  const cpx<T>* Bv = tw + (S < 0 ? P.r_bf : P.r_bi);
  auto at = [](int u, int& w, int& p) __attribute__((always_inline)) {
    const int f = threadIdx.x + u * NT;
    if (WF) {
      w = f % W;
      p = f / W;
    } else {
      p = f % L;
      w = f / L;
    }
    return f < L * W;
  };
  cpx<T> v[NG];
  // gather a_p = x_{g^-p}; x_0 of line threadIdx.x (< W) to row n
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    int w, p;
    if (at(u, w, p)) v[u] = buf[w * LS + (int)gi[p].x * ES];
  }
  cpx<T> x0{};
  if ((int)threadIdx.x < W) x0 = buf[threadIdx.x * LS];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    int w, p;
    if (at(u, w, p)) buf[w * LS + p * ES] = v[u];
  }
  if ((int)threadIdx.x < W) buf[threadIdx.x * LS + n * ES] = x0;
  __syncthreads();
  SStockham<T, -1, L, W, WF, LS, ES, NT, false, R_>::run(buf, tw + P.r_off);
  if ((int)threadIdx.x < W) {
    cpx<T>* line = buf + threadIdx.x * LS;
    const cpx<T> a0 = line[0], xz = line[n * ES];
    line[L * ES] = cpx<T>{xz.x + a0.x, xz.y + a0.y};
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    int w, p;
    if (at(u, w, p)) {
      cpx<T>* e = buf + w * LS + p * ES;
      *e = cmul(*e, Bv[p]);
    }
  }
  __syncthreads();
  SStockham<T, +1, L, W, WF, LS, ES, NT, false, R_>::run(buf, tw + P.r_off);
  // scatter X_{g^q} = x_0 + c_q and X_0
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    int w, p;
    if (at(u, w, p)) {
      const cpx<T> c = buf[w * LS + p * ES], xz = buf[w * LS + n * ES];
      v[u] = cpx<T>{xz.x + c.x, xz.y + c.y};
    }
  }
  if ((int)threadIdx.x < W) x0 = buf[threadIdx.x * LS + L * ES];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    int w, p;
    if (at(u, w, p)) buf[w * LS + (int)si[p].x * ES] = v[u];
  }
  if ((int)threadIdx.x < W) buf[threadIdx.x * LS] = x0;
  __syncthreads();
}

// full n-point DFT of sign S on W lines (layout: element (w, i) at w*LS + i*ES);
// MF: first stage on the matrix cores where use_mstage allows it.  SP::blue:
// 0 Stockham, 1 Bluestein (tables at compile-time offsets), 2 Rader (tables
// located by the plan P)
template <class T, int S, class SP, int W, bool WF, int LS, int ES, int NT, bool MF = false>
__device__ __forceinline__ void sfft(cpx<T>* buf, const cpx<T>* __restrict__ tw,
                                     const FftPlan& P) {
  using R_ = typename SP::radices;
  if constexpr (SP::blue == 0) {
    SStockham<T, S, SP::len, W, WF, LS, ES, NT, MF, R_>::run(buf, tw);
  } else if constexpr (SP::blue == 2) {
    rader_fft<T, S, SP, W, WF, LS, ES, NT>(buf, tw, P);
  } else {
    constexpr int n = SP::n, m = SP::len;
    constexpr int chirp_off = TwSizeOf<R_>::v;
    constexpr int d_off = (S < 0) ? chirp_off + n : chirp_off + n + m;
    const cpx<T>* chirp = tw + chirp_off;
    const cpx<T>* D = tw + d_off;
    for (int f = threadIdx.x; f < m * W; f += NT) {
      int w, j;
      if (WF) { w = f % W; j = f / W; } else { j = f % m; w = f / m; }
      cpx<T>* e = buf + w * LS + j * ES;
      if (j < n) {
        cpx<T> c = chirp[j];
        if (S > 0) c.y = -c.y;
        *e = cmul(*e, c);
      } else {
        *e = cpx<T>{T(0), T(0)};
      }
    }
    __syncthreads();
    SStockham<T, -1, m, W, WF, LS, ES, NT, false, R_>::run(buf, tw);
    for (int f = threadIdx.x; f < m * W; f += NT) {
      int w, j;
      if (WF) { w = f % W; j = f / W; } else { j = f % m; w = f / m; }
      cpx<T>* e = buf + w * LS + j * ES;
      *e = cmul(*e, D[j]);
    }
    __syncthreads();
    SStockham<T, +1, m, W, WF, LS, ES, NT, false, R_>::run(buf, tw);
    for (int f = threadIdx.x; f < n * W; f += NT) {
      int w, j;
      if (WF) { w = f % W; j = f / W; } else { j = f % n; w = f / n; }
      cpx<T>* e = buf + w * LS + j * ES;
      cpx<T> c = chirp[j];
      if (S > 0) c.y = -c.y;
      *e = cmul(*e, c);
    }
    __syncthreads();
  }
}

}  // namespace hom

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

template <class T, int S, int LEN, int W, bool WF, int LS, int ES, int NT, int Ns, int OFF, int... Rs>
struct SStages;
template <class T, int S, int LEN, int W, bool WF, int LS, int ES, int NT, int Ns, int OFF>
struct SStages<T, S, LEN, W, WF, LS, ES, NT, Ns, OFF> {
  __device__ __forceinline__ static void run(cpx<T>*, const cpx<T>*) {}
};
template <class T, int S, int LEN, int W, bool WF, int LS, int ES, int NT, int Ns, int OFF, int R,
          int... Rest>
struct SStages<T, S, LEN, W, WF, LS, ES, NT, Ns, OFF, R, Rest...> {
  __device__ __forceinline__ static void run(cpx<T>* buf, const cpx<T>* tw) {
    sstage<T, R, S, LEN, W, WF, LS, ES, Ns, NT>(buf, tw + OFF);
    SStages<T, S, LEN, W, WF, LS, ES, NT, Ns * R, OFF + (Ns > 1 ? Ns * (R - 1) : 0),
            Rest...>::run(buf, tw);
  }
};

template <class T, int S, int LEN, int W, bool WF, int LS, int ES, int NT, class R_>
struct SStockham;
template <class T, int S, int LEN, int W, bool WF, int LS, int ES, int NT, int... Rs>
struct SStockham<T, S, LEN, W, WF, LS, ES, NT, Rad<Rs...>> {
  __device__ __forceinline__ static void run(cpx<T>* buf, const cpx<T>* tw) {
    SStages<T, S, LEN, W, WF, LS, ES, NT, 1, 0, Rs...>::run(buf, tw);
  }
};

// full n-point DFT of sign S on W lines (layout: element (w, i) at w*LS + i*ES)
template <class T, int S, class SP, int W, bool WF, int LS, int ES, int NT>
__device__ __forceinline__ void sfft(cpx<T>* buf, const cpx<T>* __restrict__ tw) {
  using R_ = typename SP::radices;
  if constexpr (!SP::blue) {
    SStockham<T, S, SP::len, W, WF, LS, ES, NT, R_>::run(buf, tw);
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
    SStockham<T, -1, m, W, WF, LS, ES, NT, R_>::run(buf, tw);
    for (int f = threadIdx.x; f < m * W; f += NT) {
      int w, j;
      if (WF) { w = f % W; j = f / W; } else { j = f % m; w = f / m; }
      cpx<T>* e = buf + w * LS + j * ES;
      *e = cmul(*e, D[j]);
    }
    __syncthreads();
    SStockham<T, +1, m, W, WF, LS, ES, NT, R_>::run(buf, tw);
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

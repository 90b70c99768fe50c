// Register-resident Stockham FFT for compile-time lengths (gfx950).
//
// A sequence of N complex values is spread over TT = N / 8 threads, each
// holding 8 values in registers.  Stage s (radix R, span Ns) works on the
// "stage-input layout" v[u*R + r] = x[b + r*(N/R)], b = t + TT*u, u < 8/R:
// every input r is multiplied by W_{Ns*R}^{r*(b % Ns)}, a radix-R DFT is
// applied, and output r belongs at index (b - b % Ns)*R + b % Ns + r*Ns.
// Between stages the values are exchanged through LDS (padded by one
// element every eight to spread banks); after the last stage (radix RL) the
// slot u*RL + r of thread t holds X[t + TT*(u + r*8/RL)] in natural order.
// The first stage reads the natural layout x[t + TT*i] directly when its
// radix is 8, so callers load and store global memory with consecutive
// threads on consecutive elements.
#pragma once

#include "ibp_device.hpp"

namespace ibp {
namespace rfft {

constexpr int kE = 8;   // values per thread

__device__ __forceinline__ constexpr int pad8(int o) { return o + (o >> 3); }
// padding of one element every 2^SH (SH = 3: pad8)
template <int SH>
__host__ __device__ __forceinline__ constexpr int padn(int o) { return o + (o >> SH); }

// LDS elements reserved per sequence: padded length plus one, so that
// consecutive sequences start in different banks.
template <int N, int SH = 3>
struct Seq {
  static constexpr int stride = N + (N >> SH) + 1;
};

// LDS stride of C sequences of N values of size B bytes held side by side in
// the lanes (sequence c = tid % C, as the z transforms lay out kx columns):
// the padded length rounded up so that the regions of adjacent sequences
// start 64 / C four-byte banks apart (at least one value apart when C values
// fill the 64 banks).  The 16 lanes an LDS access serves per cycle then cover
// the 64 banks (a model of every exchange of the plans above: one cycle per
// access, against 2-4 at the plain stride).
template <int N, int C, int B>
__host__ __device__ constexpr int col_stride() {
  constexpr int w = B / 4;   // banks per value (2 or 4)
  constexpr int gap = 64 / C > w ? 64 / C : w;
  int s = N + (N - 1) / 8 + 1;
  while ((s * w) % 64 != gap % 64) ++s;
  return s;
}

// PW: read only w^1 of each butterfly from the table and form w^2 ... w^(R-1)
// by products of depth at most 3 (one table read per butterfly instead of
// R - 1, for kernels whose table reads compete with their data).
template <int N, int R, int Ns, bool INV, typename T, bool PW = false>
__device__ __forceinline__ void stage_compute(Cx<T> (&v)[kE], int t, const Cx<T>* __restrict__ tw,
                                              int twstride) {
  constexpr int TT = N / kE;
#pragma unroll
  for (int u = 0; u < kE / R; ++u) {
    if constexpr (Ns > 1) {
      const int b = t + TT * u;
      const int k = b % Ns;
      if constexpr (PW) {
        Cx<T> w[R];
        w[1] = tw[(k * (N / (Ns * R))) * twstride];
        if (INV) w[1].y = -w[1].y;
        if constexpr (R > 2) w[2] = cmul(w[1], w[1]);
        if constexpr (R > 3) w[3] = cmul(w[2], w[1]);
        if constexpr (R > 4) {
          w[4] = cmul(w[2], w[2]);
          w[5] = cmul(w[4], w[1]);
          w[6] = cmul(w[4], w[2]);
          w[7] = cmul(w[4], w[3]);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[u * R + r] = cmul(v[u * R + r], w[r]);
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          Cx<T> w = tw[(r * k * (N / (Ns * R))) * twstride];
          if (INV) w.y = -w.y;
          v[u * R + r] = cmul(v[u * R + r], w);
        }
      }
    }
    Bfly<R, INV, T>::run(&v[u * R]);
  }
}

template <int N, int R, int Ns, typename T, int SH = 3>
__device__ __forceinline__ void stage_store(const Cx<T> (&v)[kE], int t, Cx<T>* lds) {
  constexpr int TT = N / kE;
#pragma unroll
  for (int u = 0; u < kE / R; ++u) {
    const int b = t + TT * u;
    const int k = b % Ns;
    const int base = (b - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) lds[padn<SH>(base + r * Ns)] = v[u * R + r];
  }
}

template <int N, int R, typename T, int SH = 3>
__device__ __forceinline__ void stage_load(Cx<T> (&v)[kE], int t, const Cx<T>* lds) {
  constexpr int TT = N / kE;
#pragma unroll
  for (int u = 0; u < kE / R; ++u)
#pragma unroll
    for (int r = 0; r < R; ++r) v[u * R + r] = lds[padn<SH>(t + TT * u + r * (N / R))];
}

// Natural sub-index of register slot s after a last stage of radix RL.
template <int RL>
__device__ __forceinline__ constexpr int final_index(int s) {
  return (s / RL) + (s % RL) * (kE / RL);
}

template <int N, int Ns, bool INV, typename T, bool PW, int SH, int R, int... Rest>
struct Stages {
  static constexpr int last_radix() {
    if constexpr (sizeof...(Rest) == 0)
      return R;
    else
      return Stages<N, Ns * R, INV, T, PW, SH, Rest...>::last_radix();
  }
  // Every thread of the block must call this (it contains __syncthreads).
  __device__ __forceinline__ static void run(Cx<T> (&v)[kE], int t, Cx<T>* lds, const Cx<T>* __restrict__ tw,
                                             int twstride) {
    stage_compute<N, R, Ns, INV, T, PW>(v, t, tw, twstride);
    if constexpr (sizeof...(Rest) > 0) {
      constexpr int R2 = Stages<N, Ns * R, INV, T, PW, SH, Rest...>::first_radix();
      stage_store<N, R, Ns, T, SH>(v, t, lds);
      __syncthreads();
      stage_load<N, R2, T, SH>(v, t, lds);
      __syncthreads();
      Stages<N, Ns * R, INV, T, PW, SH, Rest...>::run(v, t, lds, tw, twstride);
    }
  }
  static constexpr int first_radix() { return R; }
};

// Radix plans of the supported lengths (first radix 8: natural input layout).
// SH: LDS padding of the exchanges, one element every 2^SH
template <int N, bool INV, typename T, bool PW = false, int SH = 3>
struct Plan;
template <bool INV, typename T, bool PW, int SH>
struct Plan<32, INV, T, PW, SH> : Stages<32, 1, INV, T, PW, SH, 8, 4> {};
template <bool INV, typename T, bool PW, int SH>
struct Plan<64, INV, T, PW, SH> : Stages<64, 1, INV, T, PW, SH, 8, 8> {};
template <bool INV, typename T, bool PW, int SH>
struct Plan<128, INV, T, PW, SH> : Stages<128, 1, INV, T, PW, SH, 8, 4, 4> {};
template <bool INV, typename T, bool PW, int SH>
struct Plan<256, INV, T, PW, SH> : Stages<256, 1, INV, T, PW, SH, 8, 8, 4> {};
template <bool INV, typename T, bool PW, int SH>
struct Plan<512, INV, T, PW, SH> : Stages<512, 1, INV, T, PW, SH, 8, 8, 8> {};
template <bool INV, typename T, bool PW, int SH>
struct Plan<1024, INV, T, PW, SH> : Stages<1024, 1, INV, T, PW, SH, 8, 8, 4, 4> {};
// 2048: only the Bluestein convolutions of z lines up to 1024 points use it
// (256 threads per line); not a length of the plain register transforms.
template <bool INV, typename T, bool PW, int SH>
struct Plan<2048, INV, T, PW, SH> : Stages<2048, 1, INV, T, PW, SH, 8, 8, 8, 4> {};

__host__ __device__ constexpr bool supported(int n) {
  return n == 32 || n == 64 || n == 128 || n == 256 || n == 512 || n == 1024;
}

}  // namespace rfft
}  // namespace ibp

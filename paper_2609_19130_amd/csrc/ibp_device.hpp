// Device-side building blocks for libibpoisson (gfx950, wave64).
//
// * Cx<T>: interleaved complex value (T = double or float), aligned so a
//   whole value moves in one 16-byte (double) or 8-byte (float) access.
// * Radix-2/3/4/5/7/8/11 DFT butterflies, and a direct-sum stage for any
//   other prime radix.
// * lds_fft: mixed-radix Stockham autosort FFT of `nb` sequences of length
//   `n` that sit in LDS, all threads of the block cooperating.  Stage with
//   radix R and span Ns (product of the radices before it): butterfly j of a
//   sequence reads elements j + r*(n/R), multiplies input r by W_{Ns*R}^{r*(j%Ns)},
//   and writes output r to (j - j%Ns)*R + j%Ns + r*Ns.  Output is in natural
//   order.  Twiddles come from a host-computed FP64 table of W_N^e.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ibp_host.hpp"

namespace ibp {

constexpr int kThreads = 256;   // every kernel uses 256-thread blocks (4 waves)
constexpr int kWave = 64;

template <typename T>
struct alignas(2 * sizeof(T)) Cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return Cx<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return Cx<T>{a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return Cx<T>{a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ Cx<T> cscale(Cx<T> a, T s) { return Cx<T>{a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ Cx<T> cconj(Cx<T> a) { return Cx<T>{a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename T>
__device__ __forceinline__ Cx<T> mul_mi(Cx<T> a) {
  return INV ? Cx<T>{-a.y, a.x} : Cx<T>{a.y, -a.x};
}

// Global-address-space view of a base pointer: accesses through it compile
// to global loads and stores.  Through a generic pointer read from memory
// (the batched kernels' per-grid argument table) they compile to flat
// accesses, which also count against the LDS wait counter, so a tile's
// loads could not overlap its LDS writes; a cast back to a generic pointer
// loses the address space again.  Kernel-argument pointers are global to
// the compiler already.  Index the returned pointer (casting an offset
// generic pointer instead has measured flat in the generated code).
#define IBP_GLOBAL __attribute__((address_space(1)))
template <typename P>
__device__ __forceinline__ IBP_GLOBAL P* gbl(P* p) {
  return (IBP_GLOBAL P*)p;
}

// A complex value through a global view, member by member (an object in the
// global address space cannot bind to the copy constructor's generic
// reference); the members of an aligned Cx merge into one access.
template <typename T>
__device__ __forceinline__ Cx<T> gld(const IBP_GLOBAL Cx<T>* p) {
  return Cx<T>{p->x, p->y};
}
template <typename T>
__device__ __forceinline__ void gst(IBP_GLOBAL Cx<T>* p, Cx<T> v) {
  p->x = v.x;
  p->y = v.y;
}

// Two consecutive doubles (16-byte aligned) through a global view, as one
// 16-byte access.
__device__ __forceinline__ double2 gld2(const IBP_GLOBAL double* p) {
  const IBP_GLOBAL Cx<double>* q = reinterpret_cast<const IBP_GLOBAL Cx<double>*>(p);
  return make_double2(q->x, q->y);
}
__device__ __forceinline__ void gst2(IBP_GLOBAL double* p, double a, double b) {
  IBP_GLOBAL Cx<double>* q = reinterpret_cast<IBP_GLOBAL Cx<double>*>(p);
  q->x = a;
  q->y = b;
}

// Reversed block order for the passes that read what the previous pass of
// the solve wrote in ascending order (the forward z pass after the x R2C,
// the x C2R after the inverse z pass): they start on the data written last,
// which is still in the Infinity Cache.  Work per block is unchanged, so
// results are bitwise the same.  Measured at 512x384x512 FP64: forward z
// 327 -> 306 us.
__device__ __forceinline__ unsigned rev_block_x() { return gridDim.x - 1 - blockIdx.x; }
__device__ __forceinline__ unsigned rev_block_y() { return gridDim.y - 1 - blockIdx.y; }

// Exact quotient t / d of small non-negative integers (0 <= t < 2^19,
// d >= 1) from a float reciprocal: r = (1/d rounded) * (1 + 1.5 * 2^-20)
// rounded, and q = trunc(t * r rounded).  The three roundings move the
// product by less than 2^-22 relative, so it lies in [t/d, t/d (1 + 2^-19));
// that never reaches floor(t/d) + 1 while t < 2^19, and never falls below an
// exact quotient, so truncation gives floor(t/d).  Three full-rate VALU
// operations per quotient instead of the integer division sequence (whose
// 32-bit multiplies issue at quarter rate); used for the index arithmetic of
// the general LDS transforms, where t and d are tile offsets and lengths.
struct QDiv {
  float r;
  int d;
};
constexpr float kQDivRaise = 1.000001430511474609375f;   // 1 + 1.5 * 2^-20, exact in FP32
__device__ __forceinline__ QDiv qdiv(int d) { return QDiv{(1.0f / (float)d) * kQDivRaise, d}; }
__device__ __forceinline__ int qquo(int t, QDiv q) { return (int)((float)t * q.r); }
// t - d * (t / d)
__device__ __forceinline__ int qrem(int t, QDiv q) { return t - __mul24(qquo(t, q), q.d); }


// ---------------------------------------------------------------- butterflies
template <int R, bool INV, typename T>
struct Bfly;

template <bool INV, typename T>
struct Bfly<2, INV, T> {
  __device__ __forceinline__ static void run(Cx<T>* v) {
    Cx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV, typename T>
struct Bfly<4, INV, T> {
  __device__ __forceinline__ static void run(Cx<T>* v) {
    Cx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    Cx<T> t2 = cadd(v[1], v[3]), t3 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <bool INV, typename T>
struct Bfly<8, INV, T> {
  __device__ __forceinline__ static void run(Cx<T>* v) {
    const T h = T(0.7071067811865476);
    Cx<T> a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[r] = cadd(v[r], v[r + 4]);
      b[r] = csub(v[r], v[r + 4]);
    }
    // b[r] *= W_8^r (forward) or its conjugate (inverse)
    b[1] = INV ? Cx<T>{h * (b[1].x - b[1].y), h * (b[1].x + b[1].y)}
               : Cx<T>{h * (b[1].x + b[1].y), h * (b[1].y - b[1].x)};
    b[2] = mul_mi<INV>(b[2]);
    b[3] = INV ? Cx<T>{-h * (b[3].x + b[3].y), h * (b[3].x - b[3].y)}
               : Cx<T>{h * (b[3].y - b[3].x), -h * (b[3].x + b[3].y)};
    Bfly<4, INV, T>::run(a);
    Bfly<4, INV, T>::run(b);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[2 * q] = a[q];
      v[2 * q + 1] = b[q];
    }
  }
};

// Odd prime radix: y_q = v_0 + sum_r (v_r + v_{R-r}) cos(2 pi q r / R)
//                        -/+ i sum_r (v_r - v_{R-r}) sin(2 pi q r / R)
template <int R>
struct OddConst;
template <>
struct OddConst<3> {
  __device__ static constexpr double c(int k) { return -0.5; }
  __device__ static constexpr double s(int k) { return 0.8660254037844386; }
};
template <>
struct OddConst<5> {
  __device__ static constexpr double c(int k) { return k == 1 ? 0.30901699437494745 : -0.8090169943749475; }
  __device__ static constexpr double s(int k) { return k == 1 ? 0.9510565162951535 : 0.5877852522924731; }
};
template <>
struct OddConst<7> {
  __device__ static constexpr double c(int k) {
    return k == 1 ? 0.6234898018587335 : (k == 2 ? -0.2225209339563144 : -0.9009688679024191);
  }
  __device__ static constexpr double s(int k) {
    return k == 1 ? 0.7818314824680298 : (k == 2 ? 0.9749279121818236 : 0.4338837391175581);
  }
};
template <>
struct OddConst<11> {
  __device__ static constexpr double c(int k) {
    return k == 1 ? 0.8412535328311812
         : k == 2 ? 0.41541501300188644
         : k == 3 ? -0.14231483827328514
         : k == 4 ? -0.6548607339452851
                  : -0.9594929736144974;
  }
  __device__ static constexpr double s(int k) {
    return k == 1 ? 0.5406408174555976
         : k == 2 ? 0.9096319953545183
         : k == 3 ? 0.9898214418809327
         : k == 4 ? 0.7557495743542583
                  : 0.28173255684142967;
  }
};

template <int R, bool INV, typename T>
struct BflyOdd {
  __device__ __forceinline__ static void run(Cx<T>* v) {
    constexpr int H = (R - 1) / 2;
    Cx<T> sp[H], sm[H];
    Cx<T> y0 = v[0];
#pragma unroll
    for (int r = 1; r <= H; ++r) {
      sp[r - 1] = cadd(v[r], v[R - r]);
      sm[r - 1] = csub(v[r], v[R - r]);
      y0 = cadd(y0, sp[r - 1]);
    }
    Cx<T> out[R];
    out[0] = y0;
#pragma unroll
    for (int q = 1; q <= H; ++q) {
      Cx<T> A = v[0], B = Cx<T>{T(0), T(0)};
#pragma unroll
      for (int r = 1; r <= H; ++r) {
        int k = (q * r) % R;
        // cos(2 pi k / R) = cos(2 pi (R-k) / R); sin(2 pi k / R) = -sin(2 pi (R-k)/R)
        const T cv = T(OddConst<R>::c(k <= H ? k : R - k));
        const T sv = T(k <= H ? OddConst<R>::s(k) : -OddConst<R>::s(R - k));
        A.x += cv * sp[r - 1].x;
        A.y += cv * sp[r - 1].y;
        B.x += sv * sm[r - 1].x;
        B.y += sv * sm[r - 1].y;
      }
      Cx<T> iB = mul_mi<INV>(B);      // -i B forward, +i B inverse
      out[q] = cadd(A, iB);
      out[R - q] = csub(A, iB);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = out[q];
  }
};
template <bool INV, typename T>
struct Bfly<3, INV, T> : BflyOdd<3, INV, T> {};
template <bool INV, typename T>
struct Bfly<5, INV, T> : BflyOdd<5, INV, T> {};
template <bool INV, typename T>
struct Bfly<7, INV, T> : BflyOdd<7, INV, T> {};
template <bool INV, typename T>
struct Bfly<11, INV, T> : BflyOdd<11, INV, T> {};

// ---------------------------------------------------------------- LDS FFT
// One Stockham stage over all sequences.  Every thread first reads and
// transforms all its butterflies into registers, then the block syncs, then
// the results are written back in place.  MAXB bounds butterflies per thread:
// the host guarantees nb * n <= MAXB * R * kThreads.
template <int R, int MAXB, bool INV, typename T>
__device__ __forceinline__ void fft_stage(Cx<T>* buf, int n, int nb, int ss, int Ns,
                                          const IBP_GLOBAL Cx<T>* __restrict__ tw, int twstride) {
  const int m = n / R;
  const int nbf = nb * m;
  const int twmul = (n / (Ns * R)) * twstride;
  const QDiv qm = qdiv(m), qs = qdiv(Ns);
  Cx<T> v[MAXB][R];
  int dst[MAXB];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int t = threadIdx.x + q * kThreads;
    dst[q] = -1;
    if (t < nbf) {
      const int b = qquo(t, qm);
      const int j = t - __mul24(b, m);
      const int k = qrem(j, qs);
      const Cx<T>* base = buf + __mul24(b, ss);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = base[j + r * m];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          Cx<T> w = gld(tw + __mul24(r * k, twmul));
          if (INV) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      Bfly<R, INV, T>::run(v[q]);
      dst[q] = __mul24(b, ss) + (j - k) * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    if (dst[q] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[q] + r * Ns] = v[q][r];
    }
  }
  __syncthreads();
}

// Stage of any radix R (the prime factors above 11): output q of butterfly j
// is the R-term DFT by definition,
//   y_q = sum_r x[j + r m] w_q^r,   w_q = W_{Ns R}^{k + q Ns},   k = j mod Ns,
// the stage twiddle W_{Ns R}^{r k} and the butterfly's own W_R^{q r} folded
// into one root per output, summed by Horner's rule (y <- y w_q + x_r from
// r = R-1 down), so each output takes one table read; a thread runs QA
// outputs of one butterfly together, so each input read from LDS serves QA
// accumulators.  O(n R) per stage.  Out of place: outputs go to
// (j - k) R + k + q Ns of `spare` (the upper half of the block's tile, which
// the host leaves free for plans with such a factor), then are copied back.
template <bool INV, typename T>
__device__ __forceinline__ void fft_stage_any(Cx<T>* buf, Cx<T>* spare, int n, int nb, int ss, int Ns, int R,
                                              const IBP_GLOBAL Cx<T>* __restrict__ tw, int twstride) {
  constexpr int QA = 4;
  const int m = n / R;
  const int twmul = (n / (Ns * R)) * twstride;
  const int QB = (R + QA - 1) / QA;   // output groups per butterfly
  const int items = nb * m * QB;
  const QDiv qmb = qdiv(m * QB), qm = qdiv(m), qs = qdiv(Ns), qn = qdiv(n);
  for (int t = threadIdx.x; t < items; t += kThreads) {
    const int b = qquo(t, qmb);
    const int w = t - __mul24(b, m * QB);
    const int qb = qquo(w, qm), j = w - __mul24(qb, m);   // consecutive threads: consecutive butterflies
    const int k = qrem(j, qs);
    const Cx<T>* base = buf + __mul24(b, ss) + j;
    Cx<T> om[QA], y[QA];
    const Cx<T> top = base[(R - 1) * m];
#pragma unroll
    for (int u = 0; u < QA; ++u) {
      const int q = qb * QA + u < R ? qb * QA + u : R - 1;
      om[u] = gld(tw + (k + q * Ns) * twmul);
      if (INV) om[u].y = -om[u].y;
      y[u] = top;
    }
    for (int r = R - 2; r >= 0; --r) {
      const Cx<T> x = base[r * m];
#pragma unroll
      for (int u = 0; u < QA; ++u) y[u] = cadd(cmul(y[u], om[u]), x);
    }
#pragma unroll
    for (int u = 0; u < QA; ++u) {
      const int q = qb * QA + u;
      if (q < R) spare[b * ss + (j - k) * R + k + q * Ns] = y[u];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nb * n; t += kThreads) {
    const int b = qquo(t, qn);
    const int i = __mul24(b, ss) + (t - __mul24(b, n));
    buf[i] = spare[i];
  }
  __syncthreads();
}

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// The Stockham stages of one factorisation over nb sequences of length n.
// WIDE = false leaves out the radix-7 and radix-11 butterflies and the
// direct-sum stage, whose registers set the kernel's whole register count
// (the caller guarantees radices 2, 3, 4, 5 and 8 only).
template <int TILE, bool INV, typename T, bool WIDE = true>
__device__ __forceinline__ void lds_stages(Cx<T>* buf, int nb, int ss, int n, int nst, const int* radix,
                                           const IBP_GLOBAL Cx<T>* __restrict__ tw, int twstride) {
  int Ns = 1;
  for (int s = 0; s < nst; ++s) {
    const int R = radix[s];
    switch (R) {
      case 8: fft_stage<8, cdiv(TILE, 8 * kThreads), INV, T>(buf, n, nb, ss, Ns, tw, twstride); break;
      case 4: fft_stage<4, cdiv(TILE, 4 * kThreads), INV, T>(buf, n, nb, ss, Ns, tw, twstride); break;
      case 2: fft_stage<2, cdiv(TILE, 2 * kThreads), INV, T>(buf, n, nb, ss, Ns, tw, twstride); break;
      case 3: fft_stage<3, cdiv(TILE, 3 * kThreads), INV, T>(buf, n, nb, ss, Ns, tw, twstride); break;
      case 5: fft_stage<5, cdiv(TILE, 5 * kThreads), INV, T>(buf, n, nb, ss, Ns, tw, twstride); break;
      case 7:
        if constexpr (WIDE) fft_stage<7, cdiv(TILE, 7 * kThreads), INV, T>(buf, n, nb, ss, Ns, tw, twstride);
        break;
      case 11:
        if constexpr (WIDE) fft_stage<11, cdiv(TILE, 11 * kThreads), INV, T>(buf, n, nb, ss, Ns, tw, twstride);
        break;
      default:
        if constexpr (WIDE) fft_stage_any<INV, T>(buf, buf + TILE / 2, n, nb, ss, Ns, R, tw, twstride);
        break;
    }
    Ns *= R;
  }
}

// Bluestein's algorithm (the DFT as a chirp convolution): with
// w_j = exp(-i pi j^2 / n), X_k = w_k sum_j (x_j w_j) conj(w_{k-j}), a cyclic
// convolution of length m >= 2n - 1 done by two length-m transforms:
//   a = x w zero-padded to m;  c = IFFT_m(FFT_m(a) * bhat) / m;  X = w c,
// bhat = FFT_m of conj(w) laid out cyclically (host table).  The inverse DFT
// is conj(forward(conj(x))).  Sequences sit at stride ss >= m.
template <int TILE, bool INV, typename T>
__device__ __forceinline__ void bluestein_fft(Cx<T>* buf, int nb, int ss, const FftPlan& fp,
                                              const IBP_GLOBAL Cx<T>* __restrict__ chirp,
                                              const IBP_GLOBAL Cx<T>* __restrict__ bhat,
                                              const IBP_GLOBAL Cx<T>* __restrict__ twm) {
  const int n = fp.n, m = fp.m;
  const QDiv qm = qdiv(m), qn = qdiv(n);
  for (int t = threadIdx.x; t < nb * m; t += kThreads) {
    const int b = qquo(t, qm), j = t - __mul24(b, m);
    Cx<T> v{T(0), T(0)};
    if (j < n) {
      v = buf[b * ss + j];
      if (INV) v = cconj(v);
      v = cmul(v, gld(chirp + j));
    }
    buf[b * ss + j] = v;
  }
  __syncthreads();
  lds_stages<TILE, false, T>(buf, nb, ss, m, fp.mst, fp.mradix, twm, 1);
  for (int t = threadIdx.x; t < nb * m; t += kThreads) {
    const int b = qquo(t, qm), k = t - __mul24(b, m);
    buf[b * ss + k] = cmul(buf[b * ss + k], gld(bhat + k));
  }
  __syncthreads();
  lds_stages<TILE, true, T>(buf, nb, ss, m, fp.mst, fp.mradix, twm, 1);
  const T inv_m = T(1) / T(m);
  for (int t = threadIdx.x; t < nb * n; t += kThreads) {
    const int b = qquo(t, qn), k = t - __mul24(b, n);
    Cx<T> v = cscale(cmul(buf[b * ss + k], gld(chirp + k)), inv_m);
    if (INV) v = cconj(v);
    buf[b * ss + k] = v;
  }
  __syncthreads();
}

// nb sequences of length fp.n; sequence b starts at buf + b*ss.
// TILE is the compile-time bound on nb * ss; a plan with a prime factor
// above 11 (fp.any) keeps nb * ss <= TILE / 2 (the direct-sum stage's spare
// half).  Bluestein plans (fp.blu) take the chirp, filter and length-m
// twiddle tables.  WIDE = false: radices 2, 3, 4, 5, 8 only, no Bluestein.
template <int TILE, bool INV, typename T, bool WIDE = true>
__device__ __forceinline__ void lds_fft(Cx<T>* buf, int nb, int ss, const FftPlan& fp,
                                        const IBP_GLOBAL Cx<T>* __restrict__ tw, int twstride,
                                        const IBP_GLOBAL Cx<T>* __restrict__ bchirp = nullptr,
                                        const IBP_GLOBAL Cx<T>* __restrict__ bhat = nullptr,
                                        const IBP_GLOBAL Cx<T>* __restrict__ btw = nullptr) {
  if constexpr (WIDE) {
    if (fp.blu) {
      bluestein_fft<TILE, INV, T>(buf, nb, ss, fp, bchirp, bhat, btw);
      return;
    }
  }
  lds_stages<TILE, INV, T, WIDE>(buf, nb, ss, fp.n, fp.nst, fp.radix, tw, twstride);
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Deterministic block reduction of NV values per thread (fixed order):
// wave butterflies, then the NT/64 wave results combined in wave order.
// sh must hold NV * NT/64 doubles.
template <int NV, int NT = kThreads>
__device__ __forceinline__ void block_reduce(double (&v)[NV], const bool (&is_max)[NV], double* sh) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = is_max[i] ? wave_max(v[i]) : wave_sum(v[i]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[wave * NV + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double r = sh[i];
    for (int w = 1; w < NT / kWave; ++w) r = is_max[i] ? fmax(r, sh[w * NV + i]) : r + sh[w * NV + i];
    v[i] = r;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- XCD-local scheduling
// Hardware id of the XCD (accelerator complex die) this wave runs on: bits
// [3:0] of the XCC_ID hardware register (register 20 on CDNA3/CDNA4).
__device__ __forceinline__ int xcc_id() {
  constexpr int kXccIdReg = 20, kSize = 4, kOffset = 0;
  return __builtin_amdgcn_readfirstlane(
      __builtin_amdgcn_s_getreg(((kSize - 1) << 11) | (kOffset << 6) | kXccIdReg) & 15);
}

// Wave 0 waits until `counter` reaches `need`; bounded (max_spins polls) so
// that a broken dependency raises the error flag instead of hanging the device.
__device__ __forceinline__ void wave_wait_count(int* counter, int need, int* error, int max_spins = 1 << 20) {
  for (int spins = 0;; ++spins) {
    const int v = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (v >= need) break;
    if (spins >= max_spins) {
      __hip_atomic_store(error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// s_waitcnt immediate for vmcnt(0) with expcnt and lgkmcnt left free
// (gfx9 encoding: vmcnt [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8]).
constexpr int kWaitVmcnt0 = 0x0F70;

}  // namespace ibp

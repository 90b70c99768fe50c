// Bluestein transforms held in registers, for line lengths n <= 1024 with a
// prime factor above 11 (the paper's 501- and 632-point grids: 501 = 3 x 167,
// 632 = 8 x 79), which the LDS kernels would run as direct-sum stages (up to
// ~170 complex multiply-adds per value) or, for primes above 256, as their
// own slower convolution.  A length-n DFT is X_k = w_k sum_j (x_j w_j) conj(w_{k-j}) with
// the chirp w_j = exp(-i pi j^2 / n): the sum is a cyclic convolution of
// length M (a power of two >= 2n - 1, at most 2048), done as two register
// FFTs of length M (ibp_regfft.hpp) around a pointwise product with the
// filter's transform bhat.  The inverse DFT (unnormalised) is
// conj(DFT(conj(X))).  Tables (host, long double rounded): chirp (n values),
// bhat (M) and W_M^e (M) in the Bluestein slots of the argument structs.
//
// z pass: C kx columns of one y plane per block, M / 8 threads per column.
// x pass: two real rows per complex line (the whole row of n points, odd or
// even n), M / 8 threads per line; R2C separates the two spectra, keeps the
// first n / 2 + 1 coefficients of each and the FP64 row sums; C2R combines
// the two half spectra into the line's full spectrum and splits real and
// imaginary parts.
#include <type_traits>

#include "ibp_internal.hpp"
#include "ibp_regfft.hpp"

namespace ibp {

using rfft::final_index;
using rfft::kE;

// One length-n line whose values v[i] (index t + TT i, zero past n) are
// already multiplied by the chirp: returns in v[q] the convolution at index
// t + TT final_index(q), unnormalised (times M).  As M >= 2n - 1, n <= M / 2:
// slots i >= kE / 2 of the input are always zero and only outputs with
// final_index(q) < kE / 2 are ever used, so a lane's chirp values (indices
// t + TT i, i < kE / 2) serve both its loads and its stores.
constexpr int kH = kE / 2;
template <int M, typename T, int SH>
__device__ __forceinline__ void blu_convolve(Cx<T> (&v)[kE], int t, Cx<T>* lds, const Cx<T>* bb, const Cx<T>* bt) {
  // w^2 ... w^7 of each butterfly formed from w^1: the chirp and filter
  // tables already compete with the line data for the vector cache
  using PF = rfft::Plan<M, false, T, true, SH>;
  using PI = rfft::Plan<M, true, T, true, SH>;
  constexpr int TT = M / kE;
  constexpr int RF = PF::last_radix();
  PF::run(v, t, lds, bt, 1);
  Cx<T> u[kE];
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int i = final_index<RF>(q);   // output q is index t + TT i
    u[i] = cmul(v[q], bb[t + TT * i]);
  }
  PI::run(u, t, lds, bt, 1);
#pragma unroll
  for (int q = 0; q < kE; ++q) v[q] = u[q];
}

// LDS layout: z regions at rfft::col_stride (adjacent columns 64 / C banks
// apart: z passes at 501 x 1001 x 501 1.77 -> 1.59 ms against the plain
// padded length); x lines at the plain padded length (one pad every 16
// elements, which a bank model rates better, measured no faster).
template <typename T, int M, int C>
constexpr int blu_z_stride() { return rfft::col_stride<M, C, sizeof(Cx<T>)>(); }
template <typename T, int M>
constexpr int blu_x_shift() { return 3; }
// threads per x block: kThreads, several lines per block up to M = 1024
// (one 1024-point line per 128-thread block measured the same: 1.82 / 1.75
// against 1.85 / 1.71 ms for the two passes at 501 x 1001 x 501)
template <int M>
constexpr int blu_x_threads() { return kThreads; }

// Column groups narrower than a 128-byte line: the S groups of one line
// (S = 128 / (C * sizeof(Cx<T>)), 2 or 4) go to blocks b, b + 8, ..., which
// the round-robin dispatch places on one XCD at about the same time, so the
// line is fetched into that XCD's L2 once.  The launch rounds the groups per
// plane up to a multiple of S (whole dead groups return at once); the last
// (blocks mod 8S) blocks take the remaining sets in order.
template <typename T, int C>
constexpr int blu_z_siblings() {
  constexpr int w = C * (int)sizeof(Cx<T>);
  return w >= 128 ? 1 : 128 / w;
}

template <typename T, bool INV, int M, int C>
__global__ __launch_bounds__(C*(M / kE)) void k_zblu_reg(ZfArgs<T> A) {
  constexpr int TT = M / kE;
  constexpr int SS = blu_z_stride<T, M, C>();
  constexpr int RI = rfft::Plan<M, true, T>::last_radix();
  constexpr int S = blu_z_siblings<T, C>();
  __shared__ Cx<T> lds[C * SS];
  if (A.check_done && A.ctl->done) return;
  int grp = blockIdx.x, pl = blockIdx.y;
  if constexpr (S > 1) {
    const long G = gridDim.x, nb = G * gridDim.y, full = nb / (8 * S) * (8 * S);
    const long b = (long)blockIdx.y * G + blockIdx.x;
    long set, h;
    if (b < full) {
      set = (b / (8 * S)) * 8 + (b % 8);
      h = (b % (8 * S)) / 8;
    } else {
      set = full / S + (b - full) / S;
      h = (b - full) % S;
    }
    pl = (int)(set / (G / S));
    grp = (int)((set % (G / S)) * S + h);
    if (grp * C >= A.hp) return;   // a whole dead group (uniform)
  }
  const int tid = threadIdx.x, c = tid % C, t = tid / C;
  const int col = grp * C + c;
  const bool live = col < A.hp;
  const int n = A.nz;
  Cx<T>* plane = A.spec + (size_t)(A.plane0 + pl) * A.ps;
  Cx<T> v[kE], ch[kH];
#pragma unroll
  for (int i = 0; i < kH; ++i) {
    const int z = t + TT * i;
    Cx<T> x{T(0), T(0)};
    ch[i] = x;
    if (live && z < n) {
      x = plane[(size_t)z * A.rs + col];
      if (INV) x = cconj(x);
      ch[i] = A.bc[z];
      x = cmul(x, ch[i]);
    }
    v[i] = x;
    v[i + kH] = Cx<T>{T(0), T(0)};
  }
  blu_convolve<M, T, 3>(v, t, lds + c * SS, A.bb, A.bt);
  if (!live) return;   // no barrier follows
  const T inv_m = T(1) / T(M);
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int fi = final_index<RI>(q);
    const int k = t + TT * fi;
    if (fi < kH && k < n) {
      Cx<T> X = cscale(cmul(ch[fi < kH ? fi : 0], v[q]), inv_m);
      if (INV) X = cconj(X);
      plane[(size_t)k * A.rs + col] = X;
    }
  }
}

// Sum over the TT threads of a line (TT a power of two; a line's threads are
// TT consecutive lanes, or whole waves when TT > 64).
template <int TT>
__device__ __forceinline__ double row_total(double s, double* sh, int lr) {
  if constexpr (TT <= kWave) {
#pragma unroll
    for (int off = TT / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
    return s;
  } else {
    s = wave_sum(s);
    const int w = (threadIdx.x % TT) / kWave;   // wave within the row
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) sh[lr * (TT / kWave) + w] = s;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < TT / kWave; ++q) r += sh[lr * (TT / kWave) + q];
    return r;
  }
}

// Two real rows a, b of length n share one complex line z = a + i b:
// with Z = DFT(z), A_k = (Z_k + conj Z_{n-k}) / 2 and
// B_k = (Z_k - conj Z_{n-k}) / (2i), so one Bluestein transform serves both.
// Rows 2p and 2p + 1 form line p; a missing second row (odd row count)
// reads as zeros and is not stored.
template <typename T>
__device__ __forceinline__ Cx<T>* xblu_spec_row(const XArgs<T>& A, long row) {
  return A.spec + row * A.rs + (row / A.nz) * (A.ps - (long)A.nz * A.rs);
}

// x R2C (FP64 right-hand side pass), two rows per line.
template <typename T, int M>
__global__ __launch_bounds__(blu_x_threads<M>()) void k_xblu_r2c(XArgs<T> A) {
  constexpr int TT = M / kE;
  constexpr int RB = blu_x_threads<M>() / TT;   // lines (row pairs) per block
  constexpr int SH = blu_x_shift<T, M>();
  constexpr int SS = rfft::Seq<M, SH>::stride;
  constexpr int RI = rfft::Plan<M, true, T>::last_radix();
  __shared__ Cx<T> lds[RB * SS];
  __shared__ double sh[blu_x_threads<M>() / kWave];
  const int tid = threadIdx.x, lr = tid / TT, t = tid % TT;
  const long r0 = 2 * ((A.row_begin / (2 * RB) + blockIdx.x) * RB + lr);
  const bool live0 = r0 < A.nrows, live1 = r0 + 1 < A.nrows;
  const int n = A.nx;
  const double* fa = A.f + (live0 ? r0 : 0) * n;
  const double* fb = A.f + (live1 ? r0 + 1 : 0) * n;
  // (the chirp is read again at the end: keeping it in registers across the
  // convolution measured slower here, 1.95 against 1.86 ms per pass at
  // 501 x 1001 x 501)
  Cx<T> v[kE];
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int i = 0; i < kH; ++i) {
    const int m = t + TT * i;
    Cx<T> x{T(0), T(0)};
    if (m < n) {
      const double av = live0 ? fa[m] : 0.0;
      const double bv = live1 ? fb[m] : 0.0;
      sa += av;
      sb += bv;
      x = cmul(Cx<T>{T(av), T(bv)}, A.bc[m]);
    }
    v[i] = x;
    v[i + kH] = Cx<T>{T(0), T(0)};
  }
  sa = row_total<TT>(sa, sh, lr);
  sb = row_total<TT>(sb, sh, lr);
  if (t == 0) {
    if (live0) A.rowsum[r0] = sa;
    if (live1) A.rowsum[r0 + 1] = sb;
  }
  Cx<T>* L = lds + lr * SS;
  blu_convolve<M, T, SH>(v, t, L, A.bb, A.bt);
  // Z_k (chirp and 1/M applied) to LDS, natural order; the last LDS access
  // of the convolution was a load followed by a barrier
  const T inv_m = T(1) / T(M);
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int fi = final_index<RI>(q);
    const int k = t + TT * fi;
    if (fi < kH && k < n) L[rfft::padn<SH>(k)] = cscale(cmul(A.bc[k], v[q]), inv_m);
  }
  __syncthreads();
  if (!live0) return;   // no barrier follows
  Cx<T>* sa_row = xblu_spec_row(A, r0);
  Cx<T>* sb_row = xblu_spec_row(A, r0 + 1);
#pragma unroll
  for (int i = 0; i < kE; ++i) {
    const int k = t + TT * i;
    if (k < A.hp) {
      const Cx<T> z = L[rfft::padn<SH>(k)];
      const Cx<T> w = L[rfft::padn<SH>(k == 0 ? 0 : n - k)];
      sa_row[k] = Cx<T>{T(0.5) * (z.x + w.x), T(0.5) * (z.y - w.y)};
      if (live1) sb_row[k] = Cx<T>{T(0.5) * (z.y + w.y), T(0.5) * (w.x - z.x)};
    }
  }
}

// x C2R (set or add), two rows per line: the line's
// spectrum is Z_k = A_k + i B_k over all k (A_{n-k} = conj A_k), its inverse
// DFT is a + i b.
template <typename T, int MODE, int M>
__global__ __launch_bounds__(blu_x_threads<M>()) void k_xblu_c2r(XArgs<T> A) {
  constexpr int TT = M / kE;
  constexpr int RB = blu_x_threads<M>() / TT;
  constexpr int SH = blu_x_shift<T, M>();
  constexpr int SS = rfft::Seq<M, SH>::stride;
  constexpr int RI = rfft::Plan<M, true, T>::last_radix();
  __shared__ Cx<T> lds[RB * SS];
  if (MODE == CM_ADD && A.ctl->done) return;
  const int tid = threadIdx.x, lr = tid / TT, t = tid % TT;
  const long r0 = 2 * ((A.row_begin / (2 * RB) + blockIdx.x) * RB + lr);
  const bool live0 = r0 < A.nrows, live1 = r0 + 1 < A.nrows;
  const int n = A.nx;
  const Cx<T>* sa_row = xblu_spec_row(A, live0 ? r0 : 0);
  const Cx<T>* sb_row = xblu_spec_row(A, live1 ? r0 + 1 : 0);
  // conj(Z_j) times the chirp (inverse DFT = conj DFT conj)
  Cx<T> v[kE], ch[kH];
#pragma unroll
  for (int i = 0; i < kH; ++i) {
    const int j = t + TT * i;
    Cx<T> y{T(0), T(0)};
    ch[i] = y;
    if (live0 && j < n) {
      Cx<T> a, b{T(0), T(0)};
      if (j < A.hp) {
        a = sa_row[j];
        if (live1) b = sb_row[j];
        if (j == 0 || 2 * j == n) a.y = b.y = T(0);   // X[0] and X[n/2] of a real sequence are real
      } else {
        a = cconj(sa_row[n - j]);
        if (live1) b = cconj(sb_row[n - j]);
      }
      // Z = a + i b; conj Z
      ch[i] = A.bc[j];
      y = cmul(Cx<T>{a.x - b.y, -(a.y + b.x)}, ch[i]);
    }
    v[i] = y;
    v[i + kH] = Cx<T>{T(0), T(0)};
  }
  blu_convolve<M, T, SH>(v, t, lds + lr * SS, A.bb, A.bt);
  if (!live0) return;   // no barrier follows
  // out_scale is 1 / (h nz) with h the general kernels' transform length
  // (nx / 2 for even nx): the whole row's inverse needs 1 / (nx nz)
  double cs = A.out_scale * (double(A.h) / double(n)) / double(M);
  if (MODE == CM_ADD) cs = cs / A.ctl->scale[A.iter & 1];
  double ca = A.phi00[(int)(r0 / A.nz)] * A.inv_nxnz;
  double cb = live1 ? A.phi00[(int)((r0 + 1) / A.nz)] * A.inv_nxnz : 0.0;
  if (MODE == CM_ADD) {
    ca -= A.ctl->phimean;
    cb -= A.ctl->phimean;
  }
  double* oa = A.out + r0 * n;
  double* ob = oa + n;
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int fi = final_index<RI>(q);
    const int j = t + TT * fi;
    if (fi < kH && j < n) {
      // a + i b = conj(w_j conv_j) / M
      const Cx<T> w = ch[fi < kH ? fi : 0];
      const double re = double(w.x) * double(v[q].x) - double(w.y) * double(v[q].y);
      const double im = double(w.x) * double(v[q].y) + double(w.y) * double(v[q].x);
      double xa = re * cs + ca;
      if (MODE == CM_ADD) xa += oa[j];
      oa[j] = xa;
      if (live1) {
        double xb = -im * cs + cb;
        if (MODE == CM_ADD) xb += ob[j];
        ob[j] = xb;
      }
    }
  }
}

// ---------------------------------------------------------------- launchers
// kx columns per z block: 128-byte segments where the block fits 1024
// threads, except FP64 at M = 512 and 1024, which take 4 columns (64-byte
// segments; two blocks per compute unit at M = 1024, so one block's loads
// overlap another's arithmetic: 2.17 -> 1.96 ms per pass at 501 x 1001 x 501
// against 8 columns), and FP64 at M = 2048, 2 columns (two blocks per unit:
// 6.19 -> 5.89 ms per pass at 632 x 1263 x 632 against 4).  The 8-column FP64 instance at M = 512 (512 threads)
// returned wrong values on the GPU for every length tried (131, 167, 255)
// while the 4- and 16-column instances of the same code are exact; the cause
// was not found, and that instance is not built.
template <typename T, int M>
constexpr int blu_z_cols() {
  if (sizeof(T) == 8 && (M == 512 || M == 1024)) return 4;
  if (sizeof(T) == 8 && M == 2048) return 2;
  constexpr int seg = 128 / (int)sizeof(Cx<T>);
  constexpr int maxc = 1024 / (M / kE);
  return seg < maxc ? seg : maxc;
}

// The M cases of a launcher: f(std::integral_constant<int, M>).
template <typename F>
hipError_t blu_dispatch(int M, F&& f) {
  switch (M) {
    case 32: return f(std::integral_constant<int, 32>{});
    case 64: return f(std::integral_constant<int, 64>{});
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    case 512: return f(std::integral_constant<int, 512>{});
    case 1024: return f(std::integral_constant<int, 1024>{});
    case 2048: return f(std::integral_constant<int, 2048>{});
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_zblu_reg(bool inverse, const ZfArgs<T>& a, int M, int nplanes, hipStream_t s) {
  if (a.nz > 1024 || 2 * a.nz - 1 > M) return hipErrorInvalidValue;
  auto go = [&](auto m_) {
    constexpr int m = decltype(m_)::value;
    constexpr int C = blu_z_cols<T, m>();
    constexpr int S = blu_z_siblings<T, C>();
    const int groups = (a.hp + C - 1) / C;
    const dim3 grid((unsigned)((groups + S - 1) / S * S), (unsigned)nplanes);
    if (inverse)
      hipLaunchKernelGGL((k_zblu_reg<T, true, m, C>), grid, dim3(C * (m / kE)), 0, s, a);
    else
      hipLaunchKernelGGL((k_zblu_reg<T, false, m, C>), grid, dim3(C * (m / kE)), 0, s, a);
    return hipGetLastError();
  };
  return blu_dispatch(M, go);
}

template <typename T>
hipError_t launch_xblu_r2c(const XArgs<T>& a, int M, hipStream_t s) {
  if (a.nx > 1024 || 2 * a.nx - 1 > M) return hipErrorInvalidValue;
  return blu_dispatch(M, [&](auto m_) {
    constexpr int m = decltype(m_)::value;
    constexpr int NT = blu_x_threads<m>();
    const int RB = 2 * (NT / (m / kE));   // rows per block
    if (a.row_begin % RB) return hipErrorInvalidValue;
    const long nb = (a.nrows - a.row_begin + RB - 1) / RB;
    hipLaunchKernelGGL((k_xblu_r2c<T, m>), dim3((unsigned)nb), dim3(NT), 0, s, a);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t launch_xblu_c2r(int mode, const XArgs<T>& a, int M, hipStream_t s) {
  if (a.nx > 1024 || 2 * a.nx - 1 > M) return hipErrorInvalidValue;
  return blu_dispatch(M, [&](auto m_) {
    constexpr int m = decltype(m_)::value;
    constexpr int NT = blu_x_threads<m>();
    const int RB = 2 * (NT / (m / kE));   // rows per block
    if (a.row_begin % RB) return hipErrorInvalidValue;
    const long nb = (a.nrows - a.row_begin + RB - 1) / RB;
    if (mode == CM_ADD)
      hipLaunchKernelGGL((k_xblu_c2r<T, CM_ADD, m>), dim3((unsigned)nb), dim3(NT), 0, s, a);
    else
      hipLaunchKernelGGL((k_xblu_c2r<T, CM_SET, m>), dim3((unsigned)nb), dim3(NT), 0, s, a);
    return hipGetLastError();
  });
}

template hipError_t launch_zblu_reg<double>(bool, const ZfArgs<double>&, int, int, hipStream_t);
template hipError_t launch_zblu_reg<float>(bool, const ZfArgs<float>&, int, int, hipStream_t);
template hipError_t launch_xblu_r2c<double>(const XArgs<double>&, int, hipStream_t);
template hipError_t launch_xblu_c2r<double>(int, const XArgs<double>&, int, hipStream_t);
template hipError_t launch_xblu_c2r<float>(int, const XArgs<float>&, int, hipStream_t);

}  // namespace ibp

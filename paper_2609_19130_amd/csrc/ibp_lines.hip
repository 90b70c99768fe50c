// Factored implicit viscous solve: one tridiagonal system per grid line and
// direction (paper: Crank-Nicolson viscous terms of eq. nstime_discr, split
// into direction-wise Thomas solves with a Sherman-Morrison correction in the
// two periodic directions; "Fluid domain" parallelisation subsection).
//
// Every line of one direction has the same matrix, so its LU is factored once
// on the host (FP64) and the kernels only apply it:
//   forward   y'_i = m_i y'_{i-1} + s_i d_i        (m_0 = 0)
//   backward  y_i  = y'_i + t_i y_{i+1}            (t_{n-1} = 0)
//   cyclic    x_i  = y_i - w_i (y_0 + g y_{n-1})   (Sherman-Morrison)
// A line's rows are split over P lanes of one wave, K rows each; the two
// affine recurrences are composed per lane, chained across the lanes with
// wave shuffles and re-swept, as in the spectral line solve.  Tables are
// zero-padded to P*K rows, so padding rows stay zero and decouple, and stored
// chunk-row major (entry i * P + p holds row p * K + i), so that the lanes of
// one line read a table row as one contiguous 8P-byte segment.  The products
// of the multipliers that the lane scans compose do not depend on the data,
// so the host tabulates them per scan step and only the data term crosses
// lanes.
#include "ibp_internal.hpp"

namespace ibp {

namespace {

template <int P>
constexpr int scan_steps() { return P == 64 ? 6 : 5; }

// Doubles of one direction's tables for P lanes of K rows.
template <int P, int K>
constexpr int line_table_size() { return 4 * P * K + 2 * scan_steps<P>() * P; }

// `tab`: the direction's tables (global or an LDS copy): m, s, t, w (P K
// each), then the forward and backward scan multipliers (scan_steps * P each).
template <int P, int K, typename Slot>
__device__ __forceinline__ void apply_line_lu(const LineArgs& A, const double* tab, double* tile, Slot slot, int m,
                                              int p) {
  constexpr int NP = P * K, S = scan_steps<P>();
  const double* tm = tab;
  const double* ts = tab + NP;
  const double* tt = tab + 2 * NP;
  const double* tw = tab + 3 * NP;
  const double* mf = tab + 4 * NP;
  const double* mb = mf + S * P;
  double d[K];
#pragma unroll
  for (int i = 0; i < K; ++i) d[i] = tile[slot(m, p, i)];
  // ---- forward: y'_out = mu y'_in + nu over the lane's rows (mu tabulated)
  {
    double nu = 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i) nu = tm[i * P + p] * nu + ts[i * P + p] * d[i];
#pragma unroll
    for (int st = 0, off = 1; off < P; ++st, off <<= 1) {   // inclusive prefix: mine after the earlier ones
      const double pn = __shfl_up(nu, off, P);
      if (p >= off) nu = mf[st * P + p] * pn + nu;
    }
    double prev = __shfl_up(nu, 1, P);
    if (p == 0) prev = 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      d[i] = tm[i * P + p] * prev + ts[i * P + p] * d[i];
      prev = d[i];
    }
  }
  // ---- backward: y_first = T y_below + V over the lane's rows (T tabulated)
  {
    double V = 0.0;
#pragma unroll
    for (int i = K - 1; i >= 0; --i) V = d[i] + tt[i * P + p] * V;
#pragma unroll
    for (int st = 0, off = 1; off < P; ++st, off <<= 1) {   // inclusive suffix: mine before the later ones
      const double nv = __shfl_down(V, off, P);
      if (p + off < P) V = mb[st * P + p] * nv + V;
    }
    double nxt = __shfl_down(V, 1, P);
    if (p == P - 1) nxt = 0.0;
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
      d[i] = d[i] + tt[i * P + p] * nxt;
      nxt = d[i];
    }
  }
  // ---- periodic lines: Sherman-Morrison correction from the two end values
  if (A.cyclic) {
    const int last = A.n - 1, lp = last / K, li = last - lp * K;
    double mine = 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i)
      if (i == li) mine = d[i];
    const double y0 = __shfl(d[0], 0, P);
    const double yl = __shfl(mine, lp, P);
    const double sc = y0 + A.g * yl;
#pragma unroll
    for (int i = 0; i < K; ++i) d[i] -= tw[i * P + p] * sc;
  }
#pragma unroll
  for (int i = 0; i < K; ++i) tile[slot(m, p, i)] = d[i];
}

// Lines contiguous in memory (x direction): block = M lines, line L at
// f + L n.  LDS tile line-major, one pad slot per lane chunk (odd stride
// K + 1, so the chunk reads fall on distinct banks).  Lines of even length
// move 16-byte pairs; odd lengths go through k_lines_contig1.
template <int M, int P, int K>
__global__ __launch_bounds__(M * P) void k_lines_contig(LineArgs A) {
  constexpr int NT = M * P;
  constexpr int CS = K + 1;
  constexpr int LS = P * CS;
  __shared__ double tile[M * LS];
  constexpr int NPAIR = P * K / 2;   // pairs per padded line
  constexpr int IT = M * NPAIR / NT;  // = K / 2 pairs per thread
  const long L0 = (long)blockIdx.x * M;
  const int n = A.n;                  // even, <= P K
  const long nl = A.ncol;             // number of lines
  const int nm = (int)((nl - L0) < M ? (nl - L0) : M);   // lines in this block
  const double2* src = reinterpret_cast<const double2*>(A.f + L0 * n);
  {
    double2 ld[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {   // all loads issued before the first LDS write
      const int e2 = threadIdx.x + NT * it;
      const int m = e2 / NPAIR, pos = 2 * (e2 - m * NPAIR);
      ld[it] = (m < nm && pos < n) ? src[(long)m * (n / 2) + pos / 2] : double2{0.0, 0.0};
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e2 = threadIdx.x + NT * it;
      const int m = e2 / NPAIR, pos = 2 * (e2 - m * NPAIR);
      const int pp = pos / K, r = pos - pp * K;   // K even: pos, pos + 1 share a chunk
      tile[m * LS + pp * CS + r] = ld[it].x;
      tile[m * LS + pp * CS + r + 1] = ld[it].y;
    }
  }
  __syncthreads();
  {
    const int p = threadIdx.x % P, m = threadIdx.x / P;
    auto slot = [](int mm, int pp, int i) { return mm * LS + pp * CS + i; };
    if (m < nm) apply_line_lu<P, K>(A, A.lu, tile, slot, m, p);
  }
  __syncthreads();
  double2* dst = reinterpret_cast<double2*>(A.f + L0 * n);
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e2 = threadIdx.x + NT * it;
    const int m = e2 / NPAIR, pos = 2 * (e2 - m * NPAIR);
    const int pp = pos / K, r = pos - pp * K;
    if (m < nm && pos < n) dst[(long)m * (n / 2) + pos / 2] = double2{tile[m * LS + pp * CS + r], tile[m * LS + pp * CS + r + 1]};
  }
}

// Odd line length: the same with single 8-byte values (K per thread).
template <int M, int P, int K>
__global__ __launch_bounds__(M * P) void k_lines_contig1(LineArgs A) {
  constexpr int NT = M * P;
  constexpr int CS = K + 1;
  constexpr int LS = P * CS;
  constexpr int NE = P * K;   // values per padded line
  __shared__ double tile[M * LS];
  const long L0 = (long)blockIdx.x * M;
  const int n = A.n;
  const long nl = A.ncol;
  const int nm = (int)((nl - L0) < M ? (nl - L0) : M);
  const double* src = A.f + L0 * n;
  {
    double ld[K];
#pragma unroll
    for (int it = 0; it < K; ++it) {
      const int e = threadIdx.x + NT * it;
      const int m = e / NE, pos = e - m * NE;
      ld[it] = (m < nm && pos < n) ? src[(long)m * n + pos] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < K; ++it) {
      const int e = threadIdx.x + NT * it;
      const int m = e / NE, pos = e - m * NE;
      const int pp = pos / K;
      tile[m * LS + pp * CS + (pos - pp * K)] = ld[it];
    }
  }
  __syncthreads();
  {
    const int p = threadIdx.x % P, m = threadIdx.x / P;
    auto slot = [](int mm, int pp, int i) { return mm * LS + pp * CS + i; };
    if (m < nm) apply_line_lu<P, K>(A, A.lu, tile, slot, m, p);
  }
  __syncthreads();
  double* dst = A.f + L0 * n;
#pragma unroll
  for (int it = 0; it < K; ++it) {
    const int e = threadIdx.x + NT * it;
    const int m = e / NE, pos = e - m * NE;
    const int pp = pos / K;
    if (m < nm && pos < n) dst[(long)m * n + pos] = tile[m * LS + pp * CS + (pos - pp * K)];
  }
}

// Lines strided in memory (z and y directions): line (o, c) holds
// f[o * ostride + c + t * stride], t < n; a block owns M consecutive columns
// c of one outer index o (M * 8 contiguous bytes per row).  LDS tile
// partition-major with one pad slot per partition, as in the spectral line
// solve.
template <int M, int P, int K>
__global__ __launch_bounds__(M * P) void k_lines_strided(LineArgs A) {
  constexpr int PS = K * M + 1;
  constexpr int NT = M * P, NTAB = line_table_size<P, K>();
  constexpr int TIT = (NTAB + NT - 1) / NT;
  __shared__ double tile[P * PS];
  __shared__ double tab[NTAB];   // the tables, staged once per block with the data loads
  const long ncg = (A.ncol + M - 1) / M;
  const long bid = A.rev ? (long)(gridDim.x - 1 - blockIdx.x) : (long)blockIdx.x;
  const long o = bid / ncg;
  const long c0 = (bid - o * ncg) * M;
  double* base = A.f + o * A.ostride + c0;
  const int n = A.n;
  {
    // every load is issued before the first wait: data from clamped (always
    // valid) addresses, values past the line or the last column discarded,
    // then the tables
    const int mm = threadIdx.x % M, row0 = threadIdx.x / M;
    const bool colok = c0 + mm < A.ncol;
    const int mc = colok ? mm : 0;
    double ld[K], tl[TIT];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int row = row0 + P * i;
      ld[i] = base[(long)(row < n ? row : n - 1) * A.stride + mc];
    }
#pragma unroll
    for (int it = 0; it < TIT; ++it) {
      const int e = threadIdx.x + NT * it;
      tl[it] = A.lu[e < NTAB ? e : NTAB - 1];
    }
#pragma unroll
    for (int it = 0; it < TIT; ++it) {   // threads past the end rewrite the last entry with its own value
      const int e = threadIdx.x + NT * it;
      tab[e < NTAB ? e : NTAB - 1] = tl[it];
    }
#pragma unroll
    for (int i = 0; i < K; ++i) ld[i] = (colok && row0 + P * i < n) ? ld[i] : 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int row = row0 + P * i;
      const int pp = row / K;
      tile[pp * PS + (row - pp * K) * M + mm] = ld[i];
    }
  }
  __syncthreads();
  {
    const int p = threadIdx.x % P, m = threadIdx.x / P;
    auto slot = [](int mm, int pp, int i) { return pp * PS + i * M + mm; };
    if (c0 + m < A.ncol) apply_line_lu<P, K>(A, tab, tile, slot, m, p);
  }
  __syncthreads();
  {
    const int mm = threadIdx.x % M, row0 = threadIdx.x / M;
    if (c0 + mm < A.ncol) {
      double st[K];
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int row = row0 + P * i;
        const int pp = row / K;
        st[i] = tile[pp * PS + (row - pp * K) * M + mm];
      }
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int row = row0 + P * i;
        if (row < n) base[(long)row * A.stride + mm] = st[i];
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_fill_zero(double* p, long n) {
  for (long e = (long)blockIdx.x * kThreads + threadIdx.x; e < n; e += (long)gridDim.x * kThreads) p[e] = 0.0;
}

template <int M, int P>
hipError_t contig_k(int K, const LineArgs& a, hipStream_t s) {
  const long nb = (a.ncol + M - 1) / M;
  const bool pairs = a.n % 2 == 0;
  switch (K) {
#define IBP_CASE(k)                                                                                  \
  case k:                                                                                            \
    if (pairs)                                                                                       \
      hipLaunchKernelGGL((k_lines_contig<M, P, k>), dim3((unsigned)nb), dim3(M * P), 0, s, a);      \
    else                                                                                             \
      hipLaunchKernelGGL((k_lines_contig1<M, P, k>), dim3((unsigned)nb), dim3(M * P), 0, s, a);     \
    break;
    IBP_CASE(2) IBP_CASE(4) IBP_CASE(8) IBP_CASE(12) IBP_CASE(16) IBP_CASE(24)
#undef IBP_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int M, int P>
hipError_t strided_k(int K, const LineArgs& a, hipStream_t s) {
  const long nb = a.nouter * ((a.ncol + M - 1) / M);
  switch (K) {
#define IBP_CASE(k) \
  case k: hipLaunchKernelGGL((k_lines_strided<M, P, k>), dim3((unsigned)nb), dim3(M * P), 0, s, a); break;
    IBP_CASE(2) IBP_CASE(4) IBP_CASE(8) IBP_CASE(12) IBP_CASE(16) IBP_CASE(24)
#undef IBP_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

int line_shape(int n, int* P, int* K) {
  static const int ks[] = {2, 4, 8, 12, 16, 24};
  for (int pl : {32, 64}) {
    if (pl == 32 && n > 32 * 16) continue;   // longer lines: 64 lanes
    for (int k : ks)
      if (pl * k >= n) {
        *P = pl;
        *K = k;
        return 1;
      }
  }
  return 0;
}

hipError_t launch_lines_contig(int P, int K, const LineArgs& a, hipStream_t s) {
  if (a.ncol <= 0) return hipSuccess;
  if ((long)P * K < a.n) return hipErrorInvalidValue;
  if (P == 32) return contig_k<8, 32>(K, a, s);
  if (P == 64) return contig_k<4, 64>(K, a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_lines_strided(int P, int K, const LineArgs& a, hipStream_t s) {
  if (a.ncol <= 0 || a.nouter <= 0) return hipSuccess;
  if ((long)P * K < a.n) return hipErrorInvalidValue;
  if (P == 32) return strided_k<16, 32>(K, a, s);
  if (P == 64) return strided_k<8, 64>(K, a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_fill_zero(double* p, long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long nb = (n + kThreads - 1) / kThreads;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)nb), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace ibp

// Wall-normal line solves, one tridiagonal system per horizontal Fourier mode
// (paper: after the FFTs, independent tridiagonal systems remain along x3 for
// each horizontal mode; "Fluid domain" parallelisation subsection), plus the
// singular (0,0) mode in FP64 and the refinement control.
//
// Mode (kx, kz) solves  a_j X_{j-1} + (b_j + lx(kx) + lz(kz)) X_j + c_j X_{j+1} = F_j,
// j = 0..ny-1, real coefficients, complex right-hand side, a_0 = c_{ny-1} = 0
// (homogeneous Neumann walls).
//
// A block owns M consecutive spectral columns, staged through LDS; P lanes of
// one wave own one column, K consecutive rows each (rows past ny are
// decoupled padding).
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "ibp_internal.hpp"
#include "ibp_ytri_body.hpp"

namespace ibp {

// Occupancy floor per precision: the all-FP32 line solve fits 4 waves per
// SIMD (<= 128 VGPRs, a 28-byte spill) and measured 1.6x faster there than at
// the compiler's own 3; with FP64 coefficients or spectra the same cap spills
// hundreds of bytes, and FP64 at 3 waves gained nothing.
template <typename T, typename U = T>
constexpr int ytri_waves() { return sizeof(T) == 4 && sizeof(U) == 4 ? 4 : 1; }

template <typename T, typename U, int M, int P, int K>
__global__ __launch_bounds__(M * P) __attribute__((amdgpu_waves_per_eu(ytri_waves<T, U>())))
void k_ytri(YArgs<T, U> A, ZeroArgs Z) {
  __shared__ Cx<T> tile[ytile_slots<M, P, K>()];
  // kx-major column order for FP64 spectra (measured 1.7% slower on the
  // mixed form's FP32 spectra, which keep the plain order)
  ytri_body<T, U, M, P, K>(A, Z, blockIdx.x, tile, sizeof(T) == 8);
}

template <int M, int P, int K, bool ADD>
__global__ __launch_bounds__(M * P) void k_ytri_out64(YArgs<float, double> A, ZeroArgs Z) {
  __shared__ Cx<double> tile[ytile_slots<M, P, K>()];
  // kx-major column order: the FP64 inverse z pass then starts on the
  // groups written last (measured: z pass -8%, this pass +5%)
  ytri_body<float, double, M, P, K, true, ADD>(A, Z, blockIdx.x, reinterpret_cast<Cx<float>*>(tile), true);
}

__global__ __launch_bounds__(kThreads) void k_check(ZeroArgs Z) {
  __shared__ double sh[(kThreads / kWave) * kPartStride];
  check_body<kThreads>(Z, sh);
}

__global__ __launch_bounds__(kThreads) void k_zero_mode(ZeroArgs Z) {
  zero_mode_part<kThreads>(Z, blockIdx.x, gridDim.x);
}

// First level of the initial pass's partial reduction (block b sums
// partials [b S, (b + 1) S) into Z.part2[b]); no solve state is read.
__global__ __launch_bounds__(kThreads) void k_part_split(ZeroArgs Z, long S) {
  __shared__ double sh[(kThreads / kWave) * kPartStride];
  const long b0 = (long)blockIdx.x * S;
  const long n = Z.nparts - b0 < S ? Z.nparts - b0 : S;
  ZeroArgs z = Z;
  z.part = Z.part + b0 * kPartStride;
  z.nparts = n > 0 ? n : 0;
  double v[kPartStride];
  reduce_parts<kThreads>(z, sh, v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kPartStride; ++q) Z.part2[blockIdx.x * kPartStride + q] = v[q];
  }
}

hipError_t launch_zero_mode(const ZeroArgs& z, hipStream_t s) {
  ZeroArgs z2 = z;
  if (z.init && z.nparts > kCheckSplitMin && z.part2 != nullptr) {   // the initial norms in two levels
    const long G = std::min<long>(kCheckSplitMax, (z.nparts + kCheckSplitMin / 2 - 1) / (kCheckSplitMin / 2));
    const long S = (z.nparts + G - 1) / G;
    hipLaunchKernelGGL(k_part_split, dim3((unsigned)G), dim3(kThreads), 0, s, z, S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    z2.part = z.part2;
    z2.nparts = G;
  }
  // one wave per plane sum
  const int nb = std::max(1, std::min(z.ny / (kThreads / kWave), 128));
  hipLaunchKernelGGL(k_zero_mode, dim3((unsigned)nb), dim3(kThreads), 0, s, z2);
  return hipGetLastError();
}

// First level of the split check: block b sums partials [b S, (b + 1) S)
// into Z.part2[b] (the same skips as the check itself).
__global__ __launch_bounds__(kThreads) void k_check_split(ZeroArgs Z, long S) {
  __shared__ double sh[(kThreads / kWave) * kPartStride];
  if (__builtin_amdgcn_readfirstlane(Z.ctl->done)) return;
  if (Z.probe && !__builtin_amdgcn_readfirstlane(Z.ctl->probe)) return;
  const long b0 = (long)blockIdx.x * S;
  const long n = Z.nparts - b0 < S ? Z.nparts - b0 : S;
  ZeroArgs z = Z;
  z.part = Z.part + b0 * kPartStride;
  z.nparts = n > 0 ? n : 0;
  double v[kPartStride];
  reduce_parts<kThreads>(z, sh, v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kPartStride; ++q) Z.part2[blockIdx.x * kPartStride + q] = v[q];
  }
}

hipError_t launch_check(const ZeroArgs& z, hipStream_t s) {
  if (z.nparts <= kCheckSplitMin || z.part2 == nullptr) {
    hipLaunchKernelGGL(k_check, dim3(1), dim3(kThreads), 0, s, z);
    return hipGetLastError();
  }
  const long G = std::min<long>(kCheckSplitMax, (z.nparts + kCheckSplitMin / 2 - 1) / (kCheckSplitMin / 2));
  const long S = (z.nparts + G - 1) / G;
  hipLaunchKernelGGL(k_check_split, dim3((unsigned)G), dim3(kThreads), 0, s, z, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  ZeroArgs z2 = z;
  z2.part = z.part2;
  z2.nparts = G;
  hipLaunchKernelGGL(k_check, dim3(1), dim3(kThreads), 0, s, z2);
  return hipGetLastError();
}

// ---------------------------------------------------------------- dispatch
// Shapes (ytri_shape): P = 32 lanes per column (P = 64 when ny > 384), K
// rows per lane from {2, 4, 8, 12, 16, 24}; M columns per block so that a
// row segment is 128 bytes, reduced while the staged tile would exceed the
// LDS budget.
// (lanes, rows per lane) pairs ytri_shape returns: 32 lanes up to 12 rows,
// 64 lanes from 8 rows (ny above 384 needs more than 6 rows of 64)
constexpr bool ytri_pair_used(int P, int K) { return P == 32 ? K <= 12 : K >= 8; }


static int ycol_override() {
  const char* e = getenv("IBP_YCOLS");   // tuning knob: columns per line-solve block
  return e ? atoi(e) : 0;
}

template <typename T>
static int ytri_cols(int P, int K, int want) {
  auto tile = [&](int M) { return ytile_slots_host(M, P, K) * (long)sizeof(Cx<T>); };
  int M = 128 / (int)sizeof(Cx<T>);
  const int o = want ? want : ycol_override();
  if (o == 2 || o == 4 || o == 8 || o == 16) M = o;
  while (M > 2 && tile(M) > kYTileBytes) M /= 2;
  while (M * P > 512) M /= 2;   // 1024-thread blocks cap the solve at 128 VGPRs and spill
  return M;
}

template <typename T, typename U, int M, int P, int K>
static hipError_t launch_ytri_mpk(const YArgs<T, U>& a, const ZeroArgs& z, hipStream_t s) {
  // only shapes ytri_shape and ytri_cols can select are instantiated
  if constexpr (ytile_slots<M, P, K>() * (long)sizeof(Cx<T>) <= kYTileBytes && M * P <= 512 &&
                ytri_pair_used(P, K)) {
    const long nb = (a.Q + M - 1) / M + zero_blocks(a.ny);   // + the (0,0)-mode blocks
    hipLaunchKernelGGL((k_ytri<T, U, M, P, K>), dim3((unsigned)nb), dim3(M * P), 0, s, a, z);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename T, typename U, int M, int P>
static hipError_t launch_ytri_mp(int K, const YArgs<T, U>& a, const ZeroArgs& z, hipStream_t s) {
  switch (K) {
    case 2: return launch_ytri_mpk<T, U, M, P, 2>(a, z, s);
    case 4: return launch_ytri_mpk<T, U, M, P, 4>(a, z, s);
    case 8: return launch_ytri_mpk<T, U, M, P, 8>(a, z, s);
    case 12: return launch_ytri_mpk<T, U, M, P, 12>(a, z, s);
    case 16: return launch_ytri_mpk<T, U, M, P, 16>(a, z, s);
    case 24: return launch_ytri_mpk<T, U, M, P, 24>(a, z, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, typename U>
hipError_t launch_ytri(int P, int K, int want, const YArgs<T, U>& a, const ZeroArgs& z, hipStream_t s) {
  const int M = ytri_cols<T>(P, K, want);
  if (P == 32) {
    switch (M) {
      case 16: return launch_ytri_mp<T, U, 16, 32>(K, a, z, s);
      case 8: return launch_ytri_mp<T, U, 8, 32>(K, a, z, s);
      case 4: return launch_ytri_mp<T, U, 4, 32>(K, a, z, s);
      case 2: return launch_ytri_mp<T, U, 2, 32>(K, a, z, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (P == 64) {
    switch (M) {
      case 16: return launch_ytri_mp<T, U, 16, 64>(K, a, z, s);
      case 8: return launch_ytri_mp<T, U, 8, 64>(K, a, z, s);
      case 4: return launch_ytri_mp<T, U, 4, 64>(K, a, z, s);
      case 2: return launch_ytri_mp<T, U, 2, 64>(K, a, z, s);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorInvalidValue;
}

// FP32 in, FP64 out: the FP64 line solve's columns per block (128-byte
// output segments, the same LDS tile)
template <int M, int P>
static hipError_t launch_out64_mp(int K, const YArgs<float, double>& a, const ZeroArgs& z, hipStream_t s) {
  auto go = [&](auto kk) {
    constexpr int KK = decltype(kk)::value;
    // only tiles within the LDS budget are instantiated
    if constexpr (ytile_slots<M, P, KK>() * (long)sizeof(Cx<double>) <= kYTileBytes) {
      const long nb = (a.Q + M - 1) / M + zero_blocks(a.ny);
      if (a.add_iter)
        hipLaunchKernelGGL((k_ytri_out64<M, P, KK, true>), dim3((unsigned)nb), dim3(M * P), 0, s, a, z);
      else
        hipLaunchKernelGGL((k_ytri_out64<M, P, KK, false>), dim3((unsigned)nb), dim3(M * P), 0, s, a, z);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  };
  if constexpr (P == 32) {
    switch (K) {
      case 2: return go(std::integral_constant<int, 2>{});
      case 4: return go(std::integral_constant<int, 4>{});
      case 8: return go(std::integral_constant<int, 8>{});
      case 12: return go(std::integral_constant<int, 12>{});
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (K) {
      case 8: return go(std::integral_constant<int, 8>{});
      case 12: return go(std::integral_constant<int, 12>{});
      case 16: return go(std::integral_constant<int, 16>{});
      case 24: return go(std::integral_constant<int, 24>{});
      default: return hipErrorInvalidValue;
    }
  }
}

hipError_t launch_ytri_out64(int P, int K, const YArgs<float, double>& a, const ZeroArgs& z, hipStream_t s) {
  int M = 8;
  while (M > 2 && ytile_slots_host(M, P, K) * (long)sizeof(Cx<double>) > kYTileBytes) M /= 2;
  if (P == 32 && M == 8) return launch_out64_mp<8, 32>(K, a, z, s);
  if (P == 64 && M == 8) return launch_out64_mp<8, 64>(K, a, z, s);
  if (P == 64 && M == 4) return launch_out64_mp<4, 64>(K, a, z, s);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- batched
__device__ __forceinline__ int ybatch_grid_of(const long* start, int count, long b) {
  int lo = 0, hi = count - 1;   // largest g with start[g] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (__builtin_amdgcn_readfirstlane((int)(start[mid] <= b))) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T, int M, int P, int K>
__global__ __launch_bounds__(M * P) __attribute__((amdgpu_waves_per_eu(ytri_waves<T>())))
void kb_ytri(const BatchGrid<T>* __restrict__ D, const long* __restrict__ start,
                                                 BatchLaunch L) {
  __shared__ Cx<T> tile[ytile_slots<M, P, K>()];
  const int g = ybatch_grid_of(start, L.count, blockIdx.x);
  YArgs<T, T> a = D[g].y;
  a.check_done = L.check_done;
  ZeroArgs z = D[g].zero;
  z.init = L.init;
  z.mixed = L.mixed;
  z.iter = L.iter;
  z.final_pass = L.final_pass;
  ytri_body<T, T, M, P, K>(a, z, (long)blockIdx.x - start[g], tile);
}

// Rows per lane for one grid of a batch whose line-solve shape is P lanes x
// K rows: K/4 or K/2 when that still holds ny, so short columns of a batch
// with one tall grid skip the padding rows.  The grids of each value run in
// a launch of their own (a kernel's registers are those of its largest K).
int batch_grid_rows_per_lane(int ny, int P, int K) {
  const int need = (ny + P - 1) / P;
  if (K % 4 == 0 && need <= K / 4) return K / 4;
  if (K % 2 == 0 && need <= K / 2) return K / 2;
  return K;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void kb_check(const BatchGrid<T>* __restrict__ D, BatchLaunch L) {
  __shared__ double sh[(kThreads / kWave) * kPartStride];
  ZeroArgs z = D[blockIdx.x].zero;
  z.init = L.init;
  z.mixed = L.mixed;
  z.iter = L.iter;
  z.final_pass = L.final_pass;
  check_body<kThreads>(z, sh);
}

template <typename T>
int batch_ytri_cols(int P, int K, int want) {
  auto tile = [&](int M) { return ytile_slots_host(M, P, K) * (long)sizeof(Cx<T>); };
  int M = (want == 2 || want == 4 || want == 8 || want == 16) ? want : 128 / (int)sizeof(Cx<T>);
  while (M > 2 && tile(M) > kYTileBytes) M /= 2;
  while (M * P > 512) M /= 2;   // 1024-thread blocks cap the solve at 128 VGPRs and spill
  return M;
}

// (lanes, rows per lane) pairs a batch can launch: ytri_shape's pairs and
// their halves and quarters
constexpr bool ytri_batch_pair(int P, int K) {
  return P == 32 ? (K == 1 || K == 2 || K == 3 || K == 4 || K == 6 || K == 8 || K == 12)
                 : (K == 2 || K == 3 || K == 4 || K == 6 || K == 8 || K == 12 || K == 16 || K == 24);
}

template <typename T, int M, int P, int K>
static hipError_t launch_kb_ytri(const BatchGrid<T>* d, const long* start, long nb, const BatchLaunch& l,
                                 hipStream_t s) {
  if constexpr (ytile_slots<M, P, K>() * (long)sizeof(Cx<T>) <= kYTileBytes && M * P <= 512 &&
                ytri_batch_pair(P, K)) {
    hipLaunchKernelGGL((kb_ytri<T, M, P, K>), dim3((unsigned)nb), dim3(M * P), 0, s, d, start, l);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename T, int M, int P>
static hipError_t launch_kb_ytri_k(int K, const BatchGrid<T>* d, const long* start, long nb, const BatchLaunch& l,
                                   hipStream_t s) {
  switch (K) {
    case 1: return launch_kb_ytri<T, M, P, 1>(d, start, nb, l, s);
    case 2: return launch_kb_ytri<T, M, P, 2>(d, start, nb, l, s);
    case 3: return launch_kb_ytri<T, M, P, 3>(d, start, nb, l, s);
    case 4: return launch_kb_ytri<T, M, P, 4>(d, start, nb, l, s);
    case 6: return launch_kb_ytri<T, M, P, 6>(d, start, nb, l, s);
    case 8: return launch_kb_ytri<T, M, P, 8>(d, start, nb, l, s);
    case 12: return launch_kb_ytri<T, M, P, 12>(d, start, nb, l, s);
    case 16: return launch_kb_ytri<T, M, P, 16>(d, start, nb, l, s);
    case 24: return launch_kb_ytri<T, M, P, 24>(d, start, nb, l, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_batch_ytri(int P, int K, int M, const BatchGrid<T>* d, const long* start, long nblocks,
                             const BatchLaunch& l, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (P == 32) {
    switch (M) {
      case 16: return launch_kb_ytri_k<T, 16, 32>(K, d, start, nblocks, l, s);
      case 8: return launch_kb_ytri_k<T, 8, 32>(K, d, start, nblocks, l, s);
      case 4: return launch_kb_ytri_k<T, 4, 32>(K, d, start, nblocks, l, s);
      case 2: return launch_kb_ytri_k<T, 2, 32>(K, d, start, nblocks, l, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (P == 64) {
    switch (M) {
      case 16: return launch_kb_ytri_k<T, 16, 64>(K, d, start, nblocks, l, s);
      case 8: return launch_kb_ytri_k<T, 8, 64>(K, d, start, nblocks, l, s);
      case 4: return launch_kb_ytri_k<T, 4, 64>(K, d, start, nblocks, l, s);
      case 2: return launch_kb_ytri_k<T, 2, 64>(K, d, start, nblocks, l, s);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_batch_check(const BatchGrid<T>* d, const BatchLaunch& l, hipStream_t s) {
  hipLaunchKernelGGL(kb_check<T>, dim3((unsigned)l.count), dim3(kThreads), 0, s, d, l);
  return hipGetLastError();
}

template int batch_ytri_cols<double>(int, int, int);
template int batch_ytri_cols<float>(int, int, int);
template hipError_t launch_batch_ytri<double>(int, int, int, const BatchGrid<double>*, const long*, long,
                                              const BatchLaunch&, hipStream_t);
template hipError_t launch_batch_ytri<float>(int, int, int, const BatchGrid<float>*, const long*, long,
                                             const BatchLaunch&, hipStream_t);
template hipError_t launch_batch_check<double>(const BatchGrid<double>*, const BatchLaunch&, hipStream_t);
template hipError_t launch_batch_check<float>(const BatchGrid<float>*, const BatchLaunch&, hipStream_t);

template hipError_t launch_ytri<double, double>(int, int, int, const YArgs<double, double>&, const ZeroArgs&,
                                                hipStream_t);
template hipError_t launch_ytri<float, float>(int, int, int, const YArgs<float, float>&, const ZeroArgs&, hipStream_t);
template hipError_t launch_ytri<float, double>(int, int, int, const YArgs<float, double>&, const ZeroArgs&,
                                               hipStream_t);

}  // namespace ibp
